"""Host-side checks of bench.py that need no GPU."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""


def test_algorithmic_bytes_of_the_two_passes():
    """Per-stage bytes of the unfused method (each stage reads and writes its
    F fields once; the update reads two sets): derivative 2Fs, forward FFT
    2Fs, update 3Fs, inverse FFT 2Fs per point.  The row pass performs the
    derivative and the x halves of both FFTs (4Fs), the column pass the
    update and the y halves (5Fs); together the whole step's 9Fs."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2306_04322_amd import inputs as I
    cfg, _ = I.workload_config("W2")
    P = 1024 * 1024
    assert bench.algorithmic_bytes(cfg, "f32", "row") == 4 * 5 * 4 * P
    assert bench.algorithmic_bytes(cfg, "f32", "col") == 5 * 5 * 4 * P
    assert bench.algorithmic_bytes(cfg, "f64", "step") == 9 * 5 * 8 * P
    assert (bench.algorithmic_bytes(cfg, "f32", "row") + bench.algorithmic_bytes(cfg, "f32", "col")
            == bench.algorithmic_bytes(cfg, "f32", "step"))


def test_compulsory_bytes_of_the_two_passes():
    """Row pass: 2F half-spectra (F read, F written); column pass: 2F + 2
    (the carried c spectrum is read and written as well).  A half-spectrum
    of the 1024^2 FP32 grid is 1024 rows of 513 complex values of 8 bytes."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2306_04322_amd import inputs as I
    cfg, _ = I.workload_config("W2")
    half = 1024 * 513 * 8
    assert bench.compulsory_bytes(cfg, "f32", "row") == 10 * half
    assert bench.compulsory_bytes(cfg, "f32", "col") == 12 * half


def test_rel_l2_floor():
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    ref = np.stack([np.ones((4, 4)), np.zeros((4, 4))])
    got = ref.copy()
    got[0, 0, 0] += 0.4
    e = bench.rel_l2(got, ref)
    assert abs(e[0] - 0.1) < 1e-15 and e[1] is None
    assert bench.max_err(e) == e[0]


def test_committed_traffic_summary_matches_the_current_kernels():
    """The committed counter summary carries the digest of the kernel
    sources it was taken with; bench.py reports its bytes only while they
    match, and they must then lie near the algorithmic bytes."""
    sys.path.insert(0, ROOT)
    import bench
    path = os.path.join(ROOT, "profiles", "fs2d_1024_f32_row_col_traffic.json")
    rec = json.load(open(path))
    from paper_2306_04322_amd.build import fs_kernel_digest
    if rec["kernel_digest"] != fs_kernel_digest():
        pytest.skip("the row / column kernels changed since the counters were taken")
    for kind, alg in (("row", 10), ("col", 12)):
        got = bench.traffic_from_profile(kind)
        assert got == rec[kind]["bytes_per_launch"]
        assert 0.9 * alg * 1024 * 513 * 8 <= got <= 1.3 * alg * 1024 * 513 * 8
