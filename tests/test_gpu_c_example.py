"""The C-ABI example program (paper_2306_04322_amd/examples/fs_example.cpp):
a host program with no Python or torch in it drives the library through
include/pfspec.h alone; its result must match the FP64 oracle."""

import os
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import energy as oen
from oracle import fs as ofs
from paper_2306_04322_amd import inputs as I
from parity_util import announce, gpu_or_fail, max_rel, rel_l2

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2306_04322_amd", "examples", "fs_example")


def test_c_example_matches_oracle():
    gpu_or_fail()
    if not os.path.exists(EXE):
        pytest.skip("example not built (python -m paper_2306_04322_amd.build builds it)")
    n, steps, dt = 64, 50, 0.01
    announce("c example", n, steps)
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "fields.bin")
        r = subprocess.run([EXE, str(n), str(steps), repr(dt), out], capture_output=True,
                           text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        data = np.fromfile(out, dtype=np.float64).reshape(2, 5, n, n)
    u0, got = data[0], data[1]
    cfg = I.make_config(2, n, 1.0, 4, I.PAPER_FE)
    ref = ofs.fs_run(u0, cfg, dt, steps)
    assert max_rel(rel_l2(got, ref)) <= 1e-10
    e = [float(v) for v in r.stdout.split()[1::2]]
    eref = oen.energy(ref, cfg, "fs")
    for i in range(5):
        assert abs(e[i] - eref[i]) <= 1e-10 * max(abs(eref[i]), 1e-3 * abs(eref[0])), (e, eref)
