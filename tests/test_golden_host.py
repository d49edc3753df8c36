"""Host checks of the stored full-size oracle values (no GPU).

The values are written by `tests/golden/make_fullsize_golden.py`, which runs
only the oracle.  Here: the file was written by the current oracle and input
module (source digest), it has the expected layout, and it satisfies a
property of the method that holds at any size: neither the FS step (Eq. (14)
at xi = 0) nor the FD step (the divergence form of Eq. (2)) changes the sum
of c over the grid, so it equals that of the initial state."""

import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_fullsize_golden as G  # noqa: E402


@pytest.mark.parametrize("name", ["w2", "paper", "w3", "w2_4k", "fd3"])
def test_stored_values_current_and_consistent(name):
    z = np.load(G.path_of(name))
    assert str(z["digest"]) == G.source_digest(), "rerun make_fullsize_golden.py"
    cfg, dt, steps, u0 = G.trajectory(name)
    assert float(z["dt"]) == dt and int(z["steps"]) == steps
    F = 1 + cfg["p"]
    nlines = (len(G.ROWS_2D) if cfg["n"][0] == 1024 else len(G.ROWS_4K)) if cfg["ndim"] == 2 \
        else len(G.LINES_3D)
    assert z["sample"].shape == (F, nlines, cfg["n"][0])
    assert np.all(np.isfinite(z["sample"]))
    s0 = u0[0].sum()
    assert abs(z["field_sum"][0] - s0) <= 1e-12 * abs(s0)
    # the root-mean-square of the sampled lines is of the order of the
    # whole field's (a sample taken from the stored trajectory, not zeros)
    P = u0[0].size
    rms = np.sqrt(z["field_sumsq"][0] / P)
    assert 0.5 * rms <= np.sqrt(np.mean(z["sample"][0] ** 2)) <= 2.0 * rms


def test_sample_lines_cover_both_axis_ends():
    assert 0 in G.ROWS_2D and 1023 in G.ROWS_2D
    zs = [z for z, _ in G.LINES_3D]
    ys = [y for _, y in G.LINES_3D]
    assert min(zs) == 0 and max(zs) == 255 and min(ys) == 0 and max(ys) == 255


def test_stored_adjoint_values_current():
    z = np.load(G.path_of("w5"))
    assert str(z["digest"]) == G.source_digest(), "rerun make_fullsize_golden.py w5"
    cfg, dt, steps, u0 = G.trajectory("w5")
    assert float(z["dt"]) == dt and int(z["steps"]) == steps
    assert cfg["n"] == (128, 128, 128) and cfg["p"] == 4
    assert z["sample"].shape == (5, len(G.LINES_W5), 128)
    assert np.all(np.isfinite(z["sample"])) and np.all(np.isfinite(z["dpar"]))
    assert z["dpar"].shape == (4,) and np.all(z["dpar"] != 0)
    zs = [zz for zz, _ in G.LINES_W5]
    ys = [y for _, y in G.LINES_W5]
    assert min(zs) == 0 and max(zs) == 127 and min(ys) == 0 and max(ys) == 127
