"""The expected values of the uniform-state GPU test (test_gpu_degenerate.py)
agree with the oracle's FS and FD runs on a small uniform grid: both schemes
reduce to the pointwise recurrence there (Eq. (14), (15); Sec. 2.2), and both
gradient parts of the energy (Eq. (1)) vanish."""

import numpy as np

import test_gpu_degenerate as T
from oracle import energy as OE
from oracle import fd as OFD
from oracle import freeenergy as OFE
from oracle import fs as OFS
from paper_2306_04322_amd import inputs as I
from parity_util import DISTINCT


def test_recurrence_matches_oracle_fs_and_fd():
    cfg = I.make_config(2, (16, 8), 1.0, 4, I.PAPER_FE, **DISTINCT)
    u0 = np.array(T.U0)
    exp = T._expected(u0, cfg).reshape(5, 1, 1)
    u = np.broadcast_to(u0.reshape(5, 1, 1), (5, 8, 16)).copy()
    assert np.max(np.abs(OFS.fs_run(u, cfg, T.DT, T.STEPS) - exp)) <= 1e-15
    assert np.max(np.abs(OFD.fd_run(u, cfg, T.DT, T.STEPS) - exp)) <= 1e-15
    # the order parameters move: the check is not of a fixed point
    assert np.all(np.abs(exp[1:, 0, 0] - u0[1:]) > 1e-2 * np.abs(u0[1:]))
    chem = 128 * float(OFE.density(u0.reshape(-1, 1), cfg["fe"])[0])
    for sch in ("fs", "fd"):
        e = OE.energy(u, cfg, sch)
        assert e[2] == 0.0 and e[3] == 0.0
        assert abs(e[1] - chem) <= 1e-12 * chem
        assert abs(e[4] - 128 * u0[0]) <= 1e-12 * 128 * u0[0]
