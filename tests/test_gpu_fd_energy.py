"""GPU parity of the FD step (pf_step_fd) and the free-energy reductions
(pf_energy) against the FP64 oracle."""

import numpy as np
import pytest

from oracle import energy as oen
from oracle import fd as ofd
from oracle import fs as ofs
from paper_2306_04322_amd import inputs as I
from parity_util import DISTINCT, announce, fp32_rounded, gpu_or_fail, max_rel, rel_l2

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-10, "f32": 1e-4}


def _solver(cfg, prec, u0):
    gpu_or_fail()
    from paper_2306_04322_amd.pfspec import Solver
    s = Solver(cfg, prec)
    s.set_fields(u0)
    return s


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fd_workload_parity(prec):
    cfg, w = I.workload_config("WO")
    u0 = I.workload_ic(cfg, w)
    if prec == "f32":
        u0 = fp32_rounded(u0)
    announce("fd parity WO", prec)
    s = _solver(cfg, prec, u0)
    s.step_fd(w["dt_fd"], 101)  # odd count exercises the ping-pong copy
    s.step_fd(w["dt_fd"], 99)
    got = s.get_fields()
    ref = ofd.fd_run(u0, cfg, w["dt_fd"], 200)
    errs = rel_l2(got, ref)
    print("FD WO", prec, errs)
    assert max_rel(errs) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("ndim,n,p", [(2, (32, 8), 1), (2, (16, 64), 4), (3, (16, 8, 32), 4),
                                      (3, (8, 8, 8), 8),
                                      (2, (64, 16), 1), (2, (128, 32), 2), (2, (256, 64), 8),
                                      (3, (64, 16, 8), 4), (3, (128, 32, 8), 3),
                                      # two points per thread, XCD bands
                                      (2, (512, 512), 4),
                                      # four (FP32) / two (FP64) points per thread,
                                      # with bands and with planes too large for them
                                      (3, (128, 64, 64), 2), (3, (256, 256, 8), 4),
                                      # planes too large for bands: threads march along z,
                                      # four blocks of 8 planes (p = 4), two blocks with
                                      # p = 2, and one block with p = 8 at one point per
                                      # thread (FP64; in FP32 these planes take XCD bands)
                                      (3, (256, 256, 32), 4), (3, (256, 256, 16), 2),
                                      (3, (128, 128, 8), 8),
                                      # the marching form with the current plane in
                                      # LDS: tiles of 8 (FP32) / 4 (FP64) rows above,
                                      # two-row tiles here in FP32 (FP64: registers)
                                      (3, (1024, 128, 8), 1),
                                      # longest axes
                                      (2, (4096, 8), 1), (2, (8, 4096), 2), (3, (8, 8, 1024), 2)])
def test_fd_shapes_parity(ndim, n, p, prec):
    dx = (1.0, 0.8, 1.2)[:ndim]
    cfg = I.make_config(ndim, n, dx, p, I.PAPER_FE, **DISTINCT)
    u0 = I.random_ic(cfg, seed=9)
    if prec == "f32":
        u0 = fp32_rounded(u0)
    announce("fd shapes", ndim, n, p, prec)
    s = _solver(cfg, prec, u0)
    s.step_fd(2e-4, 20)
    got = s.get_fields()
    ref = ofd.fd_run(u0, cfg, 2e-4, 20)
    assert max_rel(rel_l2(got, ref)) <= (1e-12 if prec == "f64" else 1e-5)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("scheme", ["fs", "fd"])
@pytest.mark.parametrize("case", ["WO", "rand2d", "rand3d", "rand3d_wide", "poly", "rand2d_p8"])
def test_energy_parity(case, scheme, prec):
    if case == "rand2d_p8":
        cfg = I.make_config(2, (64, 32), (1.0, 0.8), 8, I.PAPER_FE, **DISTINCT)
        u0 = I.random_ic(cfg, 7)
    elif case == "WO":
        cfg, w = I.workload_config("WO")
        u0 = I.workload_ic(cfg, w)
    elif case == "rand2d":
        cfg = I.make_config(2, (64, 128), (0.5, 1.5), 2, I.PAPER_FE, "fd4", **DISTINCT)
        u0 = I.random_ic(cfg, 4)
    elif case == "rand3d":
        cfg = I.make_config(3, (16, 32, 8), 1.0, 4, I.PAPER_FE, **DISTINCT)
        u0 = I.random_ic(cfg, 5, c0=0.45)
    elif case == "rand3d_wide":
        # several full column tiles plus the Nyquist column on both strided axes
        cfg = I.make_config(3, (64, 32, 32), (1.0, 0.9, 1.1), 2, I.PAPER_FE, **DISTINCT)
        u0 = I.random_ic(cfg, 8, c0=0.45)
    else:
        cfg = I.make_config(2, 32, 1.0, 3, I.POLY_FE, **DISTINCT)
        u0 = I.random_ic(cfg, 6)
    if prec == "f32":
        u0 = fp32_rounded(u0)
    announce("energy", case, scheme, prec)
    s = _solver(cfg, prec, u0)
    got = s.energy(scheme)
    ref = oen.energy(u0, cfg, scheme)
    tol = 1e-12 if prec == "f64" else 2e-6
    for i in range(5):
        assert abs(got[i] - ref[i]) <= tol * max(abs(ref[i]), 1e-3 * abs(ref[0])), (i, got, ref)


def test_energy_decreases_along_gpu_fs_run():
    cfg, w = I.workload_config("WO")
    u0 = I.workload_ic(cfg, w)
    announce("energy monotone fs f64")
    s = _solver(cfg, "f64", u0)
    E = [s.energy("fs")[0]]
    for _ in range(10):
        s.step_fs(0.01, 20)
        E.append(s.energy("fs")[0])
    assert all(b <= a * (1 + 1e-13) for a, b in zip(E[:-1], E[1:]))


def test_energy_reports_nonfinite():
    gpu_or_fail()
    from paper_2306_04322_amd.pfspec import PF_ERR_NONFINITE, PFError
    cfg = I.make_config(2, 16, 1.0, 2, I.PAPER_FE)
    u0 = I.random_ic(cfg, 1)
    u0[0, 3, 4] = np.nan
    announce("energy nonfinite")
    s = _solver(cfg, "f64", u0)
    with pytest.raises(PFError) as ei:
        s.energy("fd")
    assert ei.value.status == PF_ERR_NONFINITE


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fd_full_size_2d_1024(prec):
    """2D 1024^2, c + 4 eta, in the launch configuration the benchmark times:
    two FD steps compared element by element with the oracle."""
    cfg, w = I.workload_config("W2")
    u0 = I.workload_ic(cfg, w)
    if prec == "f32":
        u0 = fp32_rounded(u0)
    announce("fd full 1024^2", prec)
    s = _solver(cfg, prec, u0)
    s.step_fd(w["dt_fd"], 2)
    got = s.get_fields()
    ref = ofd.fd_run(u0, cfg, w["dt_fd"], 2)
    assert max_rel(rel_l2(got, ref)) <= (1e-13 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("scheme", ["fs", "fd"])
def test_energy_full_size_2d_1024(scheme, prec):
    """The five scalars of pf_energy at the 2D throughput shape (1024^2,
    c + 4 eta) against the oracle, in the launch configuration the benchmark
    times."""
    cfg, w = I.workload_config("W2")
    u0 = I.workload_ic(cfg, w)
    if prec == "f32":
        u0 = fp32_rounded(u0)
    announce("energy full 1024^2", scheme, prec)
    s = _solver(cfg, prec, u0)
    got = s.energy(scheme)
    ref = oen.energy(u0, cfg, scheme)
    tol = 1e-12 if prec == "f64" else 2e-6
    for i in range(5):
        assert abs(got[i] - ref[i]) <= tol * max(abs(ref[i]), 1e-3 * abs(ref[0])), (i, got, ref)
