"""Pins for the oracle's discrete adjoint of the FS step (no GPU).

The adjoint is checked against central finite differences of the oracle's
own forward rollout: a dot-product test in the initial fields, a gradient
check in each of (M, kappa_c, L, kappa_eta), and the exact zero of the
gradient when the target is produced by the same parameters."""

import numpy as np
import pytest

from oracle import adjoint, fs
from paper_2306_04322_amd import inputs as I


def _cfg(kind, kmode="spectral", ndim=2, n=(16, 8)):
    fe = I.PAPER_FE if kind == "paper" else I.POLY_FE
    return I.make_config(ndim, n, 1.0, 2, fe, kmode, M=4.0, kappa_c=2.0, L=3.0, kappa_eta=1.5)


def _with(cfg, **kw):
    c = dict(cfg)
    c.update(kw)
    return c


@pytest.mark.parametrize("kind,kmode,ndim,n", [("paper", "spectral", 2, (16, 8)),
                                               ("poly", "spectral", 2, (8, 8)),
                                               ("paper", "fd2", 2, (8, 16)),
                                               ("paper", "spectral", 3, (4, 8, 4))])
def test_dot_product_in_initial_fields(kind, kmode, ndim, n):
    cfg = _cfg(kind, kmode, ndim, n)
    dt, steps = 0.02, 4
    u0 = I.random_ic(cfg, 21)
    v = I.random_direction(cfg, 22, 1.0)
    w = I.random_direction(cfg, 23, 1.0)
    traj = adjoint.trajectory(u0, cfg, dt, steps)
    lam0, _ = adjoint.fs_adjoint(traj, w, cfg, dt)
    h = 1e-5
    up = fs.fs_run(u0 + h * v, cfg, dt, steps)
    um = fs.fs_run(u0 - h * v, cfg, dt, steps)
    jv = np.sum(w * (up - um)) / (2 * h)
    assert abs(np.sum(lam0 * v) - jv) <= 1e-7 * max(1.0, abs(jv))


@pytest.mark.parametrize("kind", ["paper", "poly"])
def test_parameter_gradients_match_central_differences(kind):
    cfg = _cfg(kind)
    dt, steps = 0.02, 5
    u0 = I.random_ic(cfg, 31)
    target = fs.fs_run(u0, _with(cfg, M=3.0, kappa_c=2.5), dt, steps)[0]
    traj = adjoint.trajectory(u0, cfg, dt, steps)
    lam_T = adjoint.loss_seed(traj[-1], target)
    _, dpar = adjoint.fs_adjoint(traj, lam_T, cfg, dt)
    h = 1e-6
    for i, name in enumerate(["M", "kappa_c", "L", "kappa_eta"]):
        jp = adjoint.loss_terminal(fs.fs_run(u0, _with(cfg, **{name: cfg[name] + h}), dt, steps)[0], target)
        jm = adjoint.loss_terminal(fs.fs_run(u0, _with(cfg, **{name: cfg[name] - h}), dt, steps)[0], target)
        num = (jp - jm) / (2 * h)
        assert abs(dpar[i] - num) <= 1e-6 * max(abs(num), 1e-8), (name, dpar[i], num)


def test_loss_gradient_in_initial_fields():
    cfg = _cfg("paper")
    dt, steps = 0.05, 3
    u0 = I.random_ic(cfg, 41)
    target = fs.fs_run(I.random_ic(cfg, 42), cfg, dt, steps)[0]
    traj = adjoint.trajectory(u0, cfg, dt, steps)
    lam0, _ = adjoint.fs_adjoint(traj, adjoint.loss_seed(traj[-1], target), cfg, dt)
    v = I.random_direction(cfg, 43)
    h = 1e-6
    jp = adjoint.loss_terminal(fs.fs_run(u0 + h * v, cfg, dt, steps)[0], target)
    jm = adjoint.loss_terminal(fs.fs_run(u0 - h * v, cfg, dt, steps)[0], target)
    num = (jp - jm) / (2 * h)
    assert abs(np.sum(lam0 * v) - num) <= 1e-6 * abs(num)


def test_gradient_vanishes_at_target_parameters():
    # the target is a run with the same seed and parameters: J = 0 and
    # dJ/dtheta = 0 exactly
    cfg = _cfg("paper")
    u0 = I.random_ic(cfg, 51)
    traj = adjoint.trajectory(u0, cfg, 0.05, 4)
    lam_T = adjoint.loss_seed(traj[-1], traj[-1][0].copy())
    lam0, dpar = adjoint.fs_adjoint(traj, lam_T, cfg, 0.05)
    assert np.all(lam0 == 0.0) and np.all(dpar == 0.0)
