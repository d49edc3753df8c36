"""Oracle discrete adjoint of the FS step, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

One FS step (Sec. 2.2, Eq. (10)-(15)) maps real fields u^n to u^(n+1):

    c^(n+1)     = S_c c^n     - dt M Q_c g_c(u^n)
    eta_i^(n+1) = S_eta eta_i^n - dt L S_eta g_i(u^n)

with the k-space multipliers D_c = 1/(1 + dt M kappa_c |xi|^4),
D_eta = 1/(1 + dt L kappa_eta |xi|^2), and the real symmetric operators
S_c = F^-1 D_c F, Q_c = F^-1 D_c |xi|^2 F, S_eta = F^-1 D_eta F (D is real
and even in k, and the adjoint of F is P F^-1).  g = grad f is pointwise.

Given lambda = dJ/du^(n+1), the adjoint step is

    a_c = S_c lambda_c,  b_c = Q_c lambda_c,  a_i = S_eta lambda_i
    v   = (dt M b_c, dt L a_1, ..., dt L a_p)
    lambda^n = (a_c, a_1, ..., a_p) - H_f(u^n) v

and the step adds to the parameter gradients (using
dt M kappa_c |xi|^4 D_c = 1 - D_c and dt L kappa_eta |xi|^2 D_eta = 1 - D_eta):

    dJ/dM       += -dt <b_c, g_c> - (1/M) <lambda_c - a_c, c^(n+1)>
    dJ/dkappa_c += -(1/kappa_c) <lambda_c - a_c, c^(n+1)>
    dJ/dL       += -dt sum_i <a_i, g_i> - (1/L) sum_i <lambda_i - a_i, eta_i^(n+1)>
    dJ/dkappa_eta += -(1/kappa_eta) sum_i <lambda_i - a_i, eta_i^(n+1)>

<.,.> is the plain sum over grid points.  The tests pin this module to
central finite differences of `fs.fs_run` (dot-product test and gradient
check), so a wrong sign or a dropped term fails there.
"""

import numpy as np

from . import fft as _fft
from . import freeenergy as _fe
from .fs import fs_run, geometry, k2_of


def trajectory(u0, cfg, dt, nsteps):
    """States u^0..u^n of an FS run (list of (F, ...) arrays)."""
    _, snaps = fs_run(u0, cfg, dt, nsteps, record_every=1)
    return snaps


def loss_terminal(c_T, c_target):
    """J = mean((c_T - c_target)^2)."""
    return float(np.mean((c_T - c_target) ** 2))


def loss_seed(uT, c_target):
    """dJ/du^T for J = mean((c_T - c_target)^2): only the c field is seeded."""
    lam = np.zeros_like(uT)
    lam[0] = 2.0 * (uT[0] - c_target) / uT[0].size
    return lam


def fs_adjoint(traj, lam_T, cfg, dt):
    """Backpropagate lam_T = dJ/du^n through the steps of `traj`.

    Returns (dJ/du^0, array [dJ/dM, dJ/dkappa_c, dJ/dL, dJ/dkappa_eta]).
    """
    _, _, axes = geometry(cfg)
    fe = cfg["fe"]
    M, kc, L, ke = cfg["M"], cfg["kappa_c"], cfg["L"], cfg["kappa_eta"]
    k2 = k2_of(cfg)
    Dc = 1.0 / (1.0 + dt * M * kc * k2 * k2)
    De = 1.0 / (1.0 + dt * L * ke * k2)
    sp = tuple(a - 1 for a in axes)
    lam = np.array(lam_T, dtype=np.float64)
    dpar = np.zeros(4)
    for n in range(len(traj) - 2, -1, -1):
        u = traj[n]
        unext = traj[n + 1]
        lhat = _fft.fftn(lam, axes)
        a = np.empty_like(lam)
        a[0] = _fft.ifftn(Dc * lhat[0], sp).real
        b_c = _fft.ifftn(Dc * k2 * lhat[0], sp).real
        for i in range(1, lam.shape[0]):
            a[i] = _fft.ifftn(De * lhat[i], sp).real
        g = _fe.gradient(u, fe)
        v = np.empty_like(lam)
        v[0] = dt * M * b_c
        v[1:] = dt * L * a[1:]
        new = a - _fe.hessian_vector(u, fe, v)
        rc = float(np.sum((lam[0] - a[0]) * unext[0]))
        re = float(np.sum((lam[1:] - a[1:]) * unext[1:]))
        dpar[0] += -dt * float(np.sum(b_c * g[0])) - rc / M
        dpar[1] += -rc / kc
        dpar[2] += -dt * float(np.sum(a[1:] * g[1:])) - re / L
        dpar[3] += -re / ke
        lam = new
    return lam, dpar
