"""Oracle explicit finite-difference (FD) comparison step, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2 (the FD solver): first-order forward Euler in time, second-order
centred differences in space, 5-point (2D) / 7-point (3D) Laplacian on a
periodic grid.  One step computes, all from the fields at time t,

    mu       = df/dc - kappa_c lap_h(c)
    c'       = c + dt M lap_h(mu)
    eta_i'   = eta_i - dt L (df/deta_i - kappa_eta lap_h(eta_i))

The paper swaps the current and next arrays only after all three kernels,
so the eta update sees c at time t (pure forward Euler).
"""

import numpy as np

from . import freeenergy as _fe
from .fs import geometry


def laplacian_h(v, dxs, axes):
    """Periodic second-order centred Laplacian of `v` over `axes`.

    `axes` lists the spatial axes of `v`; the last of them is x, whose
    spacing is dxs[0].
    """
    nd = len(axes)
    out = np.zeros_like(v)
    for i, ax in enumerate(axes):
        d = dxs[nd - 1 - i]
        out = out + (np.roll(v, -1, axis=ax) - 2.0 * v + np.roll(v, 1, axis=ax)) / d ** 2
    return out


def fd_step(u, cfg, dt):
    shape, dxs, axes = geometry(cfg)
    fe = cfg["fe"]
    M, kc, L, ke = cfg["M"], cfg["kappa_c"], cfg["L"], cfg["kappa_eta"]
    sp_axes = tuple(range(len(shape)))
    g = _fe.gradient(u, fe)
    c = u[0]
    mu = g[0] - kc * laplacian_h(c, dxs, sp_axes)
    out = np.empty_like(u)
    out[0] = c + dt * M * laplacian_h(mu, dxs, sp_axes)
    for i in range(1, u.shape[0]):
        out[i] = u[i] - dt * L * (g[i] - ke * laplacian_h(u[i], dxs, sp_axes))
    return out


def fd_run(u0, cfg, dt, nsteps):
    u = np.array(u0, dtype=np.float64)
    for step in range(nsteps):
        u = fd_step(u, cfg, dt)
        if not np.all(np.isfinite(u)):
            raise FloatingPointError("FD run diverged at step %d" % (step + 1))
    return u
