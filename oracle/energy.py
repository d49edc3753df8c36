"""Oracle total free energy Eq. (1) and mass, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. (1): F = integral of f_chem + kappa_c/2 |grad c|^2 + sum_i kappa_eta/2 |grad eta_i|^2.
Sec. 3.1 monitors the total and its parts: the chemical part, the c-gradient
part and the eta-gradient part.  On the grid the integral is dV times the
sum over points, dV = prod_d dx_d.  The gradient parts are discretised two
ways, matching the two schemes:

  fs: spectral gradient with the scheme's own |xi|^2 (Parseval):
      sum_x |grad v|^2 = (1/P) sum_k |xi_k|^2 |v^_k|^2
  fd: forward-difference squares sum_x sum_d ((v(x+e_d) - v(x)) / dx_d)^2

The mass is dV * sum_x c.  Returned order:
  [E_total, E_chem, E_grad_c, E_grad_eta, mass].
"""

import numpy as np

from . import fft as _fft
from . import freeenergy as _fe
from .fs import geometry, k2_of


def energy(u, cfg, scheme="fs"):
    shape, dxs, axes = geometry(cfg)
    dV = float(np.prod(dxs))
    P = int(np.prod(shape))
    kc, ke = cfg["kappa_c"], cfg["kappa_eta"]
    chem = dV * float(np.sum(_fe.density(u, cfg["fe"])))
    if scheme == "fs":
        k2 = k2_of(cfg)
        uhat = _fft.fftn(u, axes)
        sq = k2 * np.abs(uhat) ** 2
        gc = 0.5 * kc * dV * float(np.sum(sq[0])) / P
        ge = 0.5 * ke * dV * float(np.sum(sq[1:])) / P
    elif scheme == "fd":
        nd = len(shape)
        gc = 0.0
        ge = 0.0
        for a in range(nd):
            d = dxs[nd - 1 - a]
            diff = (np.roll(u, -1, axis=a + 1) - u) / d
            gc += 0.5 * kc * dV * float(np.sum(diff[0] ** 2))
            ge += 0.5 * ke * dV * float(np.sum(diff[1:] ** 2))
    else:
        raise ValueError("scheme must be 'fs' or 'fd'")
    mass = dV * float(np.sum(u[0]))
    return np.array([chem + gc + ge, chem, gc, ge, mass])
