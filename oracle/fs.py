"""Oracle semi-implicit Fourier-spectral (FS) time step, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Sec. 2.2 and Algorithm 1.  Per step, with every explicit term taken
at time t (Eq. (7), (8)):

  1. derivatives df/dc, df/deta_i of the chemical free energy at t;
  2. their forward transforms (Algorithm 1, first two lines of the loop);
  3. right-hand sides, Eq. (12), (13):
        b_c   = c^(t)   - M dt |xi|^2 F[df/dc]
        b_eta = eta^(t) - L dt F[df/deta_i]
  4. diagonal solves, Eq. (14), (15):
        c^   = b_c   / (1 + M dt kappa_c |xi|^4)
        eta^ = b_eta / (1 + L dt kappa_eta |xi|^2)
  5. inverse transforms back to real space.

The spectra c^, eta^ are carried from one step to the next, as Algorithm 1
does (it uses c^(t) from the previous solve and never re-transforms c).
"""

import numpy as np

from . import fft as _fft
from . import freeenergy as _fe
from . import kspace as _ks


def geometry(cfg):
    """(spatial shape with x last, dx tuple in (x, y, z) order, field axes)."""
    nd = cfg["ndim"]
    n = cfg["n"]
    shape = tuple(n[d] for d in reversed(range(nd)))
    dxs = tuple(cfg["dx"][d] for d in range(nd))
    axes = tuple(range(1, nd + 1))
    return shape, dxs, axes


def k2_of(cfg):
    shape, dxs, _ = geometry(cfg)
    return _ks.k2_grid(shape, dxs, cfg.get("kmode", "spectral"))


def _real(z, what):
    """Real part of an inverse transform, checking that the imaginary part is
    negligible (the carried spectra stay Hermitian up to rounding)."""
    scale = max(1.0, float(np.max(np.abs(z.real))))
    if float(np.max(np.abs(z.imag))) > 1e-9 * scale:
        raise FloatingPointError("non-Hermitian %s spectrum" % what)
    return z.real.copy()


def fs_run(u0, cfg, dt, nsteps, record_every=0, workers=1):
    """Advance `u0` (F, ...) by `nsteps` FS steps of size `dt`.

    Returns the final fields, or (final, [snapshots]) when `record_every`
    is positive (snapshot list starts with u0).  `workers` > 1 runs the
    transforms of the F fields on that many threads (bit-identical result;
    for the large grids of the tests).
    """
    shape, dxs, axes = geometry(cfg)
    fe = cfg["fe"]
    M, kc, L, ke = cfg["M"], cfg["kappa_c"], cfg["L"], cfg["kappa_eta"]
    k2 = k2_of(cfg)
    k4 = k2 * k2
    u = np.array(u0, dtype=np.float64)
    uhat = _fft.fftn(u, axes, workers)
    snaps = [u.copy()] if record_every else None
    for step in range(nsteps):
        g = _fe.gradient(u, fe)
        ghat = _fft.fftn(g, axes, workers)
        b_c = uhat[0] - M * dt * k2 * ghat[0]
        b_eta = uhat[1:] - L * dt * ghat[1:]
        uhat = np.empty_like(uhat)
        uhat[0] = b_c / (1.0 + M * dt * kc * k4)
        uhat[1:] = b_eta / (1.0 + L * dt * ke * k2)
        u = _real(_fft.ifftn(uhat, axes, workers), "state")
        if not np.all(np.isfinite(u)):
            raise FloatingPointError("FS run diverged at step %d" % (step + 1))
        if record_every and (step + 1) % record_every == 0:
            snaps.append(u.copy())
    if record_every:
        return u, snaps
    return u
