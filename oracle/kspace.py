"""Oracle frequency grids (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.2: on a periodic box of length l_d = N_d * dx_d the discrete
frequency along axis d is xi_d = 2 pi n_d / l_d, with the index vector
n_d = [0, 1, ..., N_d/2, -(N_d/2 - 1), ..., -1]  (Eq. (16) in 2D, Eq. (19)
in 3D).  The squared frequency used by Eq. (14), (15) is
    spectral   |xi|^2     = sum_d xi_d^2                        (Eq. 16/19)
    fd2        |xi_c2|^2  = -2 sum_d (cos(dx_d xi_d) - 1) / dx_d^2   (Eq. 17/20)
    fd4        |xi_c4|^2  = -(1/6) sum_d (16 cos(dx_d xi_d) - cos(2 dx_d xi_d) - 15) / dx_d^2
                                                             (Eq. 18/21)
and |xi|^4 is the square of whichever |xi|^2 is in use (Algorithm 1
writes ||xi||^4 next to ||xi||^2).

Grid points sit at x_j = j dx, j = 0..N-1 (periodic, end point excluded).
"""

import numpy as np


def index_vector(n):
    """n_d of Eq. (16): [0..N/2, -(N/2-1)..-1] (N even)."""
    if n % 2:
        raise ValueError("even axis length required")
    return np.concatenate([np.arange(0, n // 2 + 1), np.arange(-(n // 2 - 1), 0)])


def xi_axis(n, dx):
    """xi_d = 2 pi n_d / (N dx) for one axis."""
    return 2.0 * np.pi * index_vector(n) / (n * dx)


def sq_axis(n, dx, kmode):
    """Contribution of one axis to |xi|^2 (spectral, fd2 or fd4)."""
    xi = xi_axis(n, dx)
    if kmode == "spectral":
        return xi ** 2
    if kmode == "fd2":
        return -2.0 * (np.cos(dx * xi) - 1.0) / dx ** 2
    if kmode == "fd4":
        return -(16.0 * np.cos(dx * xi) - np.cos(2.0 * dx * xi) - 15.0) / (6.0 * dx ** 2)
    raise ValueError("unknown kmode %r" % kmode)


def k2_grid(shape, dx, kmode="spectral"):
    """Full |xi|^2 grid for an array of spatial `shape` (x is the last axis).

    `dx` is given in (dx, dy[, dz]) order, i.e. reversed with respect to
    `shape`.
    """
    nd = len(shape)
    k2 = np.zeros(shape)
    for a in range(nd):
        n = shape[a]
        d = dx[nd - 1 - a]
        t = sq_axis(n, d, kmode)
        sl = [None] * nd
        sl[a] = slice(None)
        k2 = k2 + t[tuple(sl)]
    return k2
