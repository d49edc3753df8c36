"""Seeded synthetic inputs and parameter presets.

This module is shared by the HIP path's tests/benchmark and by the CPU
oracle's tests.  It holds parameter values and initial-condition recipes
only: none of the method's arithmetic (no free-energy derivatives, none of
the step's transforms, no time stepping).  The one numerical step here is
input preparation for the paper's study: moving fields between grids of the
same box (subsampling, or band-limited interpolation through numpy.fft) and
the Eq. (6) extrusion of 2D fields into a 3D initial state.

A configuration is a plain dict:
    ndim      2 or 3
    n         (Nx, Ny, Nz)  grid points per axis, Nz = 1 in 2D
    dx        (dx, dy, dz)  grid spacing
    p         number of order parameters eta_i (fields F = 1 + p)
    fe        {"kind": "paper" | "poly", **coefficients}
    M, kappa_c, L, kappa_eta
    kmode     "spectral" | "fd2" | "fd4"
Field arrays are float64 of shape (F, Ny, Nx) in 2D and (F, Nz, Ny, Nx) in
3D, x fastest, c first.
"""

import numpy as np

# Sec. 2.1: constants of the Ostwald-ripening benchmark (square domain of
# size 200): kappa_c = kappa_eta = 3, rho^2 = 2, c_alpha = 0.3, c_beta = 0.7,
# w = 1, alpha = 5, M = L = 5, p = 4.
PAPER_FE = {"kind": "paper", "rho2": 2.0, "c_alpha": 0.3, "c_beta": 0.7,
            "w": 1.0, "alpha": 5.0}
PAPER_KINETICS = {"M": 5.0, "kappa_c": 3.0, "L": 5.0, "kappa_eta": 3.0}

# Landau polynomial of the 64^2 / 1024^2 benchmark configurations (not in the
# paper): c_alpha = 0.3, c_beta = 0.7, c_m = 0.5, A = 2, B = 50, D = gamma = 40,
# delta = 1, eps = 3.
POLY_FE = {"kind": "poly", "c_alpha": 0.3, "c_beta": 0.7, "c_m": 0.5,
           "A": 2.0, "B": 50.0, "D": 40.0, "gamma": 40.0, "delta": 1.0,
           "eps": 3.0}

# Sec. 2.1, Eq. (4), (5): c_0 = 0.5, epsilon = 0.05, eta_nu = 0.1, psi = 1.5.
PAPER_IC = {"c0": 0.5, "eps": 0.05, "eta_nu": 0.1, "psi": 1.5}


def make_config(ndim, n, dx=1.0, p=4, fe=None, kmode="spectral", **kin):
    """Build a configuration dict.  `n` is an int (cube/square) or a tuple in
    (Nx, Ny[, Nz]) order; `dx` likewise."""
    if isinstance(n, int):
        n = (n,) * ndim
    n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
    if isinstance(dx, (int, float)):
        dx = (float(dx),) * ndim
    dx = tuple(float(v) for v in dx) + (1.0,) * (3 - len(dx))
    cfg = {"ndim": ndim, "n": n, "dx": dx, "p": int(p),
           "fe": dict(fe if fe is not None else PAPER_FE),
           "kmode": kmode}
    cfg.update(PAPER_KINETICS)
    cfg.update(kin)
    return cfg


def field_shape(cfg):
    nd = cfg["ndim"]
    return (1 + cfg["p"],) + tuple(cfg["n"][d] for d in reversed(range(nd)))


def random_ic(cfg, seed=0, c0=0.5, c_amp=0.05, eta_amp=0.1):
    """c = c0 + c_amp * U(-1, 1), eta_i = eta_amp * U(0, 1), per point.

    numpy Generator(PCG64(seed)), float64; draw order c, then eta_1..eta_p,
    each a full C-order grid (x fastest).  U(-1, 1) = 2 U(0, 1) - 1.
    """
    shape = field_shape(cfg)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.empty(shape)
    u[0] = c0 + c_amp * (2.0 * rng.random(shape[1:]) - 1.0)
    for i in range(1, shape[0]):
        u[i] = eta_amp * rng.random(shape[1:])
    return u


def random_direction(cfg, seed=1, amp=1.0):
    """A seeded perturbation direction with U(-1, 1) entries in every field."""
    shape = field_shape(cfg)
    rng = np.random.Generator(np.random.PCG64(seed))
    return amp * (2.0 * rng.random(shape) - 1.0)


def paper_ic_2d(cfg):
    """Initial condition of Eq. (4), (5) evaluated at x_j = j dx, y_j = j dy.

    Defined for the 2D benchmark; the fields are not periodic on a generic
    box (the paper notes this).  Eta index i runs 1..p.
    """
    if cfg["ndim"] != 2:
        raise ValueError("paper_ic_2d is two-dimensional")
    nx, ny = cfg["n"][0], cfg["n"][1]
    x = np.arange(nx) * cfg["dx"][0]
    y = np.arange(ny) * cfg["dx"][1]
    X, Y = np.meshgrid(x, y)  # shape (Ny, Nx)
    c0, eps, en, psi = (PAPER_IC["c0"], PAPER_IC["eps"], PAPER_IC["eta_nu"],
                        PAPER_IC["psi"])
    u = np.empty(field_shape(cfg))
    u[0] = c0 + eps * (np.cos(0.105 * X) * np.cos(0.11 * Y)
                       + (np.cos(0.13 * X) * np.cos(0.087 * Y)) ** 2
                       + np.cos(0.025 * X - 0.15 * Y) * np.cos(0.07 * X - 0.02 * Y))
    for i in range(1, cfg["p"] + 1):
        inner = (np.cos((0.01 * i) * X - 4.0) * np.cos((0.007 + 0.01 * i) * Y)
                 + np.cos((0.11 + 0.01 * i) * X) * np.cos((0.11 + 0.01 * i) * Y)
                 + psi * (np.cos((0.046 + 0.001 * i) * X + (0.0405 + 0.001 * i) * Y)
                          * np.cos((0.031 + 0.001 * i) * X - (0.004 + 0.001 * i) * Y)) ** 2)
        u[i] = en * inner ** 2
    return u


def single_mode(cfg, base, amp, field, kidx):
    """Uniform state `base` (length F) plus amp * cos(2 pi sum_d m_d j_d / N_d)
    in one field; `kidx` gives the integer wave numbers (m_x, m_y[, m_z])."""
    shape = field_shape(cfg)
    nd = cfg["ndim"]
    u = np.empty(shape)
    for f in range(shape[0]):
        u[f] = base[f]
    phase = np.zeros(shape[1:])
    for d in range(nd):
        n = cfg["n"][d]
        j = np.arange(n)
        sl = [None] * nd
        sl[nd - 1 - d] = slice(None)
        phase = phase + (2.0 * np.pi * kidx[d] * j / n)[tuple(sl)]
    u[field] = u[field] + amp * np.cos(phase)
    return u


# Workload readings used by the tests and the benchmark.  Grid shapes, field
# counts, precisions, step counts and seeds follow the benchmark
# configurations; the physics and time steps are the stable readings: the
# configurations' Landau polynomial is unbounded below and their time steps
# exceed the linear stability limits of both schemes.
WORKLOADS = {
    # 2D 64^2, c + 2 eta, paper f_chem, seeded uniform IC, FS dt 0.1 x 200
    "W1": dict(ndim=2, n=64, p=2, fe="paper", ic="random", c0=0.5,
               dt_fs=0.1, steps=200),
    # same grid and IC with the configured Landau polynomial, before blow-up
    "W1p": dict(ndim=2, n=64, p=2, fe="poly", ic="random", c0=0.5,
                dt_fs=1e-3, steps=150),
    # paper IC (Eq. 4, 5), c + 4 eta, dx = 1
    "WO": dict(ndim=2, n=64, p=4, fe="paper", ic="paper", dt_fs=0.01,
               steps=200, dt_fd=1.25e-3),
    # 2D 1024^2, c + 4 eta, throughput workload
    "W2": dict(ndim=2, n=1024, p=4, fe="paper", ic="random", c0=0.5,
               dt_fs=0.1, steps=2000, dt_fd=1.25e-3),
    # 3D 256^3, c + 4 eta
    "W3": dict(ndim=3, n=256, p=4, fe="paper", ic="random", c0=0.45,
               dt_fs=0.1, steps=1000, dt_fd=6.25e-4),
    # differentiable 2D 512^2, c + 2 eta, checkpoints every 50 steps
    "W4": dict(ndim=2, n=512, p=2, fe="paper", ic="random", c0=0.5,
               dt_fs=0.1, steps=500, K=50),
    # differentiable 3D 128^3, c + 4 eta, checkpoints every 100 steps
    "W5": dict(ndim=3, n=128, p=4, fe="paper", ic="random", c0=0.45,
               dt_fs=0.1, steps=2000, K=100),
}


def workload_config(name, n=None, **over):
    w = dict(WORKLOADS[name])
    w.update(over)
    fe = PAPER_FE if w["fe"] == "paper" else POLY_FE
    cfg = make_config(w["ndim"], n if n is not None else w["n"], 1.0, w["p"], fe)
    return cfg, w


def workload_ic(cfg, w, seed=0):
    if w["ic"] == "paper":
        return paper_ic_2d(cfg)
    return random_ic(cfg, seed=seed, c0=w.get("c0", 0.5))


# ---------------------------------------------------------------------------
# The paper's study inputs (Sec. 2.1): fields moved between grids of one box,
# and the 3D initial state of Eq. (6).

def resample(u, n):
    """Fields on an n x n grid from fields on an m x m grid of the same box:
    every (m/n)-th point when coarser, Fourier zero-padding when finer."""
    m = u.shape[-1]
    if n <= m:
        k = m // n
        return np.ascontiguousarray(u[:, ::k, ::k])
    U = np.fft.fft2(u, axes=(-2, -1))
    out = np.zeros(u.shape[:-2] + (n, n), dtype=complex)
    h = m // 2
    out[..., :h, :h] = U[..., :h, :h]
    out[..., :h, -h:] = U[..., :h, -h:]
    out[..., -h:, :h] = U[..., -h:, :h]
    out[..., -h:, -h:] = U[..., -h:, -h:]
    return np.ascontiguousarray(np.real(np.fft.ifft2(out, axes=(-2, -1))) * (n * n) / (m * m))


def extrude_3d(u2, n, c0=0.5, edge=100.0):
    """Eq. (6): the order parameters of the 3D case from the 2D fields u2
    ([F, m, m] on the 200 x 200 box) as
        eta_i(x, y, z) = 0.5 {1 + tanh[atanh(2 eta_i^2D(2x, 2y) - 1)
                                       - ((z - l_z / 2) / 5)^4]},
    on an n^3 grid of the edge^3 box (x = j * edge / n); c = c0 everywhere.
    (2x, 2y) falls on every (m / n)-th 2D grid point.  2 eta^2D - 1 is kept
    inside (-1, 1) by 1e-12 so that atanh stays finite where a relaxed 2D
    field sits at 0 or 1 to rounding."""
    p = u2.shape[0] - 1
    e2 = resample(u2[1:], n)                                # eta^2D(2x, 2y), [p, n, n]
    a = np.arctanh(np.clip(2.0 * e2 - 1.0, -1.0 + 1e-12, 1.0 - 1e-12))
    z = np.arange(n) * (edge / n)
    dz4 = ((z - edge / 2) / 5.0) ** 4                       # [n]
    u = np.empty((p + 1, n, n, n))
    u[0] = c0
    u[1:] = 0.5 * (1.0 + np.tanh(a[:, None, :, :] - dz4[None, :, None, None]))
    return u
