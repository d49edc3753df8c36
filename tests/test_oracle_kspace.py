"""Pins for the oracle's frequency grids (no GPU).

Eq. (17)/(20) redefine |xi|^2 as the symbol of the second-order centred
Laplacian; Eq. (18)/(21) as that of the fourth-order one.  Applying those
stencils (written out here as shifted sums) to a plane wave exp(i xi.x)
must return exactly -|xi|^2 times the wave."""

import numpy as np
import pytest

from oracle import kspace, fd


def test_index_vector_as_printed():
    # Eq. (16): [0, ..., p/2, -(p/2 - 1), ..., -1]
    assert list(kspace.index_vector(8)) == [0, 1, 2, 3, 4, -3, -2, -1]
    assert list(kspace.index_vector(2)) == [0, 1]


def test_spectral_k2_values():
    # l = N dx; xi = 2 pi n / l
    t = kspace.sq_axis(8, 0.5, "spectral")
    expect = (2 * np.pi * np.array([0, 1, 2, 3, 4, -3, -2, -1]) / 4.0) ** 2
    assert np.max(np.abs(t - expect)) <= 1e-14


def _plane_wave(shape, dxs, m):
    nd = len(shape)
    phase = np.zeros(shape)
    for a in range(nd):
        n = shape[a]
        j = np.arange(n)
        sl = [None] * nd
        sl[a] = slice(None)
        phase = phase + (2 * np.pi * m[a] * j / n)[tuple(sl)]
    return np.exp(1j * phase)


@pytest.mark.parametrize("shape,dxs", [((8, 16), (0.7, 1.3)), ((4, 8, 16), (1.0, 0.5, 2.0))])
def test_fd2_symbol_is_5_7_point_eigenvalue(shape, dxs):
    nd = len(shape)
    k2 = kspace.k2_grid(shape, dxs, "fd2")
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(6):
        m = [int(rng.integers(0, n)) for n in shape]
        w = _plane_wave(shape, dxs, m)
        lap = fd.laplacian_h(w, dxs, tuple(range(nd)))
        idx = tuple(m)
        assert np.max(np.abs(lap + k2[idx] * w)) <= 1e-11 * max(1.0, k2[idx])


@pytest.mark.parametrize("shape,dxs", [((8, 16), (0.7, 1.3)), ((4, 8, 8), (1.0, 0.5, 2.0))])
def test_fd4_symbol_is_fourth_order_stencil_eigenvalue(shape, dxs):
    nd = len(shape)
    k2 = kspace.k2_grid(shape, dxs, "fd4")
    rng = np.random.Generator(np.random.PCG64(6))
    for _ in range(6):
        m = [int(rng.integers(0, n)) for n in shape]
        w = _plane_wave(shape, dxs, m)
        lap = np.zeros_like(w)
        for a in range(nd):
            d = dxs[nd - 1 - a]
            lap += (-np.roll(w, -2, a) + 16 * np.roll(w, -1, a) - 30 * w
                    + 16 * np.roll(w, 1, a) - np.roll(w, 2, a)) / (12 * d * d)
        idx = tuple(m)
        assert np.max(np.abs(lap + k2[idx] * w)) <= 1e-11 * max(1.0, k2[idx])


def test_fd_symbols_converge_to_spectral():
    # for a fixed physical wave number the FD symbols approach xi^2 as
    # O(dx^2) and O(dx^4)
    errs2, errs4 = [], []
    for n in (16, 32, 64):
        dx = 10.0 / n
        s = kspace.sq_axis(n, dx, "spectral")[2]
        errs2.append(abs(kspace.sq_axis(n, dx, "fd2")[2] - s) / s)
        errs4.append(abs(kspace.sq_axis(n, dx, "fd4")[2] - s) / s)
    assert 3.5 < errs2[0] / errs2[1] < 4.5 and 3.5 < errs2[1] / errs2[2] < 4.5
    assert 14 < errs4[0] / errs4[1] < 18 and 14 < errs4[1] / errs4[2] < 18
    assert np.all(kspace.sq_axis(32, 0.3, "fd2") >= 0)
    assert np.all(kspace.sq_axis(32, 0.3, "fd4") >= 0)
