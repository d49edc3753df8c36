"""Pins for the oracle's free energies, gradients and Hessians (no GPU).

Gradients and Hessians are checked against central differences of the
density itself; the density is checked at the equilibrium states Sec. 2.1
names (alpha matrix: eta = 0 at c_alpha; a beta particle: eta_i = 1 at
c_beta), where the paper's f_chem and its gradient vanish, and at a point
evaluated by hand for the Landau polynomial."""

import numpy as np
import pytest

from oracle import freeenergy as fe
from paper_2306_04322_amd.inputs import PAPER_FE, POLY_FE


def _points(p, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.empty((1 + p, n))
    u[0] = rng.uniform(0.0, 1.0, n)
    u[1:] = rng.uniform(-0.2, 1.2, (p, n))
    return u


@pytest.mark.parametrize("kind", ["paper", "poly"])
@pytest.mark.parametrize("p", [1, 2, 4])
def test_gradient_matches_central_differences(kind, p):
    f = PAPER_FE if kind == "paper" else POLY_FE
    u = _points(p, 200, 7)
    g = fe.gradient(u, f)
    h = 1e-6
    for a in range(1 + p):
        up = u.copy()
        um = u.copy()
        up[a] += h
        um[a] -= h
        num = (fe.density(up, f) - fe.density(um, f)) / (2 * h)
        assert np.max(np.abs(num - g[a])) <= 1e-7 * max(1.0, np.max(np.abs(g[a])))


@pytest.mark.parametrize("kind", ["paper", "poly"])
@pytest.mark.parametrize("p", [1, 3])
def test_hessian_matches_central_differences(kind, p):
    f = PAPER_FE if kind == "paper" else POLY_FE
    u = _points(p, 100, 8)
    H = fe.hessian(u, f)
    h = 1e-6
    for b in range(1 + p):
        up = u.copy()
        um = u.copy()
        up[b] += h
        um[b] -= h
        num = (fe.gradient(up, f) - fe.gradient(um, f)) / (2 * h)
        for a in range(1 + p):
            assert np.max(np.abs(num[a] - H[a, b])) <= 1e-6 * max(1.0, np.max(np.abs(H[a, b])))
    assert np.max(np.abs(H - np.swapaxes(H, 0, 1))) <= 1e-14 * np.max(np.abs(H))
    v = _points(p, 100, 9)
    hv = fe.hessian_vector(u, f, v)
    manual = sum(H[:, b] * v[b] for b in range(1 + p))
    assert np.max(np.abs(hv - manual)) <= 1e-12


@pytest.mark.parametrize("p", [1, 4])
def test_paper_equilibria_are_zero_energy_minima(p):
    f = PAPER_FE
    alpha = np.zeros((1 + p, 1))
    alpha[0] = f["c_alpha"]
    assert fe.density(alpha, f)[0] == 0.0
    assert np.max(np.abs(fe.gradient(alpha, f))) == 0.0
    for i in range(p):
        beta = np.zeros((1 + p, 1))
        beta[0] = f["c_beta"]
        beta[1 + i] = 1.0
        assert abs(fe.density(beta, f)[0]) <= 1e-15
        assert np.max(np.abs(fe.gradient(beta, f))) <= 1e-14
    # the interpolation function runs from h(0) = 0 to h(1) = 1: halfway in
    # c between the phases with one eta at 1/2 the density is
    # rho2 * 0.2^2 * (1 - 1/2) + rho2 * 0.2^2 * 1/2 + w * (1/16)
    mid = np.zeros((1 + p, 1))
    mid[0] = 0.5
    mid[1] = 0.5
    assert abs(fe.density(mid, f)[0] - (2.0 * 0.04 + 1.0 / 16.0)) <= 1e-15


def test_pair_term_counts_ordered_pairs():
    # two order parameters at 1/2 each, c = c_alpha: the alpha-weighted
    # double sum over ordered pairs i != j contributes 2 * (1/4 * 1/4).
    f = PAPER_FE
    u = np.array([[0.3], [0.5], [0.5]])
    h = 2 * (0.5 ** 3 * (6 * 0.25 - 7.5 + 10))
    fb = 2.0 * 0.4 ** 2
    expect = fb * h + 1.0 * (2 * 0.0625 + 5.0 * 2 * 0.0625)
    assert abs(fe.density(u, f)[0] - expect) <= 1e-14


def test_poly_hand_values():
    f = POLY_FE
    # c = c_m = 0.5, eta = 0: only the two D/4 quartics survive: 2 * 10 * 0.2^4
    u = np.array([[0.5], [0.0], [0.0]])
    assert abs(fe.density(u, f)[0] - 0.032) <= 1e-15
    # curvature at that point: -A + 3 D (0.04 + 0.04) = 7.6
    assert abs(fe.hessian(u, f)[0, 0, 0] - 7.6) <= 1e-13
