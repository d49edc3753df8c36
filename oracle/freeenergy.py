"""Oracle chemical free energies, their gradients and Hessians (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two densities are supported:

* ``paper`` -- the chemical free energy of Sec. 2.1:
      f = f_alpha (1 - h) + f_beta h + w g,
      f_alpha = rho2 (c - c_alpha)^2,  f_beta = rho2 (c_beta - c)^2,
      h = sum_i eta_i^3 (6 eta_i^2 - 15 eta_i + 10),
      g = sum_i eta_i^2 (1 - eta_i)^2 + alpha sum_i sum_{j != i} eta_i^2 eta_j^2.
  The double sum runs over ordered pairs, as written.

* ``poly`` -- a Landau polynomial used by one benchmark configuration of
  this library (it is not in the paper):
      f = -A/2 (c-c_m)^2 + B/4 (c-c_m)^4 + D/4 (c-c_alpha)^4 + D/4 (c-c_beta)^4
          - gamma/2 (c-c_alpha)^2 sum_i eta_i^2 + delta/4 sum_i eta_i^4
          + eps/2 sum_i sum_{j != i} eta_i^2 eta_j^2.

`u` is an array of shape (F, ...) with u[0] = c and u[1:] = eta_i.
`fe` is a dict {"kind": "paper"|"poly", **coefficients}.

The derivatives below are the hand-differentiated forms; tests pin each of
them to central differences of `density` itself.
"""

import numpy as np


def density(u, fe):
    """Pointwise chemical free-energy density f(c, eta_1..eta_p)."""
    c = u[0]
    eta = u[1:]
    if fe["kind"] == "paper":
        rho2, ca, cb, w, al = (fe["rho2"], fe["c_alpha"], fe["c_beta"],
                               fe["w"], fe["alpha"])
        h = np.sum(eta ** 3 * (6.0 * eta ** 2 - 15.0 * eta + 10.0), axis=0)
        s2 = np.sum(eta ** 2, axis=0)
        pair = np.zeros_like(c)
        for i in range(eta.shape[0]):
            pair = pair + eta[i] ** 2 * (s2 - eta[i] ** 2)
        g = np.sum(eta ** 2 * (1.0 - eta) ** 2, axis=0) + al * pair
        fa = rho2 * (c - ca) ** 2
        fb = rho2 * (cb - c) ** 2
        return fa * (1.0 - h) + fb * h + w * g
    if fe["kind"] == "poly":
        ca, cb, cm = fe["c_alpha"], fe["c_beta"], fe["c_m"]
        A, B, D = fe["A"], fe["B"], fe["D"]
        gam, dl, ep = fe["gamma"], fe["delta"], fe["eps"]
        s2 = np.sum(eta ** 2, axis=0)
        pair = np.zeros_like(c)
        for i in range(eta.shape[0]):
            pair = pair + eta[i] ** 2 * (s2 - eta[i] ** 2)
        return (-A / 2.0 * (c - cm) ** 2 + B / 4.0 * (c - cm) ** 4
                + D / 4.0 * (c - ca) ** 4 + D / 4.0 * (c - cb) ** 4
                - gam / 2.0 * (c - ca) ** 2 * s2
                + dl / 4.0 * np.sum(eta ** 4, axis=0)
                + ep / 2.0 * pair)
    raise ValueError("unknown free energy kind %r" % fe["kind"])


def _h1(e):
    """dh/deta for one order parameter: 30 eta^2 (1-eta)^2."""
    return 30.0 * e ** 2 * (1.0 - e) ** 2


def _h2(e):
    """d2h/deta2: 60 eta (1-eta)(1-2 eta)."""
    return 60.0 * e * (1.0 - e) * (1.0 - 2.0 * e)


def gradient(u, fe):
    """(df/dc, df/deta_1, ..., df/deta_p): the explicit terms of Eq. (2), (3)."""
    c = u[0]
    eta = u[1:]
    out = np.empty_like(u)
    s2 = np.sum(eta ** 2, axis=0)
    if fe["kind"] == "paper":
        rho2, ca, cb, w, al = (fe["rho2"], fe["c_alpha"], fe["c_beta"],
                               fe["w"], fe["alpha"])
        h = np.sum(eta ** 3 * (6.0 * eta ** 2 - 15.0 * eta + 10.0), axis=0)
        out[0] = 2.0 * rho2 * ((c - ca) - (cb - ca) * h)
        jump = rho2 * ((cb - c) ** 2 - (c - ca) ** 2)
        for i in range(eta.shape[0]):
            e = eta[i]
            out[1 + i] = (jump * _h1(e)
                          + w * (2.0 * e * (1.0 - e) * (1.0 - 2.0 * e)
                                 + 4.0 * al * e * (s2 - e ** 2)))
        return out
    if fe["kind"] == "poly":
        ca, cb, cm = fe["c_alpha"], fe["c_beta"], fe["c_m"]
        A, B, D = fe["A"], fe["B"], fe["D"]
        gam, dl, ep = fe["gamma"], fe["delta"], fe["eps"]
        out[0] = (-A * (c - cm) + B * (c - cm) ** 3 + D * (c - ca) ** 3
                  + D * (c - cb) ** 3 - gam * (c - ca) * s2)
        for i in range(eta.shape[0]):
            e = eta[i]
            out[1 + i] = (-gam * (c - ca) ** 2 * e + dl * e ** 3
                          + 2.0 * ep * e * (s2 - e ** 2))
        return out
    raise ValueError("unknown free energy kind %r" % fe["kind"])


def hessian(u, fe):
    """Pointwise Hessian H[a, b] = d2f / du_a du_b, shape (F, F, ...)."""
    c = u[0]
    eta = u[1:]
    p = eta.shape[0]
    F = p + 1
    H = np.zeros((F, F) + c.shape)
    s2 = np.sum(eta ** 2, axis=0)
    if fe["kind"] == "paper":
        rho2, ca, cb, w, al = (fe["rho2"], fe["c_alpha"], fe["c_beta"],
                               fe["w"], fe["alpha"])
        H[0, 0] = 2.0 * rho2
        jump = rho2 * ((cb - c) ** 2 - (c - ca) ** 2)
        for i in range(p):
            e = eta[i]
            H[0, 1 + i] = H[1 + i, 0] = -2.0 * rho2 * (cb - ca) * _h1(e)
            H[1 + i, 1 + i] = (jump * _h2(e)
                               + w * (2.0 * (1.0 - 6.0 * e + 6.0 * e ** 2)
                                      + 4.0 * al * (s2 - e ** 2)))
            for j in range(p):
                if j != i:
                    H[1 + i, 1 + j] = 8.0 * w * al * e * eta[j]
        return H
    if fe["kind"] == "poly":
        ca, cb, cm = fe["c_alpha"], fe["c_beta"], fe["c_m"]
        A, B, D = fe["A"], fe["B"], fe["D"]
        gam, dl, ep = fe["gamma"], fe["delta"], fe["eps"]
        H[0, 0] = (-A + 3.0 * B * (c - cm) ** 2 + 3.0 * D * (c - ca) ** 2
                   + 3.0 * D * (c - cb) ** 2 - gam * s2)
        for i in range(p):
            e = eta[i]
            H[0, 1 + i] = H[1 + i, 0] = -2.0 * gam * (c - ca) * e
            H[1 + i, 1 + i] = (-gam * (c - ca) ** 2 + 3.0 * dl * e ** 2
                               + 2.0 * ep * (s2 - e ** 2))
            for j in range(p):
                if j != i:
                    H[1 + i, 1 + j] = 4.0 * ep * e * eta[j]
        return H
    raise ValueError("unknown free energy kind %r" % fe["kind"])


def hessian_vector(u, fe, v):
    """Pointwise product H(u) v for a stack v of shape (F, ...)."""
    H = hessian(u, fe)
    return np.einsum("ab...,b...->a...", H, v)
