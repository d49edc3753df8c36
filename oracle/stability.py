"""Oracle linear stability bounds of the FS and FD steps.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3 reports that the largest stable time steps were found by trial and
error, that the FS step's limit does not shrink as the grid is refined, and
that the FD limit does.  This module gives the per-Fourier-mode bounds of
both schemes linearised about a uniform state with curvatures
f_cc = d2f/dc2 and f_ee = d2f/deta2 (no coupling at eta = 0):

FS Cahn-Hilliard (Eq. (14)): G(x) = (1 - a x) / (1 + b x^2), x = |xi|^2,
  a = dt M f_cc, b = dt M kappa_c.  G <= 1 always; G >= -1 for every x >= 0
  iff a^2 <= 8 b, i.e. dt <= 8 kappa_c / (M f_cc^2)  (grid independent).
FS Allen-Cahn (Eq. (15)): G = (1 - dt L f_ee) / (1 + dt L kappa_eta x),
  worst at x = 0: dt <= 2 / (L f_ee).
FD (forward Euler, 2nd-order Laplacian with symbol q in [0, q_max],
  q_max = sum_d 4 / dx_d^2):
  Cahn-Hilliard G = 1 - dt M q (f_cc + kappa_c q): dt <= 2 / (M q_max (f_cc + kappa_c q_max))
  Allen-Cahn    G = 1 - dt L (f_ee + kappa_eta q): dt <= 2 / (L (f_ee + kappa_eta q_max))

A non-positive curvature is a physical instability (spinodal growth), not a
numerical one; those bounds are reported as +inf.
"""

import math


def fs_bound(M, kappa_c, L, f_cc, f_ee):
    ch = math.inf if f_cc <= 0 else 8.0 * kappa_c / (M * f_cc * f_cc)
    ac = math.inf if f_ee <= 0 else 2.0 / (L * f_ee)
    return min(ch, ac)


def fd_bound(M, kappa_c, L, kappa_eta, f_cc, f_ee, dxs):
    qmax = sum(4.0 / (d * d) for d in dxs)
    ch = 2.0 / (M * qmax * (max(f_cc, 0.0) + kappa_c * qmax))
    ac = 2.0 / (L * (max(f_ee, 0.0) + kappa_eta * qmax))
    return min(ch, ac)
