"""Checkerboard (sparse) form of the kinetic factor of a slice matrix.

"Formalism of SLDQMC" counts the chain of a cumulative update as beta N^2,
which presumes slice matrices that factor into sparse pieces whose number
grows like N.  On an lx x ly torus
with even sides the nearest-neighbour bonds split into four groups of
disjoint bonds: x bonds leaving an even x (A), leaving an odd x (B), y bonds
leaving an even y (C), leaving an odd y (D).  The hopping of one group,
K_g = -t sum_{(i,j) in g} (|i><j| + |j><i|), has exp(-dtau K_g) = a rotation
cosh(dtau t) + sinh(dtau t) sigma_x on each of its bonds.  The symmetric
(Strang) split

    E_cb = e^{dtau mu} e^{-dtau K_A/2} e^{-dtau K_B/2} e^{-dtau K_C/2} e^{-dtau K_D}
                       e^{-dtau K_C/2} e^{-dtau K_B/2} e^{-dtau K_A/2}

is symmetric and differs from E = exp(-dtau K) by O(dtau^3); with it
B_l = E_cb diag(d_l) is a different discretisation of the same model, and its
weight det(1 + B_L ... B_1) is evaluated exactly like the dense one's.  A
length-2 side lists its doubled bond once in each of its two groups, so the
groups sum to the hopping matrix with the multiplicity convention of K.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import stable


def bond_groups(lx: int, ly: int):
    """The four groups (A, B, C, D) of bonds (i, j), each a list of disjoint pairs."""
    if lx % 2 or ly % 2:
        raise ValueError("the checkerboard split needs even lx and ly")
    groups = [[], [], [], []]
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            groups[x % 2].append((i, (x + 1) % lx + lx * y))
            groups[2 + y % 2].append((i, x + lx * ((y + 1) % ly)))
    return groups


def group_hopping(n: int, bonds, t: float) -> np.ndarray:
    k = np.zeros((n, n))
    for i, j in bonds:
        k[i, j] -= t
        k[j, i] -= t
    return k


def propagator(lx: int, ly: int, t: float, mu: float, dtau: float) -> np.ndarray:
    """E_cb as the product of the seven group exponentials (matrix exponentials of
    the dense group matrices) times e^{dtau mu}."""
    n = lx * ly
    a, b, c, d = (group_hopping(n, g, t) for g in bond_groups(lx, ly))
    half = [sla.expm(-0.5 * dtau * k) for k in (a, b, c)]
    mid = sla.expm(-dtau * d)
    e = half[0] @ half[1] @ half[2] @ mid @ half[2] @ half[1] @ half[0]
    return np.exp(dtau * mu) * e


def weight(model, s):
    """(log|W|, sign) of det(1 + B_L ... B_1) with B_l = E_cb diag(d_l), stabilised."""
    e = propagator(model.lx, model.ly, model.t, model.mu, model.dtau)
    return stable.udv_finish(*stable.udv_chain(model, s, e=e), want_green=False)[:2]


def green(model, s):
    """(log|W|, sign, G) with the checkerboard slice matrices."""
    e = propagator(model.lx, model.ly, model.t, model.mu, model.dtau)
    return stable.udv_finish(*stable.udv_chain(model, s, e=e))
