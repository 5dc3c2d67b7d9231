"""Equal-time measurements from the Green's function G_ij = <c_i c_j^dag>
(the quantity the local updates of "Basics of DQMC" carry along) and the
Ising susceptibility of "Results".

For one fermion flavour and one auxiliary-field configuration the fermions
are free, so every equal-time expectation follows from G (Wick's theorem):

    <c_i^dag c_j> = delta_ij - G_ji,
    <n_i n_j>     = (1 - G_ii)(1 - G_jj) + (delta_ij - G_ji) G_ij.

Measured per configuration (its Monte Carlo average is the observable):
    density      n = (1/N) sum_i (1 - G_ii)
    hopping      e = (1/N) sum_{i != j} K_ij <c_i^dag c_j>   (K of the model, without mu)
    S(pi, pi)    (1/N) sum_ij (-1)^(x_i + y_i + x_j + y_j) <n_i n_j>   (even lx, ly)

Susceptibility of the Ising spins ("Results"):
    chi = (1/(beta N)) sum_ij int_0^beta dtau <s_i(tau) s_j(0)>
        = dtau^2 <M^2> / (beta^2 N),   M = sum_{i,l} s_{i,l},
(the integral as a sum over slices, time-translation averaged).

Time-displaced Green's function of one configuration:
    G(tau_l, 0) = <c(tau_l) c^dag(0)> = B_l ... B_1 G,   1 <= l <= L,
the plain product (valid while it stays well inside the FP64 range, i.e. at
small beta).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import stable
from .lattice import hopping_matrix, chain_product


def equal_time(model, g) -> np.ndarray:
    """(density, hopping energy per site, S(pi, pi)) of one Green's function."""
    n, lx = model.n_sites, model.lx
    g = np.asarray(g, dtype=np.float64)
    k = hopping_matrix(model.lx, model.ly, model.t, 0.0)
    cdc = np.eye(n) - g.T                            # <c_i^dag c_j>
    dens = float(np.mean(1.0 - np.diag(g)))
    hop = float(sum(k[i, j] * cdc[i, j] for i in range(n) for j in range(n) if i != j)) / n
    sgn = np.array([(-1) ** ((i % lx) + (i // lx)) for i in range(n)], dtype=np.float64)
    s = 0.0
    for i in range(n):
        for j in range(n):
            nn = (1.0 - g[i, i]) * (1.0 - g[j, j]) + cdc[i, j] * g[i, j]
            s += sgn[i] * sgn[j] * nn
    return np.array([dens, hop, s / n])


def susceptibility(model, m2: float) -> float:
    """chi from <M^2> of the total magnetisation M = sum_{i,l} s_{i,l}."""
    return model.dtau ** 2 * m2 / (model.beta ** 2 * model.n_sites)


def green_displaced(model, s, l: int) -> np.ndarray:
    """G(tau_l, 0) = B_l ... B_1 G (plain product; small beta only)."""
    _, _, g = stable.green(model, s)
    return chain_product(model, s, range(1, l + 1)) @ g
