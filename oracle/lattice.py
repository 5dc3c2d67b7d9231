"""Hopping matrix, slice propagators and the exact fermion weight by definition.

Follows "Basics of DQMC", Eq. (1): for one auxiliary-field configuration
C = {s_{i,l}} the fermion weight is det(1 + B(beta,0;C)) with
B(beta,0) = B^L ... B^1, and each slice matrix is the kinetic propagator times
the exponential of the field coupling.  Sign conventions (the reading taken):

    K_ij = -t for nearest neighbours (bond multiplicity kept on Lx=2), K_ii = -mu
    E    = exp(-dtau K),   d_l = exp(-dtau xi s_{., l}),   B_l = E diag(d_l)
    W_f(s) = det(1 + B_L ... B_1),   G = (1 + B_L ... B_1)^{-1}

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def hopping_matrix(lx: int, ly: int, t: float, mu: float) -> np.ndarray:
    """Tight-binding matrix K of the periodic lx x ly square lattice (site
    i = x + lx*y); each bond to +x and +y is added once, so a dimension of
    length 2 carries a doubled bond, matching eps_k = -2t(cos kx + cos ky) - mu."""
    n = lx * ly
    k = np.zeros((n, n))
    for y in range(ly):
        for x in range(lx):
            i = x + lx * y
            for dx, dy in ((1, 0), (0, 1)):
                j = (x + dx) % lx + lx * ((y + dy) % ly)
                k[i, j] -= t
                k[j, i] -= t
            k[i, i] -= mu
    return k


def kinetic_propagators(lx, ly, t, mu, dtau):
    """E = exp(-dtau K) and its inverse from the eigendecomposition of K."""
    w, q = np.linalg.eigh(hopping_matrix(lx, ly, t, mu))
    e = (q * np.exp(-dtau * w)) @ q.T
    einv = (q * np.exp(dtau * w)) @ q.T
    return e, einv


def field_diagonal(s_l, dtau: float, xi: float) -> np.ndarray:
    """Diagonal of exp(V) for one slice: exp(-dtau xi s_i)."""
    return np.exp(-dtau * xi * np.asarray(s_l, dtype=np.float64))


def slice_matrix(e, s_l, dtau, xi) -> np.ndarray:
    """B_l = E diag(d_l)."""
    return e * field_diagonal(s_l, dtau, xi)[None, :]


def chain_product(model, s, order=None) -> np.ndarray:
    """Plain (unstabilised) product B_{order[-1]} ... B_{order[0]}; by default
    order = 1..L, i.e. B(beta,0) = B_L ... B_1.  Slice l uses s[l-1]."""
    e, _ = kinetic_propagators(model.lx, model.ly, model.t, model.mu, model.dtau)
    order = range(1, model.n_slices + 1) if order is None else order
    p = np.eye(model.n_sites)
    for l in order:
        p = slice_matrix(e, s[l - 1], model.dtau, model.xi) @ p
    return p


def weight_direct(model, s):
    """(log|W_f|, sign W_f) from det(1 + B_L ... B_1) without stabilisation.
    Only valid while the plain product stays well inside FP64 range."""
    sign, logabs = np.linalg.slogdet(np.eye(model.n_sites) + chain_product(model, s))
    return float(logabs), int(np.sign(sign))


def green_direct(model, s) -> np.ndarray:
    """G = (1 + B_L ... B_1)^{-1} without stabilisation."""
    return np.linalg.inv(np.eye(model.n_sites) + chain_product(model, s))


def green_at_slice(model, s, m: int) -> np.ndarray:
    """G_m = (1 + B_m ... B_1 B_L ... B_{m+1})^{-1} without stabilisation;
    G_0 = G_L = G."""
    L = model.n_slices
    order = list(range(m + 1, L + 1)) + list(range(1, m + 1))
    return np.linalg.inv(np.eye(model.n_sites) + chain_product(model, s, order))


def spacetime_matrix(model, s) -> np.ndarray:
    """The NL x NL block matrix with identity diagonal blocks, -B_{b+1} at block
    (b, b-1) for b = 1..L-1 and +B_1 at block (0, L-1) (0-based).  Its
    determinant equals det(1 + B_L ... B_1), and diagonal block b of its
    inverse is G_{b+1}; it reaches both without ever forming the chain."""
    e, _ = kinetic_propagators(model.lx, model.ly, model.t, model.mu, model.dtau)
    n, L = model.n_sites, model.n_slices
    o = np.eye(n * L)
    for b in range(L):
        blk = slice_matrix(e, s[b], model.dtau, model.xi)      # B_{b+1}
        if b == 0:
            o[0:n, (L - 1) * n:L * n] += blk
        else:
            o[b * n:(b + 1) * n, (b - 1) * n:b * n] -= blk
    return o


def weight_spacetime(model, s):
    """(log|W_f|, sign, G) from the space-time block matrix."""
    o = spacetime_matrix(model, s)
    lu, piv = sla.lu_factor(o)
    d = np.diag(lu)
    logabs = float(np.sum(np.log(np.abs(d))))
    nswap = int(np.count_nonzero(piv != np.arange(len(piv))))
    sign = (-1) ** nswap * int(np.prod(np.sign(d)))
    n, L = model.n_sites, model.n_slices
    rhs = np.zeros((n * L, n))
    rhs[(L - 1) * n:, :] = np.eye(n)
    g = sla.lu_solve((lu, piv), rhs)[(L - 1) * n:, :]
    return logabs, sign, g
