"""Brute-force many-body trace for tiny lattices (pins sign and G ordering).

The fermion weight of Eq. (1) is the trace over the fermion Fock space of the
ordered product of slice operators
    W_f = Tr[ prod_{l=L..1} exp(-dtau H_K) exp(-dtau xi sum_i s_{i,l} n_i) ],
with H_K = sum_ij K_ij c_i^dag c_j.  For N sites the Fock space has 2^N states,
so this is only for N <= 6 or so.  Creation/annihilation operators come from
the Jordan-Wigner construction.  Equal-time Green's function
G_ij = <c_i c_j^dag> = Tr(U c_i c_j^dag) / Tr(U).

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from .lattice import hopping_matrix


def annihilators(n: int):
    """Jordan-Wigner matrices c_0..c_{n-1} on the 2^n-dimensional Fock space."""
    a = np.array([[0.0, 1.0], [0.0, 0.0]])      # |1> -> |0>
    z = np.diag([1.0, -1.0])
    i2 = np.eye(2)
    ops = []
    for j in range(n):
        m = np.array([[1.0]])
        for k in range(n):
            m = np.kron(m, z if k < j else (a if k == j else i2))
        ops.append(m)
    return ops


def fock_weight_and_green(model, s):
    """(W_f, G) by explicit trace over the 2^N Fock states."""
    n, L = model.n_sites, model.n_slices
    c = annihilators(n)
    cd = [m.T for m in c]
    k = hopping_matrix(model.lx, model.ly, model.t, model.mu)
    hk = sum(k[i, j] * cd[i] @ c[j] for i in range(n) for j in range(n))
    w, q = np.linalg.eigh(hk)
    ek = (q * np.exp(-model.dtau * w)) @ q.T
    num = [cd[i] @ c[i] for i in range(n)]
    u = np.eye(2 ** n)
    for l in range(1, L + 1):
        v = sum(model.dtau * model.xi * float(s[l - 1][i]) * num[i] for i in range(n))
        ev = np.diag(np.exp(-np.diag(v)))            # number operators are diagonal
        u = ek @ ev @ u
    z = np.trace(u)
    g = np.array([[np.trace(u @ c[i] @ cd[j]) for j in range(n)] for i in range(n)]) / z
    return float(z), g
