"""Pins of the equal-time measurements (oracle/measure.py): free fermions
against momentum sums, a random field against the many-body trace over the
Fock space (which does not use Wick's theorem), and the susceptibility of a
fully ordered field."""
import math

import numpy as np

from oracle import measure, stable, fock
from oracle.lattice import hopping_matrix
from slq_inputs import Model, iid_field


def test_free_fermions_match_momentum_sums():
    m = Model(4, 6, 20, t=1.0, mu=-0.4, dtau=0.1, xi=0.0, n_stab=5)
    s = iid_field(m, 3)                      # xi = 0: the field does not enter
    _, _, g = stable.green(m, s)
    dens, hop, _ = measure.equal_time(m, g)
    n_k, e_k = [], []
    for a in range(m.lx):
        for b in range(m.ly):
            eps = -2 * m.t * (math.cos(2 * math.pi * a / m.lx) + math.cos(2 * math.pi * b / m.ly)) - m.mu
            f = 1.0 / (1.0 + math.exp(m.beta * eps))
            n_k.append(f)
            e_k.append((eps + m.mu) * f)
    assert abs(dens - np.mean(n_k)) < 1e-12
    assert abs(hop - np.mean(e_k)) < 1e-12


def test_random_field_matches_fock_trace():
    m = Model(2, 2, 4, t=1.0, mu=-0.3, dtau=0.3, xi=1.4, n_stab=2)
    n = m.n_sites
    c = fock.annihilators(n)
    cd = [x.T for x in c]
    k = hopping_matrix(m.lx, m.ly, m.t, m.mu)
    hk = sum(k[i, j] * cd[i] @ c[j] for i in range(n) for j in range(n))
    w, q = np.linalg.eigh(hk)
    ek = (q * np.exp(-m.dtau * w)) @ q.T
    num = [cd[i] @ c[i] for i in range(n)]
    for key in (5, 6):
        s = iid_field(m, key)
        u = np.eye(2 ** n)
        for l in range(1, m.n_slices + 1):
            v = sum(m.dtau * m.xi * float(s[l - 1][i]) * num[i] for i in range(n))
            u = ek @ np.diag(np.exp(-np.diag(v))) @ u
        z = np.trace(u)
        ex = lambda op: float(np.trace(u @ op)) / z
        k0 = hopping_matrix(m.lx, m.ly, m.t, 0.0)
        dens = np.mean([ex(num[i]) for i in range(n)])
        hop = sum(k0[i, j] * ex(cd[i] @ c[j]) for i in range(n) for j in range(n) if i != j) / n
        sg = [(-1) ** ((i % m.lx) + (i // m.lx)) for i in range(n)]
        spp = sum(sg[i] * sg[j] * ex(num[i] @ num[j]) for i in range(n) for j in range(n)) / n
        _, _, g = stable.green(m, s)
        got = measure.equal_time(m, g)
        np.testing.assert_allclose(got, [dens, hop, spp], rtol=0, atol=1e-12)


def test_susceptibility_of_an_ordered_field_is_n():
    m = Model(3, 5, 20, dtau=0.05)
    mtot = m.n_sites * m.n_slices              # s = +1 everywhere
    assert abs(measure.susceptibility(m, float(mtot) ** 2) - m.n_sites) < 1e-12


def test_displaced_green_is_the_spacetime_inverse_block():
    """Block (l-1, L-1) of the inverse of the space-time matrix is
    -G(tau_l, 0) for l < L, an independent route to the same object; and
    G(beta, 0) = 1 - G."""
    from oracle import lattice
    m = Model(3, 2, 6, t=1.0, mu=-0.3, dtau=0.2, xi=1.1, n_stab=3)
    s = iid_field(m, 4)
    n, L = m.n_sites, m.n_slices
    rhs = np.zeros((n * L, n))
    rhs[(L - 1) * n:, :] = np.eye(n)
    col = np.linalg.solve(lattice.spacetime_matrix(m, s), rhs)
    for l in range(1, L):
        np.testing.assert_allclose(measure.green_displaced(m, s, l), -col[(l - 1) * n:l * n], atol=1e-13)
    _, _, g = stable.green(m, s)
    np.testing.assert_allclose(measure.green_displaced(m, s, L), np.eye(n) - g, atol=1e-13)
