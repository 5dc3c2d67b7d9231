"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, a brute-force Fock-space trace, the space-time block matrix,
lattice symmetries, a library generator and exact small-case enumerations."""
import json
import math
import os

import numpy as np
import pytest

from oracle import lattice, stable, fock, philox
from slq_inputs import Model, SMALL_4x4, iid_field

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def eps_k(m, nx, ny):
    return -2 * m.t * (math.cos(2 * math.pi * nx / m.lx) + math.cos(2 * math.pi * ny / m.ly)) - m.mu


def free_logw(m, extra=0.0):
    """sum_k log(1 + exp(-beta eps_k - extra)) by explicit momentum loops."""
    return sum(math.log1p(math.exp(-m.beta * eps_k(m, nx, ny) - extra))
               for nx in range(m.lx) for ny in range(m.ly))


def free_green(m, extra=0.0):
    """G_ij = (1/N) sum_k cos(k.(r_i - r_j)) / (1 + exp(-beta eps_k - extra))."""
    n = m.n_sites
    g = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            dx, dy = i % m.lx - j % m.lx, i // m.lx - j // m.lx
            g[i, j] = sum(math.cos(2 * math.pi * (nx * dx / m.lx + ny * dy / m.ly))
                          / (1 + math.exp(-m.beta * eps_k(m, nx, ny) - extra))
                          for nx in range(m.lx) for ny in range(m.ly)) / n
    return g


# ---------------------------------------------------------------- Philox ----
@pytest.mark.parametrize("ctr,key", [((1, 0, 0, 0), (0, 0)), ((5, 7, 9, 11), (123, 456)),
                                      ((2 ** 63 + 17, 3, 2 ** 64 - 1, 1), (2 ** 64 - 5, 1)),
                                      ((12, 0, 7, 3), (0x5D0C, philox.TAG_LOCAL))])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox increments its counter before each block of four words.
    before = np.array([ctr[0] - 1, ctr[1], ctr[2], ctr[3]], dtype=np.uint64)
    ref = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=before).random_raw(8)
    assert list(philox.philox4x64_10(ctr, key)) == [int(x) for x in ref[:4]]
    nxt = (ctr[0] + 1, ctr[1], ctr[2], ctr[3])
    assert list(philox.philox4x64_10(nxt, key)) == [int(x) for x in ref[4:]]


def test_philox_uniform_and_below_ranges():
    us = [philox.uniform((i, 1, 2, 3), (9, 1)) for i in range(2000)]
    assert 0.0 <= min(us) and max(us) < 1.0 and abs(np.mean(us) - 0.5) < 0.03
    bs = [philox.below(7, (i, 0, 0, 0), (9, 2)) for i in range(2000)]
    assert set(bs) == set(range(7))


# ------------------------------------------------------------ model prep ----
def test_kinetic_propagator_spectrum_and_inverse():
    m = Model(4, 6, 10, t=1.0, mu=-0.5, dtau=0.1)
    e, einv = lattice.kinetic_propagators(m.lx, m.ly, m.t, m.mu, m.dtau)
    assert np.max(np.abs(e @ einv - np.eye(m.n_sites))) < 1e-14
    # eigenvalues of E are exp(-dtau eps_k) for the lattice momenta
    ref = sorted(math.exp(-m.dtau * eps_k(m, nx, ny)) for nx in range(m.lx) for ny in range(m.ly))
    assert np.allclose(sorted(np.linalg.eigvalsh(e)), ref, rtol=1e-14, atol=0)
    # translation invariance of E: E[i, j] depends on r_i - r_j only
    assert abs(e[0, 1] - e[m.lx + 2, m.lx + 3]) < 1e-15


def test_bond_multiplicity_on_two_site_dimension():
    k = lattice.hopping_matrix(2, 3, 1.0, 0.25)
    assert k[0, 1] == -2.0 and k[0, 2] == -1.0 and k[0, 0] == -0.25


# --------------------------------------------------------- closed forms -----
def test_free_fermions_logw_and_green():
    m = SMALL_4x4.with_(xi=0.0)
    s = iid_field(SMALL_4x4, 1000)
    logabs, sign, g = stable.green(m, s)
    assert sign == 1
    assert abs(logabs - 28.30475331944794) < 1e-12 * 28.3
    assert abs(free_logw(m) - 28.30475331944794) < 1e-12 * 28.3
    assert np.max(np.abs(g - free_green(m))) < 1e-13


@pytest.mark.parametrize("spin,expected", [(1, 15.281703935017592), (-1, 47.28170393501759)])
def test_uniform_field_shifts_mu(spin, expected):
    m = SMALL_4x4
    s = np.full((m.n_slices, m.n_sites), spin, np.int8)
    logabs, sign, g = stable.green(m, s)
    ref = free_logw(m, extra=m.dtau * m.xi * spin * m.n_slices)
    assert abs(ref - expected) < 1e-12 * expected
    assert sign == 1 and abs(logabs - ref) < 1e-13 * ref
    assert np.max(np.abs(g - free_green(m, extra=m.dtau * m.xi * spin * m.n_slices))) < 1e-13


def test_space_uniform_time_varying_field():
    m = Model(4, 4, 20, t=1.0, mu=0.3, dtau=0.1, xi=1.2, n_stab=7)
    prof = np.where(np.arange(m.n_slices) % 3 == 0, 1, -1).astype(np.int8)
    s = np.repeat(prof[:, None], m.n_sites, axis=1)
    ref = free_logw(m, extra=m.dtau * m.xi * float(prof.sum()))
    assert abs(stable.weight(m, s)[0] - ref) < 1e-13 * abs(ref)


def test_zero_hopping_is_a_product_over_sites():
    m = Model(3, 4, 16, t=0.0, mu=0.4, dtau=0.125, xi=1.3, n_stab=5)
    s = iid_field(m, 77)
    tot = s.astype(np.float64).sum(axis=0)
    x = m.beta * m.mu - m.dtau * m.xi * tot
    logabs, sign, g = stable.green(m, s)
    assert sign == 1 and abs(logabs - np.sum(np.log1p(np.exp(x)))) < 1e-13 * abs(logabs)
    assert np.max(np.abs(g - np.diag(1.0 / (1.0 + np.exp(x))))) < 1e-14


# ---------------------------------------------------- brute-force traces ----
def test_fock_trace_random_fields():
    m = Model(2, 2, 4, t=1.0, mu=-0.5, dtau=0.5, xi=1.7, n_stab=3)
    g0 = np.random.default_rng(3)
    for _ in range(12):
        s = (2 * g0.integers(0, 2, (4, 4)) - 1).astype(np.int8)
        z, gf = fock.fock_weight_and_green(m, s)
        logabs, sign, g = stable.green(m, s)
        assert sign == np.sign(z) and abs(logabs - math.log(abs(z))) < 1e-12 * max(1, abs(logabs))
        assert np.max(np.abs(g - gf)) < 1e-12
        # the transposed ordering is a different matrix: G_ij = <c_i c_j^dag>
        assert np.max(np.abs(g.T - gf)) > 1e-3 or np.max(np.abs(g - g.T)) < 1e-12


def test_fock_trace_negative_weights():
    fx = json.load(open(os.path.join(GOLDEN, "negative_weights_2x2_L4.json")))
    m = Model(**fx["model"])
    assert len(fx["negative_codes"]) == 288
    for code, w in list(zip(fx["negative_codes"], fx["negative_weights"]))[::24]:
        bits = (code >> np.arange(16)) & 1
        s = (2 * bits - 1).astype(np.int8).reshape(4, 4)
        z, gf = fock.fock_weight_and_green(m, s)
        assert z < 0 and abs(z - w) < 1e-10 * abs(w)
        logabs, sign, g = stable.green(m, s)
        assert sign == -1 and abs(logabs - math.log(-z)) < 1e-11 * max(1, abs(logabs))
        assert np.max(np.abs(g - gf)) < 1e-9 * max(1.0, np.max(np.abs(gf)))


def test_spacetime_matrix_matches_stabilised_chain():
    m = SMALL_4x4
    s = iid_field(m, 1001)
    la, sg, g = lattice.weight_spacetime(m, s)
    lb, sb, gb = stable.green(m, s)
    assert sg == sb and abs(la - lb) < 1e-12 * abs(la)
    assert np.max(np.abs(g - gb)) < 1e-12


def test_stabilisation_at_low_temperature():
    """beta = 8 on 4x4: the plain product has lost digits, the block matrix has not."""
    m = Model(4, 4, 80, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10)
    s = iid_field(m, 1002)
    la, sg, g = lattice.weight_spacetime(m, s)
    lb, sb, gb = stable.green(m, s)
    assert sg == sb and abs(la - lb) < 1e-12 * abs(la)
    assert np.max(np.abs(g - gb)) < 1e-11
    # the stabilisation interval does not change the result
    lc, sc, gc = stable.green(m.with_(n_stab=3), s)
    assert abs(lc - lb) < 1e-12 * abs(lb) and np.max(np.abs(gc - gb)) < 1e-11


def test_unstabilised_product_agrees_at_small_beta():
    m = SMALL_4x4
    s = iid_field(m, 1003)
    la, sa = lattice.weight_direct(m, s)
    lb, sb = stable.weight(m, s)
    assert sa == sb and abs(la - lb) < 1e-10 * abs(la)
    assert np.max(np.abs(lattice.green_direct(m, s) - stable.green(m, s)[2])) < 1e-8


# -------------------------------------------------------------- symmetry ----
def test_lattice_and_time_symmetries():
    m = Model(4, 4, 12, t=1.0, mu=-0.3, dtau=0.15, xi=1.4, n_stab=5)
    s = iid_field(m, 1004)
    ref = stable.weight(m, s)[0]
    s3 = s.reshape(m.n_slices, m.ly, m.lx)
    variants = {
        "translate": np.roll(s3, (1, 2), axis=(1, 2)),
        "rotate": np.rot90(s3, 1, axes=(1, 2)),
        "mirror": s3[:, :, ::-1],
        "time shift": np.roll(s3, 5, axis=0),
        "time reversal": s3[::-1],
    }
    for name, v in variants.items():
        got = stable.weight(m, np.ascontiguousarray(v).reshape(m.n_slices, m.n_sites))[0]
        assert abs(got - ref) < 1e-12 * abs(ref), name
    # a genuinely different field gives a different weight (the test can fail)
    other = s.copy()
    other[0, 0] *= -1
    assert abs(stable.weight(m, other)[0] - ref) > 1e-6


def test_particle_hole_at_half_filling():
    m = Model(4, 4, 20, t=1.0, mu=0.0, dtau=0.1, xi=1.0, n_stab=10)
    s = iid_field(m, 1005)
    a = stable.weight(m, s)[0]
    b = stable.weight(m, -s)[0]
    assert abs(a - (b - m.dtau * m.xi * float(s.astype(np.float64).sum()))) < 1e-12 * abs(a)
