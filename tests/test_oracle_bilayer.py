"""Pins of the bilayer workload's oracle (oracle/bilayer.py; "Results", Eq. 6).

* The bare Ising weight phi: for one spin the imaginary-time chain sums to
  the transverse-field partition function 2 cosh(beta h) exactly (all
  slices); for two coupled spins the Trotterised sum over every configuration
  converges to Tr exp(-beta H_s) with an error that falls as dtau^2.
* The four-flavour fermion weight [W_f(s) W_f(-s)]^2: equal to the
  determinant of the 4N-dimensional single-particle problem written directly
  from Eq. 6's coupling -xi s (sigma^z_1 - sigma^z_2), and to the many-body
  trace over the 2^(4N) Fock states of the four flavours.
* The local update: its ratio equals the recomputed ratio of weights, and the
  tracked weight and both Green's functions after sweeps equal recomputed ones.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import bilayer, stable
from slq_inputs import Model, iid_field


def all_fields(model):
    n = model.n_sites * model.n_slices
    for bits in itertools.product((1, -1), repeat=n):
        yield np.array(bits, dtype=np.int8).reshape(model.n_slices, model.n_sites)


@pytest.mark.parametrize("M,h", [(4, 0.7), (7, 2.774), (10, 1.3)])
def test_single_spin_chain_is_the_transverse_field_partition_function(M, h):
    m = Model(1, 1, M, dtau=1.0 / M)          # beta = 1; J = 0 (a single spin has no bonds of its own)
    a2 = 0.5 * math.sinh(2 * m.dtau * h)       # squared constant of one transfer-matrix element
    z = sum(math.exp(bilayer.bare_log_weight(m, 0.0, h, s)) for s in all_fields(m)) * a2 ** (M / 2)
    assert abs(z - 2 * math.cosh(m.beta * h)) < 1e-12 * z


def test_two_spins_converge_to_the_transverse_field_ising_model():
    """Lattice 2x1: the x bond is listed twice and each site has a y bond to
    itself, so H_s = -J (2 s0 s1 + 2) - h (sx0 + sx1).  The Trotter error of
    the partition function falls as dtau^2 (checked between M = 5 and 8)."""
    J, h, beta = 0.6, 1.1, 1.0
    sz = np.diag([1.0, -1.0])
    sx = np.array([[0.0, 1.0], [1.0, 0.0]])
    i2 = np.eye(2)
    H = -J * (2 * np.kron(sz, sz) + 2 * np.eye(4)) - h * (np.kron(sx, i2) + np.kron(i2, sx))
    z_exact = float(np.trace(sla.expm(-beta * H)))
    errs = {}
    for M in (5, 8):
        m = Model(2, 1, M, dtau=beta / M)
        a2 = 0.5 * math.sinh(2 * m.dtau * h)
        z = sum(math.exp(bilayer.bare_log_weight(m, J, h, s)) for s in all_fields(m)) * a2 ** (2 * M / 2)
        errs[M] = (z - z_exact) / z_exact
    assert abs(errs[8]) < 0.02
    assert 0.5 * (8 / 5) ** 2 < errs[5] / errs[8] < 1.5 * (8 / 5) ** 2


@pytest.mark.parametrize("model", [
    Model(4, 4, 20, t=1.0, mu=-0.5, dtau=0.05, xi=1.0, n_stab=10),
    Model(3, 2, 6, t=1.0, mu=0.3, dtau=0.2, xi=1.5, n_stab=3),
])
def test_four_flavour_weight_equals_the_single_particle_determinant(model):
    for key in (11, 12, 13):
        s = iid_field(model, key)
        la, _ = stable.weight(model, s)
        lb, _ = stable.weight(model, -s)
        ref = bilayer.fermion_log_weight_single_particle(model, s)
        assert abs(2 * (la + lb) - ref) < 1e-10 * max(1.0, abs(ref))
        J, h = 0.8, 2.774
        assert abs(bilayer.log_weight(model, J, h, s) - ref - bilayer.bare_log_weight(model, J, h, s)) < 1e-9


def test_four_flavour_weight_equals_the_fock_trace():
    m = Model(2, 1, 4, t=1.0, mu=-0.4, dtau=0.25, xi=1.2, n_stab=2)
    for key in (21, 22, 23):
        s = iid_field(m, key)
        w = bilayer.fermion_weight_fock(m, s)
        la, _ = stable.weight(m, s)
        lb, _ = stable.weight(m, -s)
        assert w > 0 and abs(math.log(w) - 2 * (la + lb)) < 1e-11


def test_local_ratio_is_the_weight_ratio():
    m = Model(3, 4, 8, t=1.0, mu=-0.5, dtau=0.05, xi=1.0, n_stab=4)
    J, h = 1.0, 2.774
    s = iid_field(m, 31)
    lw = bilayer.log_weight(m, J, h, s)
    ga, gb = bilayer.green_pair(m, s)   # chain ending at B_L; rotate to slice 1 via the cyclic chain
    # the ratio at slice 1 uses the Green's functions of the chain ending at B_1
    ga1 = stable.green_at_slice(m, s, 0)
    gb1 = stable.green_at_slice(m, -s, 0)
    np.testing.assert_allclose(ga1, ga, atol=1e-12)
    kt = bilayer.bare_coupling(m.dtau, h)
    for i in (0, 5, 11):
        si = float(s[0, i])
        nb = [j for a, b in bilayer.bonds(m.lx, m.ly) for (u, j) in ((a, b), (b, a)) if u == i]
        hloc = m.dtau * J * sum(float(s[0, j]) for j in nb) + kt * (float(s[1, i]) + float(s[-1, i]))
        da, db = math.exp(2 * m.dtau * m.xi * si) - 1, math.exp(-2 * m.dtau * m.xi * si) - 1
        r = math.exp(-2 * si * hloc) * ((1 + da * (1 - ga1[i, i])) * (1 + db * (1 - gb1[i, i]))) ** 2
        s2 = s.copy()
        s2[0, i] = -s2[0, i]
        assert abs(math.log(r) - (bilayer.log_weight(m, J, h, s2) - lw)) < 1e-10


def test_sweeps_track_the_weight_and_green_functions():
    m = Model(3, 3, 8, t=1.0, mu=-0.5, dtau=0.05, xi=1.0, n_stab=4)
    J, h = 1.0, 2.774
    s = iid_field(m, 41)
    ga, gb = bilayer.green_pair(m, s)
    lw = bilayer.log_weight(m, J, h, s)
    acc_tot = 0
    for k in range(3):
        lw, acc, drift = bilayer.sweep(m, J, h, s, ga, gb, lw, seed=5, sweep_index=k, chain=0)
        acc_tot += acc
        assert drift < 1e-10
    assert 0 < acc_tot < 3 * m.n_sites * m.n_slices
    assert abs(lw - bilayer.log_weight(m, J, h, s)) < 1e-9 * max(1.0, abs(lw))
    ra, rb = bilayer.green_pair(m, s)
    np.testing.assert_allclose(ga, ra, atol=1e-10)
    np.testing.assert_allclose(gb, rb, atol=1e-10)
