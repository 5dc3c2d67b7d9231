"""Pins of the checkerboard slice propagator (oracle/checkerboard.py).

* The four bond groups hold disjoint bonds and together give the hopping
  matrix (with the doubled bond of a length-2 side).
* Each group's exponential is the closed-form rotation cosh + sinh sigma_x on
  its bonds.
* E_cb is symmetric, det E_cb = e^{N dtau mu}, and E_cb - exp(-dtau K) falls as
  dtau^3 (the symmetric split's local error).
* With t = 0 the weight is the product over sites, as for the dense E.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import checkerboard, stable
from oracle.lattice import hopping_matrix, kinetic_propagators
from slq_inputs import Model, iid_field


@pytest.mark.parametrize("lx,ly", [(4, 4), (2, 6), (6, 2), (8, 4)])
def test_groups_are_disjoint_and_sum_to_the_hopping(lx, ly):
    n = lx * ly
    groups = checkerboard.bond_groups(lx, ly)
    total = np.zeros((n, n))
    for g in groups:
        sites = [i for b in g for i in b]
        assert len(sites) == len(set(sites)) == n      # every site in exactly one bond of the group
        total += checkerboard.group_hopping(n, g, 1.3)
    np.testing.assert_array_equal(total, hopping_matrix(lx, ly, 1.3, 0.0))


def test_group_exponential_is_a_rotation_per_bond():
    n, t, dt = 16, 0.9, 0.17
    g = checkerboard.bond_groups(4, 4)[2]
    e = sla.expm(-dt * checkerboard.group_hopping(n, g, t))
    ref = np.zeros((n, n))
    for i, j in g:
        ref[i, i] = ref[j, j] = math.cosh(dt * t)
        ref[i, j] = ref[j, i] = math.sinh(dt * t)
    np.testing.assert_allclose(e, ref, atol=1e-14)


def test_symmetric_unit_determinant_and_third_order_error():
    lx, ly, t, mu = 6, 4, 1.0, -0.5
    errs = []
    for dt in (0.1, 0.05):
        ecb = checkerboard.propagator(lx, ly, t, mu, dt)
        np.testing.assert_allclose(ecb, ecb.T, atol=1e-15)
        assert abs(np.linalg.slogdet(ecb)[1] - lx * ly * dt * mu) < 1e-12
        e, _ = kinetic_propagators(lx, ly, t, mu, dt)
        errs.append(np.max(np.abs(ecb - e)))
    assert 6.0 < errs[0] / errs[1] < 10.0


def test_no_hopping_gives_the_product_over_sites():
    m = Model(4, 2, 12, t=0.0, mu=0.3, dtau=0.1, xi=1.2, n_stab=4)
    s = iid_field(m, 8)
    la, sg = checkerboard.weight(m, s)
    ref = sum(math.log1p(math.exp(m.beta * m.mu - m.dtau * m.xi * float(s[:, i].sum()))) for i in range(m.n_sites))
    assert sg == 1 and abs(la - ref) < 1e-12 * ref


def test_weight_and_green_converge_to_the_dense_ones():
    """The checkerboard and dense discretisations of the same model approach
    each other as dtau^2 at fixed beta (the global Trotter error of the
    split): on a 6x4 lattice with a uniform field, halving dtau divides the
    difference of log W by 4.  (On 4x4 the two spectra happen to coincide.)"""
    diffs = []
    for L in (10, 20, 40):
        m = Model(6, 4, L, t=1.0, mu=-0.3, dtau=1.0 / L, xi=0.5, n_stab=5)
        s = np.ones((L, m.n_sites), dtype=np.int8)
        la_cb, _, g_cb = checkerboard.green(m, s)
        la, _, g = stable.green(m, s)
        diffs.append(abs(la_cb - la))
    assert 3.5 < diffs[0] / diffs[1] < 4.5 and 3.5 < diffs[1] / diffs[2] < 4.5
