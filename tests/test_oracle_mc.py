"""Pins of the oracle's Monte Carlo parts: determinant ratio and rank-1 update
against recomputation, the wrap identity, effective-action changes against
brute force, exact detailed balance of the cumulative update on an enumerable
state space, a sampling histogram, the regression and the autocorrelation time."""
import itertools
import math

import numpy as np
import pytest

from oracle import lattice, stable, dqmc, effective, fit, autocorr, philox
from slq_inputs import Model, SMALL_4x4, iid_field, default_terms


# ------------------------------------------------------------ local DQMC ----
def test_ratio_and_rank1_update_match_recomputation():
    m = Model(3, 4, 6, t=1.0, mu=-0.4, dtau=0.2, xi=1.3, n_stab=3)
    s = iid_field(m, 11)
    for l, i in [(1, 0), (3, 5), (6, 11)]:
        g = lattice.green_at_slice(m, s, l - 1)                     # G_{l-1}
        w0, sg0 = lattice.weight_direct(m, s)
        delta = math.exp(2 * m.dtau * m.xi * s[l - 1, i]) - 1
        r = 1 + delta * (1 - g[i, i])
        s2 = s.copy()
        s2[l - 1, i] *= -1
        w1, sg1 = lattice.weight_direct(m, s2)
        assert abs(math.log(abs(r)) - (w1 - w0)) < 1e-12 and np.sign(r) == sg0 * sg1
        col = -g[:, i].copy()
        col[i] += 1
        g2 = g - (delta / r) * np.outer(col, g[i, :])
        assert np.max(np.abs(g2 - lattice.green_at_slice(m, s2, l - 1))) < 1e-13
        # the row/column-swapped form of the update is wrong for this ordering
        g_bad = g - (delta / r) * np.outer(g[:, i], col)
        assert np.max(np.abs(g_bad - lattice.green_at_slice(m, s2, l - 1))) > 1e-4


def test_wrap_identity():
    m = Model(4, 3, 8, t=1.0, mu=0.2, dtau=0.1, xi=1.5, n_stab=4)
    s = iid_field(m, 12)
    e, einv = lattice.kinetic_propagators(m.lx, m.ly, m.t, m.mu, m.dtau)
    for l in (1, 4, 8):
        g = lattice.green_at_slice(m, s, l - 1)
        b = lattice.slice_matrix(e, s[l - 1], m.dtau, m.xi)
        assert np.max(np.abs(b @ g @ np.linalg.inv(b) - lattice.green_at_slice(m, s, l))) < 1e-13


def test_sweep_tracks_weight_and_green():
    m = SMALL_4x4
    s = iid_field(m, 13)
    logabs, sign, g = stable.green(m, s)
    for sw in range(2):
        logabs, sign, acc, drift, tr = dqmc.sweep(m, s, g, logabs, sign, seed=0x5D0C, sweep_index=sw,
                                                  want_trace=True)
        assert 0 < acc < m.n_sites * m.n_slices and drift < 1e-10
        assert len(tr) == m.n_sites * m.n_slices
    la, sb, gb = stable.green(m, s)
    assert sb == sign and abs(la - logabs) < 1e-10 * abs(la)
    assert np.max(np.abs(g - gb)) < 1e-10
    # the acceptance draws are the documented Philox counters
    l, i, r, u, a = tr[37]
    assert u == philox.uniform((i, l - 1, 1, 0), (0x5D0C, philox.TAG_LOCAL)) and a == (u < abs(r))


# ------------------------------------------------------- effective model ----
def test_shells():
    assert effective.shell_offsets(0) == ((0, 0),)
    assert sorted(effective.shell_offsets(1)) == [(-1, 0), (0, -1), (0, 1), (1, 0)]
    assert sorted(effective.shell_offsets(2)) == [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    assert sorted(effective.shell_offsets(3)) == [(-2, 0), (0, -2), (0, 2), (2, 0)]
    assert len(effective.shell_offsets(4)) == 8


def test_default_terms_count():
    assert len(default_terms(20)) == 17          # one-body + 2 spatial + 10 temporal + 4 space-time


def test_one_body_term_is_the_magnetisation():
    """F of the term (0, 0) is sum_x s_x, its local field is 1 and a flip of x
    changes it by -2 s_x, independently of every other site."""
    m = Model(3, 4, 6, xi=1.0)
    s = iid_field(m, 23)
    f = effective.features(m, [(0, 0), (1, 0)], s)
    assert f[0] == int(s.astype(np.int64).sum())
    assert np.array_equal(effective.local_fields(m, [(0, 0)], s)[0], np.ones((6, 12)))
    assert effective.flip_delta(m, [(0, 0)], [0.3], s, 4, 2) == -2.0 * 0.3 * s[1, 4]
    assert effective.partners(m, (0, 0), 4, 2) == []


def test_local_fields_vectorised_equals_partner_lists():
    m = Model(3, 4, 6, xi=1.0)
    terms = default_terms(6) + [(3, 0), (4, 1)]
    s = iid_field(m, 21)
    a = effective.local_fields(m, terms, s)
    b = effective.local_fields_bruteforce(m, terms, s)
    assert np.array_equal(a, b)
    for l in range(1, m.n_slices + 1):
        assert np.array_equal(effective.local_fields_slice(m, terms, s, l), b[:, l - 1])
    m2 = Model(5, 3, 9, xi=1.0)
    terms2 = default_terms(9) + [(2, 3), (5, 4)]
    s2 = iid_field(m2, 22)
    b2 = effective.local_fields_bruteforce(m2, terms2, s2)
    for l in range(1, m2.n_slices + 1):
        assert np.array_equal(effective.local_fields_slice(m2, terms2, s2, l), b2[:, l - 1])


def test_flip_delta_equals_action_difference():
    m = Model(4, 4, 8, xi=1.0)
    terms = default_terms(8)
    effective.check_terms(m, terms)
    lam = np.random.default_rng(5).normal(size=len(terms))
    s = iid_field(m, 22)
    f = effective.features(m, terms, s)
    assert np.array_equal(2 * f, np.round(2 * f))                  # half-integers
    base = effective.action(m, terms, 0.7, lam, s)
    for i, l in [(0, 1), (5, 4), (15, 8)]:
        s2 = s.copy()
        s2[l - 1, i] *= -1
        d = effective.flip_delta(m, terms, lam, s, i, l)
        assert abs(d - (effective.action(m, terms, 0.7, lam, s2) - base)) < 1e-12


def test_self_partner_terms_rejected():
    with pytest.raises(ValueError):
        effective.check_terms(Model(2, 4, 8), [(3, 0)])            # (+-2, 0) wraps onto itself
    with pytest.raises(ValueError):
        effective.check_terms(Model(4, 4, 8), [(1, 5)])            # dl > L/2


def test_colour_classes_hold_no_coupled_pair():
    m = Model(5, 4, 6)
    terms = default_terms(6)
    classes = effective.colour_classes(m, terms)
    covered = sorted((l, i) for l, sites in classes for i in sites)
    assert covered == [(l, i) for l in range(1, 7) for i in range(20)]
    for l, sites in classes:
        for i in sites:
            for k in terms:
                assert not any((j, ll) == (jj, l) for j, ll in effective.partners(m, k, i, l) for jj in sites)


def _states(m):
    n = m.n_sites * m.n_slices
    return [np.array([(1 if (c >> b) & 1 else -1) for b in range(n)], np.int8).reshape(m.n_slices, m.n_sites)
            for c in range(2 ** n)]


def test_cumulative_update_detailed_balance_exact():
    """Exact transition matrix on the 2x2, L=2 space (256 states)."""
    m = Model(2, 2, 2, t=1.0, mu=-0.3, dtau=0.4, xi=1.2, n_stab=1)
    terms = [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1)]
    effective.check_terms(m, terms)
    lam = np.array([-0.2, 0.15, -0.05, 0.3, 0.02])
    states = _states(m)
    ns = len(states)
    w = np.array([stable.weight(m, s)[0] for s in states])
    sa = np.array([effective.action(m, terms, 0.0, lam, s) for s in states])
    classes = effective.colour_classes(m, terms)
    idx = {s.tobytes(): a for a, s in enumerate(states)}
    keff = np.zeros((ns, ns))
    for a, s in enumerate(states):
        for l, sites in classes:
            probs = [min(1.0, math.exp(effective.flip_delta(m, terms, lam, s, i, l))) for i in sites]
            for pat in itertools.product([0, 1], repeat=len(sites)):
                t = s.copy()
                p = 1.0
                for i, f, q in zip(sites, pat, probs):
                    p *= q if f else 1 - q
                    if f:
                        t[l - 1, i] *= -1
                keff[a, idx[t.tobytes()]] += p / len(classes)
    assert np.allclose(keff.sum(1), 1, atol=1e-13)
    # the effective chain alone is reversible for exp(S_eff)
    flow = np.exp(sa)[:, None] * keff
    assert np.max(np.abs(flow - flow.T)) < 1e-12 * np.max(flow)
    prop = np.linalg.matrix_power(keff, 3)
    log_a = (w[None, :] - w[:, None]) - (sa[None, :] - sa[:, None])
    t = prop * np.minimum(1.0, np.exp(log_a))
    np.fill_diagonal(t, 0)
    np.fill_diagonal(t, 1 - t.sum(1))
    flow = np.exp(w - w.max())[:, None] * t
    assert np.max(np.abs(flow - flow.T)) < 1e-12
    # a plausible mistake (dropping the effective-action term of Eq. 4) breaks it
    bad = prop * np.minimum(1.0, np.exp(w[None, :] - w[:, None]))
    np.fill_diagonal(bad, 0)
    np.fill_diagonal(bad, 1 - bad.sum(1))
    fb = np.exp(w - w.max())[:, None] * bad
    assert np.max(np.abs(fb - fb.T)) > 1e-4


def test_cumulative_update_samples_weight_histogram():
    """The sampling code itself (Philox draws included) reproduces |W| on 2x2, L=2."""
    m = Model(2, 2, 2, t=1.0, mu=-0.3, dtau=0.4, xi=1.2, n_stab=1)
    terms = [(1, 0), (0, 1)]
    states = _states(m)
    w = np.array([stable.weight(m, s)[0] for s in states])
    feats = np.array([effective.features(m, terms, s) for s in states])
    c0, lam, r2 = fit.fit(m, terms, states, w)
    p = np.exp(w - w.max())
    p /= p.sum()
    cache = {s.tobytes(): (wv, 1) for s, wv in zip(states, w)}
    classes = effective.colour_classes(m, terms)
    s = states[0].copy()
    logabs, sign = cache[s.tobytes()]
    counts = np.zeros(len(states))
    idx = {st.tobytes(): a for a, st in enumerate(states)}
    n = 6000
    acc = 0
    for step in range(n):
        s, logabs, sign, ok, _ = effective.cumulative_step(
            m, terms, c0, lam, s, logabs, sign, 2, lambda x: cache[x.tobytes()],
            seed=99, step=step, classes=classes)
        acc += ok
        counts[idx[s.tobytes()]] += 1
    assert 0.2 < acc / n < 1.0
    # chi-square over the magnetisation sectors (M = sum s, 9 values)
    mag = np.array([int(st.sum()) for st in states])
    obs = np.array([counts[mag == v].sum() for v in range(-8, 9, 2)])
    exp = np.array([p[mag == v].sum() * n for v in range(-8, 9, 2)])
    keep = exp > 20
    chi2 = float((((obs - exp) ** 2) / exp)[keep].sum())
    from scipy.stats import chi2 as c2
    # correlated samples: inflate by a generous factor for the autocorrelation
    assert c2.sf(chi2 / 4.0, keep.sum() - 1) > 1e-3, (obs, exp)


def test_perfect_effective_action_always_accepts():
    m = Model(2, 2, 2, t=1.0, mu=-0.3, dtau=0.4, xi=1.2, n_stab=1)
    terms = [(1, 0), (0, 1)]
    s0 = iid_field(m, 5)
    # an exactly linear "true" log-weight: acceptance must be 1 for every proposal
    lam = np.array([0.2, -0.1])
    true = lambda x: (effective.action(m, terms, 1.5, lam, x), 1)   # noqa: E731
    s, la, sg = s0.copy(), true(s0)[0], 1
    for step in range(20):
        s, la, sg, ok, log_a = effective.cumulative_step(m, terms, 1.5, lam, s, la, sg, 3, true,
                                                          seed=7, step=step)
        assert ok and abs(log_a) < 1e-12


# ------------------------------------------------------------------- fit ----
def test_fit_recovers_exactly_linear_target():
    m = Model(4, 4, 8)
    terms = default_terms(8)
    fields = [iid_field(m, 300 + i) for i in range(60)]
    lam = np.random.default_rng(1).normal(size=len(terms))
    y = [effective.action(m, terms, -2.5, lam, s) for s in fields]
    c0, got, r2 = fit.fit(m, terms, fields, y)
    assert abs(c0 + 2.5) < 1e-9 and np.max(np.abs(got - lam)) < 1e-10 and abs(r2 - 1) < 1e-12


def test_fit_on_random_labels_scores_low():
    m = Model(4, 4, 8)
    terms = [(1, 0), (0, 1)]
    fields = [iid_field(m, 400 + i) for i in range(400)]
    y = np.random.default_rng(2).normal(size=400)
    assert fit.fit(m, terms, fields, y)[2] < 0.05


# ------------------------------------------------------ autocorrelation ----
@pytest.mark.parametrize("rho", [-0.9, -0.5, 0.0, 0.5, 0.9])
def test_tau_int_ar1(rho):
    g = np.random.default_rng(4)
    n = 200000
    x = np.empty(n)
    x[0] = g.normal()
    noise = g.normal(size=n)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + noise[t]
    exact = (1 + rho) / (2 * (1 - rho))
    assert abs(autocorr.tau_int(x) - exact) < 0.06 * exact + 0.02


def test_tau_int_of_a_period_two_series_is_its_closed_form():
    """An anticorrelated AR(1) (rho = -0.8): tau_int = (1 + rho) / (2 (1 - rho)),
    far below 1/2, where the windowed sum alone would stop at a negative value."""
    g = np.random.default_rng(5)
    rho, n = -0.8, 400000
    x = np.empty(n)
    x[0] = g.normal()
    noise = g.normal(size=n)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + noise[t]
    exact = (1 + rho) / (2 * (1 - rho))
    assert 0.5 + autocorr.autocorrelation(x)[1] < 0    # the window's own estimate is negative
    assert abs(autocorr.tau_int(x) - exact) < 0.01


# ------------------------------------------- package analysis vs oracle ----
def test_package_tau_int_matches_ar1_and_oracle():
    from paper_1612_03804_amd.analysis import tau_int_chains
    g = np.random.default_rng(8)
    rho, chains, T = 0.7, 64, 4000
    x = np.empty((chains, T))
    x[:, 0] = g.normal(size=chains) / np.sqrt(1 - rho * rho)
    noise = g.normal(size=(chains, T))
    for t in range(1, T):
        x[:, t] = rho * x[:, t - 1] + noise[:, t]
    exact = (1 + rho) / (2 * (1 - rho))
    assert abs(tau_int_chains(x) - exact) < 0.05 * exact
    assert abs(tau_int_chains(x[0]) - autocorr.tau_int(x[0])) < 0.1 * exact
    # anticorrelated chains (rho = -0.7): the initial positive sequence
    rho = -0.7
    x[:, 0] = g.normal(size=chains) / np.sqrt(1 - rho * rho)
    for t in range(1, T):
        x[:, t] = rho * x[:, t - 1] + noise[:, t]
    exact = (1 + rho) / (2 * (1 - rho))
    assert abs(tau_int_chains(x) - exact) < 0.01
