"""Pins of the oracle's learned action: a one-site lattice where every
neighbour is the site itself (closed form), translation invariance, central
finite differences of the gradient, the Adam update against its textbook
formula, and the single-flip change against two forward passes."""
import numpy as np

from oracle import net
from slq_inputs import Model, iid_field, net_init


def test_parameter_count():
    assert net.N_PARAMS == 1969 and len(net_init(1)) == 1969


def test_one_site_lattice_closed_form():
    m = Model(1, 1, 1)
    p = net_init(3, scale=2.0)
    p[-1] = 0.3
    W1, b1, W2, b2, w3, b3 = net.unpack(p)
    p[216:224] = np.linspace(-0.2, 0.2, 8)
    W1, b1, W2, b2, w3, b3 = net.unpack(p)
    for sv in (1, -1):
        h1 = np.tanh(b1 + sv * W1.reshape(8, 27).sum(1))
        h2 = np.tanh(b2 + W2.reshape(8, 8, 27).sum(2) @ h1)
        S = b3 + w3 @ h2
        assert abs(net.forward(p, m, np.array([[sv]], np.int8))[0] - S) < 1e-14


def test_translation_invariance():
    m = Model(4, 3, 5)
    p = net_init(4, scale=1.5)
    s = iid_field(m, 11)
    s3 = s.reshape(5, 3, 4)
    S0 = net.forward(p, m, s)[0]
    sh = np.roll(s3, (2, 1, 3), axis=(0, 1, 2)).reshape(5, 12)
    assert abs(net.forward(p, m, sh)[0] - S0) < 1e-12
    # and a different field gives a different value
    s2 = s.copy()
    s2[0, 0] *= -1
    assert abs(net.forward(p, m, s2)[0] - S0) > 1e-9


def test_gradient_central_differences():
    m = Model(3, 4, 4)
    p = net_init(5, scale=1.5)
    p[-9:-1] = np.random.default_rng(0).normal(size=8)
    fields = [iid_field(m, 20 + k) for k in range(2)]
    targets = [0.3, -1.1]
    loss, g = net.loss_and_gradient(p, m, fields, targets)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(216, 6, replace=False), 216 + rng.choice(8, 2, replace=False),
                          224 + rng.choice(1728, 8, replace=False), 1952 + np.arange(2), 1960 + np.arange(2), [1968]])
    h = 1e-6
    for k in idx:
        pp, pm = p.copy(), p.copy()
        pp[k] += h
        pm[k] -= h
        fd = (net.loss_and_gradient(pp, m, fields, targets)[0] - net.loss_and_gradient(pm, m, fields, targets)[0]) / (2 * h)
        assert abs(fd - g[k]) < 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_adam_matches_formula():
    p = np.array([1.0, -2.0])
    g = np.array([0.5, -0.1])
    m = np.zeros(2)
    v = np.zeros(2)
    p1, m1, v1 = net.adam(p, g, m, v, 1, lr=0.1)
    # first step of Adam moves each parameter by lr * sign(g) (bias-corrected)
    assert np.allclose(p1, p - 0.1 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), atol=1e-12)


def test_adam_constant_gradient_steps():
    """With a constant gradient g and zero initial moments, the bias-corrected
    moments are exactly g and g^2 at every step t, so each of the first steps
    moves a parameter by lr * g / (|g| + eps).  A wrong power in either bias
    correction (e.g. (1 - beta1)^t) breaks this from t = 2 on."""
    p = np.array([1.0, -2.0, 0.25, 3.0])
    g = np.array([0.5, -0.1, 2.0, -1e-3])
    m = np.zeros(4)
    v = np.zeros(4)
    lr, eps = 0.05, 1e-8
    for t in range(1, 6):
        p_new, m, v = net.adam(p, g, m, v, t, lr=lr, eps=eps)
        np.testing.assert_allclose(p_new, p - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-13)
        p = p_new


def test_adam_moments_are_weighted_sums():
    """The moment recursions written out: after steps with gradients g_1..g_t,
    m_t = (1 - b1) sum_k b1^(t-k) g_k and v_t = (1 - b2) sum_k b2^(t-k) g_k^2;
    the update divides them by 1 - b^t.  Checked over five steps of changing
    gradients (signs and sizes differ from step to step)."""
    b1, b2, lr, eps = 0.9, 0.999, 1e-2, 1e-8
    gs = [np.array([0.3, -1.0]), np.array([-0.7, 0.2]), np.array([1.5, 0.0]), np.array([0.1, 4.0]),
          np.array([-2.0, -0.5])]
    p = np.array([0.0, 1.0])
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(1, 6):
        p_new, m, v = net.adam(p, gs[t - 1], m, v, t, lr=lr, beta1=b1, beta2=b2, eps=eps)
        ms = (1 - b1) * sum(b1 ** (t - k) * gs[k - 1] for k in range(1, t + 1))
        vs = (1 - b2) * sum(b2 ** (t - k) * gs[k - 1] ** 2 for k in range(1, t + 1))
        np.testing.assert_allclose(m, ms, rtol=1e-14, atol=1e-16)
        np.testing.assert_allclose(v, vs, rtol=1e-14, atol=1e-16)
        step = lr * (ms / (1 - b1 ** t)) / (np.sqrt(vs / (1 - b2 ** t)) + eps)
        np.testing.assert_allclose(p_new, p - step, rtol=0, atol=1e-14)
        p = p_new


def test_single_flip_delta():
    m = Model(5, 5, 6)
    p = net_init(6, scale=1.5)
    p[-9:-1] = 1.0
    s = iid_field(m, 30)
    d = net.flip_delta(p, m, s, 7, 3)
    s2 = s.copy()
    s2[2, 7] *= -1
    assert abs(d - (net.forward(p, m, s2)[0] - net.forward(p, m, s)[0])) < 1e-12 and abs(d) > 1e-6


def test_cumulative_update_with_learned_action_detailed_balance():
    """Exact 256-state transition matrix with S_theta = S_lin + S_net (2x2, L=2)."""
    import itertools
    import math
    from oracle import effective, stable
    m = Model(2, 2, 2, t=1.0, mu=-0.3, dtau=0.4, xi=1.2, n_stab=1)
    terms = [(1, 0), (0, 1)]
    lam = np.array([0.1, 0.25])
    p = net_init(9, scale=1.5)
    p[-9:-1] = np.random.default_rng(2).normal(scale=0.3, size=8)
    states = [np.array([(1 if (c >> b) & 1 else -1) for b in range(8)], np.int8).reshape(2, 4) for c in range(256)]
    w = np.array([stable.weight(m, s)[0] for s in states])
    sa = np.array([effective.action(m, terms, 0.0, lam, s) + net.forward(p, m, s)[0] for s in states])
    classes = effective.colour_classes(m, terms, 4)
    assert all(len(sites) == 1 for _, sites in classes)
    idx = {s.tobytes(): a for a, s in enumerate(states)}
    keff = np.zeros((256, 256))
    for a, s in enumerate(states):
        for l, sites in classes:
            i = sites[0]
            t = s.copy()
            t[l - 1, i] *= -1
            q = min(1.0, math.exp(effective.flip_delta(m, terms, lam, s, i, l) + net.flip_delta(p, m, s, i, l)))
            keff[a, idx[t.tobytes()]] += q / len(classes)
            keff[a, a] += (1 - q) / len(classes)
    flow = np.exp(sa - sa.max())[:, None] * keff
    assert np.max(np.abs(flow - flow.T)) < 1e-12
    prop = np.linalg.matrix_power(keff, 2)
    log_a = (w[None, :] - w[:, None]) - (sa[None, :] - sa[:, None])
    tm = prop * np.minimum(1.0, np.exp(log_a))
    np.fill_diagonal(tm, 0)
    np.fill_diagonal(tm, 1 - tm.sum(1))
    f2 = np.exp(w - w.max())[:, None] * tm
    assert np.max(np.abs(f2 - f2.T)) < 1e-12
    # the sampling code uses the same pieces: one step reproduces the matrix row support
    s0 = states[5].copy()
    effective.effective_sweep(m, terms, lam, s0, 2, seed=3, step=0, classes=classes, net_params=p)


def test_net_classes_separate_the_network_range():
    from oracle import effective
    m = Model(12, 11, 6)
    classes = effective.colour_classes(m, [(1, 0), (2, 0)], 4)
    for l, sites in classes:
        for a in sites:
            for b in sites:
                if a == b:
                    continue
                dx = min((a % 12 - b % 12) % 12, (b % 12 - a % 12) % 12)
                dy = min((a // 12 - b // 12) % 11, (b // 12 - a // 12) % 11)
                assert max(dx, dy) >= 5
