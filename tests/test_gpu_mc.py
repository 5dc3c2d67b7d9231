"""GPU parity of the Monte Carlo entry points against the oracle: local DQMC
sweeps, effective-model moves and features, cumulative updates and the fit.
The random numbers are the same Philox streams on both sides, so accept
decisions must agree one by one (a near-tie guard skips a case whose draw is
within 1e-9 of its threshold)."""
import numpy as np
import pytest
import torch

from oracle import stable, dqmc, effective, fit, philox
from slq_inputs import Model, SMALL_4x4, DQMC_20x20, iid_field, iid_fields, default_terms

pytestmark = pytest.mark.gpu

SEED = 0x5D0C


@pytest.fixture(scope="module")
def slq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_03804_amd import slq as mod
    mod.load_library()
    return mod


def _t(shape, dtype):
    return torch.empty(shape, dtype=dtype, device="cuda")


def run_gpu_sweeps(slq, model, fields, n_sweeps, sweep0=0, chain0=0):
    from tests.gpu_util import dev, host
    b = len(fields)
    plan = slq.Plan(model, b, sweeps=True)
    s = dev(np.stack(fields))
    G = _t((b, plan.n, plan.n), torch.float64)
    la = _t(b, torch.float64)
    sg = _t(b, torch.int8)
    slq.slq_green(plan, s, G, la, sg)
    acc = _t(b, torch.int64)
    drift = _t(b, torch.float64)
    st = _t(b, torch.int32)
    slq.slq_sweep_local(plan, s, G, la, sg, n_sweeps, SEED, sweep0, chain0, acc, drift, st)
    out = dict(s=host(s), G=host(G), la=host(la), sg=host(sg), acc=host(acc), drift=host(drift), st=host(st))
    plan.close()
    return out


def run_oracle_sweeps(model, field, n_sweeps, sweep0=0, chain=0):
    s = field.copy()
    la, sg, g = stable.green(model, s)
    acc_tot, drift, near = 0, 0.0, False
    for k in range(n_sweeps):
        la, sg, acc, d, tr = dqmc.sweep(model, s, g, la, sg, seed=SEED, sweep_index=sweep0 + k, chain=chain,
                                        want_trace=True)
        acc_tot += acc
        drift = max(drift, d)
        near |= any(abs(u - abs(r)) < 1e-9 for _, _, r, u, _ in tr)
    return dict(s=s, G=g, la=la, sg=sg, acc=acc_tot, drift=drift, near=near)


@pytest.mark.parametrize("model,n_sweeps", [
    (SMALL_4x4, 3),
    (Model(5, 3, 8, t=1.0, mu=-0.2, dtau=0.1, xi=1.3, n_stab=3), 2),     # N=15, L % n_stab != 0
    (Model(8, 8, 12, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=4), 1),    # N=64 > delayed-update depth
    (Model(9, 9, 14, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=4), 1),    # N=81: blocked QR, 3 stack entries
    (Model(22, 22, 4, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=4), 1),   # N=484: delay depth 16 (LDS tables)
    (Model(24, 24, 4, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=4), 1),   # N=576: the global-table flip kernel
])
def test_local_sweeps_match_oracle(slq, model, n_sweeps):
    fields = [iid_field(model, 7000 + i) for i in range(2)]
    got = run_gpu_sweeps(slq, model, fields, n_sweeps, sweep0=5, chain0=3)
    for b, f in enumerate(fields):
        ref = run_oracle_sweeps(model, f, n_sweeps, sweep0=5, chain=3 + b)
        if ref["near"]:
            pytest.skip("near-tie draw")
        assert got["st"][b] == 0
        assert np.array_equal(got["s"][b], ref["s"])
        assert got["acc"][b] == ref["acc"]
        assert got["sg"][b] == ref["sg"]
        assert abs(got["la"][b] - ref["la"]) < 1e-10 * max(1, abs(ref["la"]))
        assert np.max(np.abs(got["G"][b] - ref["G"])) < 1e-10
        assert got["drift"][b] < 1e-8 and abs(got["drift"][b] - ref["drift"]) < 1e-9
    # the tracked weight is the weight of the final field
    for b in range(2):
        la, sg = stable.weight(model, got["s"][b])
        assert sg == got["sg"][b] and abs(la - got["la"][b]) < 1e-10 * max(1, abs(la))


def test_local_sweep_20x20_full_size(slq):
    f = iid_field(DQMC_20x20, 7100)
    got = run_gpu_sweeps(slq, DQMC_20x20, [f], 1)
    ref = run_oracle_sweeps(DQMC_20x20, f, 1)
    if ref["near"]:
        pytest.skip("near-tie draw")
    assert np.array_equal(got["s"][0], ref["s"]) and got["acc"][0] == ref["acc"]
    assert abs(got["la"][0] - ref["la"]) < 1e-10 * abs(ref["la"])
    assert np.max(np.abs(got["G"][0] - ref["G"])) < 1e-10
    assert got["drift"][0] < 1e-8


def make_eff(slq, plan, model, terms, lam, c0=0.0):
    return slq.Eff(plan, terms, lam, c0)


def test_features_exact(slq):
    from tests.gpu_util import dev, host
    m = Model(6, 5, 10)
    terms = default_terms(10) + [(3, 0), (4, 1), (5, 2)]
    fields = iid_fields(m, 4, 8000)
    plan = slq.Plan(m, 4)
    eff = make_eff(slq, plan, m, terms, np.zeros(len(terms)))
    F = _t((4, len(terms)), torch.float64)
    slq.slq_eff_features(plan, eff, dev(fields), F)
    got = host(F)
    for b in range(4):
        assert np.array_equal(got[b], effective.features(m, terms, fields[b]))


@pytest.mark.parametrize("model", [Model(6, 6, 8), Model(5, 7, 6), Model(4, 4, 20)])
def test_effective_sweep_matches_oracle(slq, model):
    from tests.gpu_util import dev, host
    terms = default_terms(model.n_slices)
    lam = np.random.default_rng(3).normal(scale=0.2, size=len(terms))
    fields = iid_fields(model, 3, 8100)
    plan = slq.Plan(model, 3)
    eff = make_eff(slq, plan, model, terms, lam)
    classes = effective.colour_classes(model, terms)
    assert eff.n_classes == len(classes)
    s = dev(fields)
    acc = _t(3, torch.int64)
    dS = _t(3, torch.float64)
    slq.slq_eff_sweep(plan, eff, s, 40, SEED, 11, 2, acc, dS)
    got_s, got_acc, got_ds = host(s), host(acc), host(dS)
    for b in range(3):
        ref = fields[b].copy()
        a, d = effective.effective_sweep(model, terms, lam, ref, 40, seed=SEED, step=11, chain=2 + b,
                                         classes=classes)
        assert np.array_equal(got_s[b], ref) and got_acc[b] == a
        assert abs(got_ds[b] - d) < 1e-9 * max(1, abs(d))
        s_eff = effective.action(model, terms, 0.0, lam, ref) - effective.action(model, terms, 0.0, lam, fields[b])
        assert abs(s_eff - d) < 1e-9 * max(1, abs(d))


def test_cumulative_steps_match_oracle(slq):
    from tests.gpu_util import dev, host
    m = Model(4, 4, 8, t=1.0, mu=-0.3, dtau=0.1, xi=1.2, n_stab=4)
    terms = default_terms(8)
    train = iid_fields(m, 60, 8200)
    y = [stable.weight(m, f)[0] for f in train]
    c0, lam, r2 = fit.fit(m, terms, train, y)
    fields = iid_fields(m, 3, 8300)
    plan = slq.Plan(m, 3)
    eff = make_eff(slq, plan, m, terms, lam, c0)
    s = dev(fields)
    la = _t(3, torch.float64)
    sg = _t(3, torch.int8)
    slq.slq_weight(plan, s, la, sg)
    accd = _t(3, torch.int8)
    logA = _t(3, torch.float64)
    ref_s = [f.copy() for f in fields]
    ref_w = [stable.weight(m, f) for f in fields]
    classes = effective.colour_classes(m, terms)
    for step in range(6):
        slq.slq_cumulative_step(plan, eff, s, la, sg, 12, SEED, step, 0, accd, logA)
        ga, gl, gs, gla = host(accd), host(logA), host(s), host(la)
        for b in range(3):
            ref_s[b], lw, sgn, ok, la_ref = effective.cumulative_step(
                m, terms, c0, lam, ref_s[b], ref_w[b][0], ref_w[b][1], 12, lambda x: stable.weight(m, x),
                seed=SEED, step=step, chain=b, classes=classes)
            ref_w[b] = (lw, sgn)
            u = philox.uniform((0, 0, step, b), (SEED, philox.TAG_CUMULATIVE))
            if abs(np.log(u) - min(0.0, la_ref)) < 1e-8:
                pytest.skip("near-tie draw")
            assert bool(ga[b]) == ok and abs(gl[b] - la_ref) < 1e-9 * max(1.0, abs(la_ref))
            assert np.array_equal(gs[b], ref_s[b]) and abs(gla[b] - lw) < 1e-10 * max(1, abs(lw))


def test_fit_matches_oracle(slq):
    from tests.gpu_util import dev, host
    m = Model(4, 4, 8, t=1.0, mu=-0.3, dtau=0.1, xi=1.2, n_stab=4)
    terms = default_terms(8)
    fields = iid_fields(m, 120, 8400)
    plan = slq.Plan(m, 1)
    eff = make_eff(slq, plan, m, terms, np.zeros(len(terms)))
    # exactly linear target: recovery to round-off
    lam = np.random.default_rng(9).normal(size=len(terms))
    y = np.array([effective.action(m, terms, 1.25, lam, f) for f in fields])
    th = _t(1 + len(terms), torch.float64)
    r2 = _t(1, torch.float64)
    slq.slq_fit_effective(plan, eff, dev(fields), dev(y), th, r2)
    t = host(th)
    assert abs(t[0] - 1.25) < 1e-8 and np.max(np.abs(t[1:] - lam)) < 1e-9 and abs(host(r2)[0] - 1) < 1e-12
    # exact weights as the target: same coefficients and score as the oracle
    y = np.array([stable.weight(m, f)[0] for f in fields])
    slq.slq_fit_effective(plan, eff, dev(fields), dev(y), th, r2)
    c0, lref, r2ref = fit.fit(m, terms, fields, y)
    t = host(th)
    assert abs(t[0] - c0) < 1e-8 * max(1, abs(c0))
    assert np.max(np.abs(t[1:] - lref)) < 1e-8 * max(1.0, np.max(np.abs(lref)))
    assert abs(host(r2)[0] - r2ref) < 1e-10


def test_local_sweeps_4x4_100_sweeps(slq):
    """The 4x4, L=20 workload's 100 local-update sweeps on two chains: every
    accept decision is replayed by the oracle with the same Philox draws, so
    the final fields, accept counts, tracked weights and G agree."""
    fields = [iid_field(SMALL_4x4, 7300 + i) for i in range(2)]
    got = run_gpu_sweeps(slq, SMALL_4x4, fields, 100, sweep0=0, chain0=0)
    for b, f in enumerate(fields):
        ref = run_oracle_sweeps(SMALL_4x4, f, 100, sweep0=0, chain=b)
        if ref["near"]:
            pytest.skip("near-tie draw")
        assert got["st"][b] == 0
        assert np.array_equal(got["s"][b], ref["s"])
        assert got["acc"][b] == ref["acc"]
        assert got["sg"][b] == ref["sg"]
        assert abs(got["la"][b] - ref["la"]) < 1e-10 * max(1, abs(ref["la"]))
        assert np.max(np.abs(got["G"][b] - ref["G"])) < 1e-10
        assert got["drift"][b] < 1e-8
        la, sg = stable.weight(SMALL_4x4, got["s"][b])
        assert sg == got["sg"][b] and abs(la - got["la"][b]) < 1e-10 * max(1, abs(la))


def test_nonfinite_green_shows_in_drift(slq):
    """A NaN planted (from the host) in one off-diagonal entry of the incoming
    G.  With t = 0 the slice propagators are diagonal, so the NaN reaches only
    one column of the wrapped G, a few lanes of the drift reduction; the drift
    must still come out NaN and the chain be flagged non-finite."""
    from tests.gpu_util import dev, host
    m = Model(4, 4, 8, t=0.0, mu=-0.3, dtau=0.1, xi=1.2, n_stab=4)
    fields = iid_fields(m, 2, 7400)
    plan = slq.Plan(m, 2, sweeps=True)
    s = dev(fields)
    G = _t((2, 16, 16), torch.float64)
    la = _t(2, torch.float64)
    sg = _t(2, torch.int8)
    slq.slq_green(plan, s, G, la, sg)
    G[0, 0, 1] = float("nan")
    acc = _t(2, torch.int64)
    drift = _t(2, torch.float64)
    st = _t(2, torch.int32)
    slq.slq_sweep_local(plan, s, G, la, sg, 1, SEED, 0, 0, acc, drift, st)
    d, stat = host(drift), host(st)
    assert np.isnan(d[0]) and (stat[0] & slq.SLQ_ST_NONFINITE)
    assert np.isfinite(d[1]) and d[1] < 1e-8 and stat[1] == 0
    plan.close()


@pytest.mark.parametrize("model", [SMALL_4x4, Model(5, 3, 7), DQMC_20x20])
def test_magnetization_matches_sum(slq, model):
    from tests.gpu_util import dev, host
    b = 5
    fields = iid_fields(model, b, 7500)
    fields[1] = 1                      # fully ordered fields: the extreme values
    fields[2] = -1
    plan = slq.Plan(model, b)
    M = _t(b, torch.int64)
    slq.slq_magnetization(plan, dev(fields), M)
    np.testing.assert_array_equal(host(M), fields.reshape(b, -1).astype(np.int64).sum(axis=1))
    plan.close()


def _cumulative_parity(slq, m, terms, c0, lam, fields, n_moves, steps, step0=0, chain_prec=0, weight_fn=None):
    """Cumulative updates of len(fields) chains on the GPU, each checked
    decision by decision against the oracle (weight_fn: the oracle's exact
    weight of the plan's discretisation, stable.weight by default)."""
    wfn = weight_fn or (lambda x: stable.weight(m, x))
    from tests.gpu_util import dev, host
    nb = len(fields)
    plan = slq.Plan(m, nb, chain_prec)
    eff = make_eff(slq, plan, m, terms, lam, c0)
    s = dev(np.stack(fields))
    la = _t(nb, torch.float64)
    sg = _t(nb, torch.int8)
    st = _t(nb, torch.int32)
    slq.slq_weight(plan, s, la, sg, st)
    accd = _t(nb, torch.int8)
    logA = _t(nb, torch.float64)
    ref_s = [f.copy() for f in fields]
    ref_w = [wfn(f) for f in fields]
    gla0 = host(la)
    for b in range(nb):
        assert abs(gla0[b] - ref_w[b][0]) < 1e-10 * max(1, abs(ref_w[b][0]))
    classes = effective.colour_classes(m, terms)
    assert eff.n_classes == len(classes)
    n_acc = 0
    for step in range(step0, step0 + steps):
        slq.slq_cumulative_step(plan, eff, s, la, sg, n_moves, SEED, step, 0, accd, logA, st)
        ga, gl, gs, gla, gst = host(accd), host(logA), host(s), host(la), host(st)
        for b in range(nb):
            ref_s[b], lw, sgn, ok, la_ref = effective.cumulative_step(
                m, terms, c0, lam, ref_s[b], ref_w[b][0], ref_w[b][1], n_moves, wfn,
                seed=SEED, step=step, chain=b, classes=classes)
            ref_w[b] = (lw, sgn)
            u = philox.uniform((0, 0, step, b), (SEED, philox.TAG_CUMULATIVE))
            if abs(np.log(u) - min(0.0, la_ref)) < 1e-8:
                pytest.skip("near-tie draw")
            assert gst[b] == 0
            assert bool(ga[b]) == ok and abs(gl[b] - la_ref) < 1e-9 * max(1.0, abs(la_ref))
            assert np.array_equal(gs[b], ref_s[b]) and abs(gla[b] - lw) < 1e-10 * max(1, abs(lw))
            n_acc += int(ok)
    eff.close()
    plan.close()
    return n_acc


def test_cumulative_steps_20x20_full_size(slq):
    """The 20x20, L=80 workload: 4 chains x 3 cumulative updates of one full
    effective sweep each (n_classes class moves), with an effective model that
    the oracle fitted (Eq. 3) on 16 exact weights."""
    m = DQMC_20x20
    terms = [(0, 0), (1, 0), (2, 0), (0, 1), (0, 2), (0, 3), (1, 1), (2, 1)]
    train = iid_fields(m, 16, 7600)
    y = [stable.weight(m, f)[0] for f in train]
    c0, lam, _ = fit.fit(m, terms, train, y)
    fields = [iid_field(m, 7700 + b) for b in range(4)]
    n_classes = len(effective.colour_classes(m, terms))
    n_acc = _cumulative_parity(slq, m, terms, c0, lam, fields, n_classes, 3)
    assert n_acc > 0            # the fitted model makes acceptable proposals


def test_cumulative_step_48x48_full_size(slq):
    """The 48x48, L=100 workload (its 230 KB field exceeds the LDS as bytes, so
    the effective moves keep it there as bits, 28.8 KB): one chain, one
    cumulative update of N L = 230 400 single-flip proposals (n_classes class
    moves)."""
    from slq_inputs import LEARNED_48x48
    m = LEARNED_48x48
    terms = [(0, 0), (1, 0), (2, 0), (0, 1), (0, 2), (1, 1)]
    lam = np.array([-0.45, 0.01, 0.005, 0.02, 0.01, 0.004])
    n_classes = len(effective.colour_classes(m, terms))
    assert m.n_slices * m.n_sites > 150 * 1024
    _cumulative_parity(slq, m, terms, 0.0, lam, [iid_field(m, 7800)], n_classes, 1)


def test_cumulative_steps_bit_field_small_lattice(slq):
    """A small lattice with a long time axis (12x12, L = 1100: a 158 KB
    field, above the LDS budget as bytes) so that the move kernel keeps the
    field as bits where the oracle is cheap: 2 chains x 2 cumulative updates."""
    m = Model(12, 12, 1100, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10)
    terms = [(0, 0), (1, 0), (2, 0), (0, 1), (0, 2), (0, 7), (1, 1), (2, 3)]
    lam = np.array([-0.45, 0.01, 0.005, 0.02, 0.01, 0.003, 0.004, 0.002])
    assert m.n_slices * m.n_sites > 150 * 1024
    fields = [iid_field(m, 7900 + b) for b in range(2)]
    _cumulative_parity(slq, m, terms, 0.0, lam, fields, 60, 2)


def test_cumulative_steps_global_moves(slq):
    """A time axis beyond the LDS kernels' slice-offset encoding (4x4, L =
    4200) sends the effective moves to the kernel that reads the field from
    global memory: 2 chains x 2 cumulative updates of 80 class moves."""
    m = Model(4, 4, 4200, t=1.0, mu=-0.5, dtau=0.002, xi=1.5, n_stab=10)  # beta = 8.4
    terms = [(0, 0), (1, 0), (0, 1), (1, 1)]
    lam = np.array([-0.45, 0.01, 0.02, 0.004])
    assert m.n_slices > 4094
    fields = [iid_field(m, 7950 + b) for b in range(2)]
    _cumulative_parity(slq, m, terms, 0.0, lam, fields, 80, 2)
