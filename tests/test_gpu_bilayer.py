"""GPU parity of the paper's bilayer workload ("Results", Eq. 6) against the
oracle: the four-flavour weight phi [W_f(s) W_f(-s)]^2 and its two Green's
functions, local sweeps decision by decision (same Philox draws), and
cumulative updates judged by the bilayer weight.  Parameters of the paper's
finite-temperature critical point: beta = 1, dtau = 0.05 (L = 20), xi = 1,
h = 2.774, with J = 1, t = 1, mu = -0.5 (J, t, mu are not given)."""
import numpy as np
import pytest
import torch

from oracle import bilayer, effective, fit, philox
from slq_inputs import Model, iid_field, iid_fields, default_terms, BILAYER_J, BILAYER_H, bilayer_model

pytestmark = pytest.mark.gpu

SEED = 0x5D0C + 6


@pytest.fixture(scope="module")
def slq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_03804_amd import slq as mod
    mod.load_library()
    return mod


def _t(shape, dtype):
    return torch.empty(shape, dtype=dtype, device="cuda")


@pytest.mark.parametrize("model", [bilayer_model(4), bilayer_model(8), Model(5, 3, 12, mu=0.2, dtau=0.1, n_stab=5)])
def test_bilayer_weight_and_green_match_oracle(slq, model):
    from tests.gpu_util import dev, host
    b = 3
    fields = iid_fields(model, b, 9500)
    plan = slq.Plan(model, 2 * b)
    lw = _t(b, torch.float64)
    st = _t(b, torch.int32)
    G = _t((2 * b, model.n_sites, model.n_sites), torch.float64)
    slq.slq_bilayer_weight(plan, BILAYER_J, BILAYER_H, dev(fields), lw, st)
    w1 = host(lw)
    slq.slq_bilayer_green(plan, BILAYER_J, BILAYER_H, dev(fields), G, lw, st)
    Gh, w2, sth = host(G), host(lw), host(st)
    assert np.all(sth == 0)
    for k in range(b):
        ref = bilayer.log_weight(model, BILAYER_J, BILAYER_H, fields[k])
        assert abs(w1[k] - ref) < 1e-12 * abs(ref) and abs(w2[k] - ref) < 1e-12 * abs(ref)
        ga, gb = bilayer.green_pair(model, fields[k])
        assert np.max(np.abs(Gh[k] - ga)) < 1e-10 and np.max(np.abs(Gh[b + k] - gb)) < 1e-10
    plan.close()


@pytest.mark.parametrize("model,n_sweeps", [(bilayer_model(4), 3), (bilayer_model(8), 1),
                                            (Model(3, 4, 8, mu=-0.2, dtau=0.1, n_stab=3), 2)])
def test_bilayer_sweeps_match_oracle(slq, model, n_sweeps):
    from tests.gpu_util import dev, host
    b = 2
    fields = iid_fields(model, b, 9600)
    plan = slq.Plan(model, 2 * b)
    s = dev(fields)
    G = _t((2 * b, model.n_sites, model.n_sites), torch.float64)
    lw = _t(b, torch.float64)
    st = _t(b, torch.int32)
    slq.slq_bilayer_green(plan, BILAYER_J, BILAYER_H, s, G, lw, st)
    acc = _t(b, torch.int64)
    drift = _t(b, torch.float64)
    slq.slq_bilayer_sweep_local(plan, BILAYER_J, BILAYER_H, s, G, lw, n_sweeps, SEED, 2, 5, acc, drift, st)
    gs, gG, glw, gacc, gdr, gst = host(s), host(G), host(lw), host(acc), host(drift), host(st)
    for k in range(b):
        rs = fields[k].copy()
        ga, gb = bilayer.green_pair(model, rs)
        rlw = bilayer.log_weight(model, BILAYER_J, BILAYER_H, rs)
        racc, rdr = 0, 0.0
        for sw in range(n_sweeps):
            rlw, a, d, tr = bilayer.sweep(model, BILAYER_J, BILAYER_H, rs, ga, gb, rlw, seed=SEED, sweep_index=2 + sw,
                                          chain=5 + k, want_trace=True)
            racc += a
            rdr = max(rdr, d)
            if any(abs(u - r) < 1e-9 for _, _, r, u, _ in tr):
                pytest.skip("near-tie draw")
        assert gst[k] == 0
        assert np.array_equal(gs[k], rs) and gacc[k] == racc and 0 < racc
        assert abs(glw[k] - rlw) < 1e-10 * abs(rlw)
        assert np.max(np.abs(gG[k] - ga)) < 1e-10 and np.max(np.abs(gG[b + k] - gb)) < 1e-10
        assert gdr[k] < 1e-8 and abs(gdr[k] - rdr) < 1e-9
        assert abs(glw[k] - bilayer.log_weight(model, BILAYER_J, BILAYER_H, rs)) < 1e-9 * abs(rlw)
    plan.close()


def test_bilayer_cumulative_steps_match_oracle(slq):
    from tests.gpu_util import dev, host
    m = bilayer_model(4)
    terms = default_terms(m.n_slices)
    train = iid_fields(m, 40, 9700)
    y = [bilayer.log_weight(m, BILAYER_J, BILAYER_H, f) for f in train]
    c0, lam, _ = fit.fit(m, terms, train, y)
    b = 2
    fields = iid_fields(m, b, 9800)
    plan = slq.Plan(m, 2 * b)
    eff = slq.Eff(plan, terms, lam, c0)
    s = dev(fields)
    lw = _t(b, torch.float64)
    slq.slq_bilayer_weight(plan, BILAYER_J, BILAYER_H, s, lw)
    accd = _t(b, torch.int8)
    logA = _t(b, torch.float64)
    st = _t(b, torch.int32)
    classes = effective.colour_classes(m, terms)
    ref_s = [f.copy() for f in fields]
    ref_w = [bilayer.log_weight(m, BILAYER_J, BILAYER_H, f) for f in fields]
    n_ok = 0
    for step in range(4):
        slq.slq_bilayer_cumulative_step(plan, eff, BILAYER_J, BILAYER_H, s, lw, len(classes), SEED, step, 0, accd,
                                        logA, st)
        ga, gl, gs, glw, gst = host(accd), host(logA), host(s), host(lw), host(st)
        for k in range(b):
            ref_s[k], w, _, ok, la_ref = effective.cumulative_step(
                m, terms, c0, lam, ref_s[k], ref_w[k], 1, len(classes),
                lambda x: (bilayer.log_weight(m, BILAYER_J, BILAYER_H, x), 1), seed=SEED, step=step, chain=k,
                classes=classes)
            ref_w[k] = w
            u = philox.uniform((0, 0, step, k), (SEED, philox.TAG_CUMULATIVE))
            if abs(np.log(u) - min(0.0, la_ref)) < 1e-8:
                pytest.skip("near-tie draw")
            assert gst[k] == 0 and bool(ga[k]) == ok and abs(gl[k] - la_ref) < 1e-9 * max(1.0, abs(la_ref))
            assert np.array_equal(gs[k], ref_s[k]) and abs(glw[k] - w) < 1e-10 * abs(w)
            n_ok += int(ok)
    assert n_ok > 0
    eff.close()
    plan.close()


def test_bilayer_refuses_small_plans_and_bad_fields(slq):
    from tests.gpu_util import dev
    m = bilayer_model(4)
    plan = slq.Plan(m, 3)
    s = dev(iid_fields(m, 2, 9900))
    with pytest.raises(slq.SlqError):
        slq.slq_bilayer_weight(plan, BILAYER_J, BILAYER_H, s, _t(2, torch.float64))   # 2 * 2 > 3
    with pytest.raises(slq.SlqError):
        slq.slq_bilayer_weight(plan, BILAYER_J, 0.0, s[:1], _t(1, torch.float64))      # h must be > 0
    plan.close()
