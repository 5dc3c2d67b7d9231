"""GPU parity of the checkerboard chain mode (SLQ_PREC_CHECKERBOARD) against
the oracle's checkerboard discretisation (oracle/checkerboard.py): the dense
E_cb and its inverse, weight, sign and G, block widths, local sweeps and
cumulative updates, and the 48x48, L=100 workload."""
import numpy as np
import pytest
import torch

from oracle import checkerboard, dqmc, effective
from slq_inputs import Model, LEARNED_48x48, iid_field, mixed_batch

pytestmark = pytest.mark.gpu

LOG_TOL = 1e-12     # relative, log|W|
G_TOL = 1e-10       # absolute, max |dG|
SEED = 0x51D0


@pytest.fixture(scope="module")
def slq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_03804_amd import slq as mod
    mod.load_library()
    return mod


def _t(shape, dtype):
    return torch.empty(shape, dtype=dtype, device="cuda")


def e_pair(m):
    """E_cb and its inverse (the same split with dtau -> -dtau)."""
    return (checkerboard.propagator(m.lx, m.ly, m.t, m.mu, m.dtau),
            checkerboard.propagator(m.lx, m.ly, m.t, m.mu, -m.dtau))


@pytest.mark.parametrize("lx,ly", [(2, 2), (4, 4), (8, 4), (4, 2), (6, 4), (2, 6), (10, 6), (12, 8)])
def test_kinetic_is_the_checkerboard_propagator(slq, lx, ly):
    """P = 4 plaquettes (both sides multiples of 4), P = 2 otherwise; sides of
    2 hold the doubled bond, sides of one plaquette are their own neighbour."""
    from tests.gpu_util import host
    m = Model(lx, ly, 4, t=1.1, mu=-0.3, dtau=0.15)
    plan = slq.Plan(m, 1, slq.SLQ_PREC_CHECKERBOARD)
    e = _t((plan.n, plan.n), torch.float64)
    ei = torch.empty_like(e)
    slq.slq_kinetic(plan, False, e)
    slq.slq_kinetic(plan, True, ei)
    ref, ref_inv = e_pair(m)
    np.testing.assert_allclose(host(e), ref, rtol=0, atol=1e-14)
    np.testing.assert_allclose(host(ei), ref_inv, rtol=0, atol=1e-14)
    plan.close()


def test_odd_side_is_refused(slq):
    with pytest.raises(RuntimeError, match="even"):
        slq.Plan(Model(5, 4, 4), 1, slq.SLQ_PREC_CHECKERBOARD)


def gpu_green(slq, m, fields, width=0):
    from tests.gpu_util import dev, host
    b = len(fields)
    plan = slq.Plan(m, b, slq.SLQ_PREC_CHECKERBOARD)
    if width:
        slq.slq_plan_set_block_width(plan, width)
    s = dev(np.stack(fields).astype(np.int8))
    G = _t((b, plan.n, plan.n), torch.float64)
    la = _t(b, torch.float64)
    sg = _t(b, torch.int8)
    st = _t(b, torch.int32)
    slq.slq_green(plan, s, G, la, sg, st)
    la2 = _t(b, torch.float64)
    sg2 = _t(b, torch.int8)
    slq.slq_weight(plan, s, la2, sg2, st)
    out = host(G), host(la), host(sg), host(st), host(la2), host(sg2)
    plan.close()
    return out


@pytest.mark.parametrize("m", [
    Model(4, 4, 20, t=1.0, mu=0.0, dtau=0.1, xi=1.0, n_stab=10),
    Model(6, 4, 12, t=1.0, mu=-0.3, dtau=0.1, xi=1.3, n_stab=4),     # P = 2
    Model(2, 6, 9, t=1.2, mu=0.2, dtau=0.1, xi=1.1, n_stab=4),       # doubled x bond, L % n_stab != 0
    Model(10, 6, 12, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=5),    # N = 60, 15 plaquettes
    Model(12, 12, 20, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10),  # N = 144: blocked QR
])
def test_weight_and_green_match_the_oracle(slq, m):
    fields = list(mixed_batch(m, 3, 8100))
    G, la, sg, st, la2, sg2 = gpu_green(slq, m, fields)
    for b, s in enumerate(fields):
        ref_la, ref_sg, ref_G = checkerboard.green(m, s)
        assert st[b] == 0
        assert sg[b] == ref_sg and sg2[b] == ref_sg
        tol = LOG_TOL * max(1.0, abs(ref_la))
        assert abs(la[b] - ref_la) <= tol and abs(la2[b] - ref_la) <= tol, (b, la[b], la2[b], ref_la)
        assert np.max(np.abs(G[b] - ref_G)) <= G_TOL


def test_block_widths_give_identical_results(slq):
    """Every vector is computed by one thread per plaquette whatever the
    number of vectors per workgroup, so the results agree bit for bit."""
    m = Model(12, 8, 10, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=5)
    fields = [iid_field(m, 8200 + i) for i in range(2)]
    base = gpu_green(slq, m, fields, width=1)
    for w in (2, 4, 8, 16):
        got = gpu_green(slq, m, fields, width=w)
        for x, y in zip(base, got):
            assert np.array_equal(x, y), w


def test_tuned_width_is_admissible(slq):
    m = Model(16, 16, 20, n_stab=10)
    plan = slq.Plan(m, 4, slq.SLQ_PREC_CHECKERBOARD)
    w = slq.slq_plan_tune(plan, 4)
    assert w in (1, 2, 4, 8, 16)
    plan.close()


def test_local_sweeps_match_the_oracle(slq):
    from tests.gpu_util import dev, host
    m = Model(6, 4, 8, t=1.0, mu=-0.2, dtau=0.1, xi=1.3, n_stab=4)
    e, einv = e_pair(m)
    fields = [iid_field(m, 8300 + i) for i in range(2)]
    plan = slq.Plan(m, 2, slq.SLQ_PREC_CHECKERBOARD, sweeps=True)
    s = dev(np.stack(fields))
    G = _t((2, plan.n, plan.n), torch.float64)
    la = _t(2, torch.float64)
    sg = _t(2, torch.int8)
    slq.slq_green(plan, s, G, la, sg)
    acc = _t(2, torch.int64)
    drift = _t(2, torch.float64)
    st = _t(2, torch.int32)
    slq.slq_sweep_local(plan, s, G, la, sg, 2, SEED, 0, 0, acc, drift, st)
    gs, gG, gla, gsg, gacc, gst = host(s), host(G), host(la), host(sg), host(acc), host(st)
    plan.close()
    for b, f in enumerate(fields):
        rs = f.copy()
        rla, rsg, rg = checkerboard.green(m, rs)
        racc = 0
        for k in range(2):
            rla, rsg, a, _, tr = dqmc.sweep(m, rs, rg, rla, rsg, seed=SEED, sweep_index=k, chain=b,
                                            e=e, einv=einv, want_trace=True)
            racc += a
            if any(abs(u - abs(r)) < 1e-9 for _, _, r, u, _ in tr):
                pytest.skip("near-tie draw")
        assert gst[b] == 0
        assert np.array_equal(gs[b], rs) and gacc[b] == racc and gsg[b] == rsg
        assert abs(gla[b] - rla) < 1e-10 * max(1, abs(rla))
        assert np.max(np.abs(gG[b] - rg)) < 1e-10


def test_cumulative_steps_match_the_oracle(slq):
    from tests.test_gpu_mc import _cumulative_parity
    m = Model(8, 8, 20, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=5)
    terms = [(0, 0), (1, 0), (0, 1), (1, 1)]
    lam = np.array([-0.45, 0.01, 0.02, 0.004])
    fields = [iid_field(m, 8400 + b) for b in range(3)]
    n_classes = len(effective.colour_classes(m, terms))
    _cumulative_parity(slq, m, terms, 0.0, lam, fields, n_classes, 2,
                       chain_prec=slq.SLQ_PREC_CHECKERBOARD, weight_fn=lambda x: checkerboard.weight(m, x))


def test_48x48_full_size_weight(slq):
    """The 48x48, L=100 workload: E_cb entry by entry and the weight of one
    field against the oracle."""
    from tests.gpu_util import dev, host
    m = LEARNED_48x48
    plan = slq.Plan(m, 1, slq.SLQ_PREC_CHECKERBOARD)
    e = _t((plan.n, plan.n), torch.float64)
    slq.slq_kinetic(plan, False, e)
    ref_e = checkerboard.propagator(m.lx, m.ly, m.t, m.mu, m.dtau)
    np.testing.assert_allclose(host(e), ref_e, rtol=0, atol=1e-14)
    f = iid_field(m, 8500)
    s = dev(f[None])
    la = _t(1, torch.float64)
    sg = _t(1, torch.int8)
    st = _t(1, torch.int32)
    slq.slq_weight(plan, s, la, sg, st)
    ref_la, ref_sg = checkerboard.weight(m, f)
    assert host(st)[0] == 0 and host(sg)[0] == ref_sg
    assert abs(host(la)[0] - ref_la) <= LOG_TOL * abs(ref_la)
    plan.close()


def test_unaligned_fields_take_the_byte_path(slq):
    """Fields at an odd byte address are read spin by spin instead of as one
    word per plaquette row: the same results bit for bit."""
    from tests.gpu_util import dev, host
    m = Model(8, 8, 10, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=5)
    fields = np.stack([iid_field(m, 8600 + i) for i in range(2)])
    plan = slq.Plan(m, 2, slq.SLQ_PREC_CHECKERBOARD)
    flat = torch.zeros(fields.size + 1, dtype=torch.int8, device="cuda")
    odd = flat[1:].view(fields.shape)
    odd.copy_(dev(fields))
    assert odd.data_ptr() % 4 == 1
    out = []
    for s in (dev(fields), odd):
        G = _t((2, plan.n, plan.n), torch.float64)
        la = _t(2, torch.float64)
        sg = _t(2, torch.int8)
        st = _t(2, torch.int32)
        slq.slq_green(plan, s, G, la, sg, st)
        out.append((host(G), host(la), host(sg), host(st)))
    plan.close()
    for x, y in zip(*out):
        assert np.array_equal(x, y)
