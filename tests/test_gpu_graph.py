"""Local sweeps and cumulative updates recorded into a HIP graph (through
torch.cuda.graph, i.e. stream capture of the library's launches) and replayed:
every replay, with eager library work and host synchronisation between the
replays, reproduces the eager call on the same inputs bit for bit.  Both calls
run on caller-owned workspaces (plan and effective model created on device
memory that the test allocates), so nothing inside them allocates."""
import numpy as np
import pytest
import torch

from slq_inputs import Model, iid_fields, default_terms

pytestmark = pytest.mark.gpu

SEED = 0x5D0C


@pytest.fixture(scope="module")
def slq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_03804_amd import slq as mod
    mod.load_library()
    return mod


def _aligned(nbytes):
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    off = (-t.data_ptr()) % 256
    return t[off:off + nbytes]


def test_captured_sweeps_and_cumulative_steps_replay_exactly(slq):
    m = Model(6, 6, 20, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=5)
    b = 3
    flags = slq.SLQ_PLAN_SWEEPS
    ws = _aligned(slq.slq_plan_workspace_size(m, b, flags=flags))
    plan = slq.Plan(m, b, sweeps=True, workspace=ws)
    terms = default_terms(m.n_slices)
    lam = np.random.default_rng(5).normal(scale=0.05, size=len(terms))
    lam[0] = -0.4
    ews = _aligned(slq.slq_eff_workspace_size(plan, len(terms)))
    eff = slq.Eff(plan, terms, lam, 0.0, workspace=ews)
    f64, i8, i32, i64 = torch.float64, torch.int8, torch.int32, torch.int64
    s0 = torch.from_numpy(iid_fields(m, b, 9100)).cuda()
    N = m.n_sites
    G0 = torch.empty((b, N, N), dtype=f64, device="cuda")
    la0 = torch.empty(b, dtype=f64, device="cuda")
    sg0 = torch.empty(b, dtype=i8, device="cuda")
    st = torch.empty(b, dtype=i32, device="cuda")
    slq.slq_green(plan, s0, G0, la0, sg0, st)
    torch.cuda.synchronize()

    # state the captured calls update in place, and their other outputs
    s, G = s0.clone(), G0.clone()
    la, sg = la0.clone(), sg0.clone()
    acc = torch.empty(b, dtype=i64, device="cuda")
    drift = torch.empty(b, dtype=f64, device="cuda")
    cacc = torch.empty(b, dtype=i8, device="cuda")
    logA = torch.empty(b, dtype=f64, device="cuda")

    def step():
        slq.slq_sweep_local(plan, s, G, la, sg, 1, SEED, 4, 0, acc, drift, st)
        slq.slq_cumulative_step(plan, eff, s, la, sg, eff.n_classes, SEED, 6, 0, cacc, logA, st)

    def restore():
        s.copy_(s0)
        G.copy_(G0)
        la.copy_(la0)
        sg.copy_(sg0)

    def snapshot():
        torch.cuda.synchronize()
        return [t.clone() for t in (s, G, la, sg, acc, drift, cacc, logA, st)]

    # eager reference (also sets the kernels' launch attributes before capture)
    restore()
    step()
    ref = snapshot()
    assert int(ref[-1].abs().max()) == 0 and int(ref[4].sum()) > 0

    g = torch.cuda.CUDAGraph()
    restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    other = torch.empty((1, N, N), dtype=f64, device="cuda")
    for rep in range(3):
        restore()
        for t in (acc, drift, logA):
            t.fill_(-7)
        g.replay()
        got = snapshot()
        for a, r in zip(got, ref):
            assert torch.equal(a, r), rep
        # eager library work and synchronisation between replays
        slq.slq_green(plan, s0[:1], other, la[:1].clone(), sg[:1].clone(), st[:1])
        torch.cuda.synchronize()
    del g
    eff.close()
    plan.close()


def test_undersized_workspace_is_refused(slq):
    m = Model(4, 4, 8, n_stab=4)
    need = slq.slq_plan_workspace_size(m, 2)
    with pytest.raises(slq.SlqError):
        slq.Plan(m, 2, workspace=_aligned(need - 256))
    plan = slq.Plan(m, 2, workspace=_aligned(need))
    # local sweeps need the section the plan was created without
    s = torch.from_numpy(iid_fields(m, 2, 9200)).cuda()
    G = torch.empty((2, 16, 16), dtype=torch.float64, device="cuda")
    la = torch.empty(2, dtype=torch.float64, device="cuda")
    sg = torch.empty(2, dtype=torch.int8, device="cuda")
    slq.slq_green(plan, s, G, la, sg)
    acc = torch.empty(2, dtype=torch.int64, device="cuda")
    drift = torch.empty(2, dtype=torch.float64, device="cuda")
    with pytest.raises(slq.SlqError):
        slq.slq_sweep_local(plan, s, G, la, sg, 1, SEED, 0, 0, acc, drift)
    plan.close()
