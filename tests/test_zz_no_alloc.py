"""slq_weight_static (the entry point for callers that cannot allocate: its
workspace is a file-scope device array) against slq_weight on a plan, called
through the C ABI: two calls in a row, the second with a smaller input, each
equal to the plan's results to the parity bar (log|W| to 1e-12 relative,
signs and status exactly)."""
import ctypes as C

import numpy as np
import pytest
import torch

from slq_inputs import Model, SMALL_4x4, iid_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_03804_amd import slq as mod
    lib = mod.load_library()
    lib.slq_weight_static.argtypes = [C.POINTER(mod.slq_model), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]
    lib.slq_weight_static.restype = C.c_int
    return mod


def static_weight(slq, model, s):
    lib = slq.load_library()
    b = s.shape[0]
    la = torch.full((b,), -1.0, dtype=torch.float64, device="cuda")
    sg = torch.full((b,), 7, dtype=torch.int8, device="cuda")
    st = torch.full((b,), -1, dtype=torch.int32, device="cuda")
    m = slq.slq_model.of(model)
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.slq_weight_static(C.byref(m), b, C.c_void_p(s.data_ptr()), C.c_void_p(la.data_ptr()),
                               C.c_void_p(sg.data_ptr()), C.c_void_p(st.data_ptr()), stream)
    assert rc == slq.SLQ_OK, lib.slq_last_error()
    torch.cuda.synchronize()
    return la.cpu().numpy(), sg.cpu().numpy(), st.cpu().numpy()


def plan_weight(slq, model, s):
    b = s.shape[0]
    plan = slq.Plan(model, b)
    la = torch.empty(b, dtype=torch.float64, device="cuda")
    sg = torch.empty(b, dtype=torch.int8, device="cuda")
    st = torch.empty(b, dtype=torch.int32, device="cuda")
    slq.slq_weight(plan, s, la, sg, st)
    torch.cuda.synchronize()
    out = la.cpu().numpy(), sg.cpu().numpy(), st.cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("model,b1,b2", [
    (SMALL_4x4, 12, 5),                                                  # N = 16: LU of M
    (Model(10, 10, 40, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10), 6, 2),   # N = 100: blocked QR, QR of M
])
def test_static_weight_matches_plan_weight(slq, model, b1, b2):
    s1 = torch.from_numpy(iid_fields(model, b1, 9300)).cuda()
    s2 = torch.from_numpy(iid_fields(model, b2, 9400)).cuda()
    for s in (s1, s2):                    # the second call is smaller than the first
        la, sg, st = static_weight(slq, model, s)
        ref_la, ref_sg, ref_st = plan_weight(slq, model, s)
        assert np.array_equal(st, ref_st) and np.all(st == 0)
        assert np.array_equal(sg, ref_sg)
        assert np.all(np.abs(la - ref_la) <= 1e-12 * np.abs(ref_la))


def test_static_weight_refuses_what_does_not_fit(slq):
    lib = slq.load_library()
    big = Model(48, 48, 100, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=10)
    s = torch.ones((4, 1, 1), dtype=torch.int8, device="cuda")  # never read: the size check comes first
    m = slq.slq_model.of(big)
    rc = lib.slq_weight_static(C.byref(m), 4, C.c_void_p(s.data_ptr()), C.c_void_p(s.data_ptr()),
                               C.c_void_p(s.data_ptr()), None, None)
    assert rc == slq.SLQ_ERR_WORKSPACE and b"scratch" in lib.slq_last_error()
