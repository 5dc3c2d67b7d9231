"""GPU equal-time measurements (slq_measure_equal_time on the GPU's G)
against the oracle's Wick contractions of the oracle's G."""
import numpy as np
import pytest
import torch

from oracle import measure, stable
from slq_inputs import Model, SMALL_4x4, DQMC_20x20, iid_fields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slq():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_03804_amd import slq as mod
    mod.load_library()
    return mod


@pytest.mark.parametrize("model", [SMALL_4x4, Model(5, 3, 12, mu=-0.3, xi=1.2, n_stab=4),
                                   Model(2, 6, 10, mu=0.2, xi=1.0, n_stab=5), DQMC_20x20])
def test_equal_time_observables_match_oracle(slq, model):
    from tests.gpu_util import dev, host
    b = 3
    fields = iid_fields(model, b, 9950)
    plan = slq.Plan(model, b)
    G = torch.empty((b, model.n_sites, model.n_sites), dtype=torch.float64, device="cuda")
    la = torch.empty(b, dtype=torch.float64, device="cuda")
    sg = torch.empty(b, dtype=torch.int8, device="cuda")
    slq.slq_green(plan, dev(fields), G, la, sg)
    out = torch.empty((b, 3), dtype=torch.float64, device="cuda")
    slq.slq_measure_equal_time(plan, G, out)
    got = host(out)
    for k in range(b):
        _, _, g = stable.green(model, fields[k])
        np.testing.assert_allclose(got[k], measure.equal_time(model, g), rtol=1e-10, atol=1e-10)
    plan.close()


@pytest.mark.parametrize("model,slices", [
    (SMALL_4x4, (1, 7, 10, 13, 20)),
    (Model(6, 6, 20, t=1.0, mu=-0.5, dtau=0.1, xi=1.5, n_stab=5), (3, 5, 12, 19)),
    (Model(5, 3, 12, mu=-0.3, xi=1.2, n_stab=4, dtau=0.15), (6, 12)),
])
def test_displaced_green_matches_oracle(slq, model, slices):
    """G(tau_l, 0) = B_l ... B_1 G against the oracle's plain product
    (beta <= 2, where the plain product is accurate), across stabilisation
    blocks."""
    from tests.gpu_util import dev, host
    b = 2
    fields = iid_fields(model, b, 9960)
    plan = slq.Plan(model, b)
    Gt = torch.empty((b, model.n_sites, model.n_sites), dtype=torch.float64, device="cuda")
    st = torch.empty(b, dtype=torch.int32, device="cuda")
    for l in slices:
        slq.slq_green_displaced(plan, dev(fields), l, Gt, st)
        got = host(Gt)
        assert np.all(host(st) == 0)
        for k in range(b):
            ref = measure.green_displaced(model, fields[k], l)
            assert np.max(np.abs(got[k] - ref)) < 1e-9, (l, k)
    plan.close()
