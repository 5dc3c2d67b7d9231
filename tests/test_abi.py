"""The C ABI without a GPU: the library builds, loads and exports every entry
point declared in include/slq.h; host-side argument checks return the
documented codes before any device work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "slq.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(slq_\w+)\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1612_03804_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    from paper_1612_03804_amd import slq
    return slq.load_library()


def test_every_declared_symbol_is_exported(lib):
    from paper_1612_03804_amd import slq
    names = declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(slq.EXPORTS)


def test_version_and_error_strings(lib):
    assert b"gfx950" in lib.slq_version()
    assert isinstance(lib.slq_last_error(), bytes)


def test_argument_errors_before_device_work(lib):
    from paper_1612_03804_amd import slq
    h = C.c_void_p()
    assert lib.slq_plan_create(None, 4, 0, None, 0, C.byref(h)) == slq.SLQ_ERR_ARG
    bad = slq.slq_model(0, 4, 10, 5, 1.0, 0.0, 0.1, 1.0)
    assert lib.slq_plan_create(C.byref(bad), 4, 0, None, 0, C.byref(h)) == slq.SLQ_ERR_ARG
    assert b"lx" in lib.slq_last_error()
    bad = slq.slq_model(4, 4, 10, 5, 1.0, 0.0, -0.1, 1.0)
    assert lib.slq_plan_create(C.byref(bad), 4, 0, None, 0, C.byref(h)) == slq.SLQ_ERR_ARG
    bad = slq.slq_model(60, 60, 10, 5, 1.0, 0.0, 0.1, 1.0)
    assert lib.slq_plan_create(C.byref(bad), 4, 0, None, 0, C.byref(h)) == slq.SLQ_ERR_ARG
    good = slq.slq_model(4, 4, 10, 5, 1.0, 0.0, 0.1, 1.0)
    assert lib.slq_plan_create(C.byref(good), 0, 0, None, 0, C.byref(h)) == slq.SLQ_ERR_ARG
    assert lib.slq_plan_create(C.byref(good), 2, 4, None, 0, C.byref(h)) == slq.SLQ_ERR_ARG  # unknown flag
    assert lib.slq_weight(None, 1, None, None, None, None, None) == slq.SLQ_ERR_ARG
    assert lib.slq_green(None, 1, None, None, None, None, None, None) == slq.SLQ_ERR_ARG
    assert lib.slq_eff_create(None, 1, None, None, 0.0, None, 0, C.byref(h)) == slq.SLQ_ERR_ARG
    assert lib.slq_eff_workspace_size(None, 3, C.byref(C.c_size_t())) == slq.SLQ_ERR_ARG
    assert lib.slq_fit_effective(None, None, 10, None, None, None, None, None) == slq.SLQ_ERR_ARG


def test_no_device_is_reported(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1612_03804_amd import slq
    h = C.c_void_p()
    good = slq.slq_model(4, 4, 10, 5, 1.0, 0.0, 0.1, 1.0)
    assert lib.slq_plan_create(C.byref(good), 2, 0, None, 0, C.byref(h)) == slq.SLQ_ERR_DEVICE


def test_workspace_size_query(lib):
    """The size query is host-only (no device needed): the sweep and network
    sections add what the header states, rounded up to 256-byte blocks, and a
    caller workspace below the size is refused before any device call."""
    from paper_1612_03804_amd import slq
    from slq_inputs import DQMC_20x20, SMALL_4x4

    def size(m, b, flags):
        v = C.c_size_t()
        assert lib.slq_plan_workspace_size(C.byref(slq.slq_model.of(m)), b, flags, C.byref(v)) == slq.SLQ_OK
        return v.value

    def up(x):
        return (x + 255) // 256 * 256

    for m, b in ((SMALL_4x4, 3), (DQMC_20x20, 8)):
        n, L, ns = m.n_sites, m.n_slices, m.n_stab
        base = size(m, b, 0)
        assert base >= 6 * 8 * n * n * b      # chain products, factors and scratch
        stack = 8 * ((L - 1) // ns + 1) * b * (2 * n * n + n) + 4 * b
        assert size(m, b, slq.SLQ_PLAN_SWEEPS) - base == up(stack)
        assert size(m, b, slq.SLQ_PLAN_NET) - base >= 6 * 8 * L * n * b * 8
        both = size(m, b, slq.SLQ_PLAN_SWEEPS | slq.SLQ_PLAN_NET)
        assert both == size(m, b, slq.SLQ_PLAN_SWEEPS) + size(m, b, slq.SLQ_PLAN_NET) - base
        assert size(m, 2 * b, 0) > base
    h = C.c_void_p()
    m = slq.slq_model.of(SMALL_4x4)
    assert lib.slq_plan_create(C.byref(m), 3, 0, C.c_void_p(256), 16, C.byref(h)) == slq.SLQ_ERR_WORKSPACE
    v = C.c_size_t()
    assert lib.slq_plan_workspace_size(C.byref(m), 3, 8, C.byref(v)) == slq.SLQ_ERR_ARG


def test_binding_rejects_host_tensors(lib):
    import torch
    from paper_1612_03804_amd import slq
    with pytest.raises(slq.SlqError):
        slq._ptr(torch.zeros(3))


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.join(ROOT, "paper_1612_03804_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, re.M), f
                assert "oracle/" not in src, f
