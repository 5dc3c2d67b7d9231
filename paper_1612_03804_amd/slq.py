"""ctypes binding of libslq (argument marshalling only).

Every function forwards to the C entry point of the same name in
include/slq.h; tensors are passed as raw device pointers together with the
current torch stream.  The library must have been built
(``python -m paper_1612_03804_amd.build``); loading fails loudly otherwise.
There is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libslq.so")

SLQ_OK, SLQ_ERR_ARG, SLQ_ERR_DEVICE, SLQ_ERR_WORKSPACE, SLQ_ERR_NUMERIC = 0, -1, -2, -3, -4
SLQ_ST_BAD_SPIN, SLQ_ST_NONFINITE, SLQ_ST_SINGULAR, SLQ_ST_PIVOT = 1, 2, 4, 8
SLQ_PLAN_SWEEPS, SLQ_PLAN_NET = 1, 2
SLQ_GROUP_EXACT_BATCHES = 1
SLQ_PREC_FP64, SLQ_PREC_FP32, SLQ_PREC_BF16, SLQ_PREC_FP64_DENSE, SLQ_PREC_CHECKERBOARD = 0, 1, 2, 3, 4

# every exported symbol of include/slq.h
EXPORTS = (
    "slq_version", "slq_last_error", "slq_plan_workspace_size", "slq_plan_create", "slq_plan_destroy",
    "slq_plan_bytes", "slq_kinetic", "slq_eff_workspace_size",
    "slq_profile_enable", "slq_profile_read", "slq_profile_read_part",
    "slq_weight", "slq_green", "slq_udv", "slq_sweep_local", "slq_eff_create", "slq_eff_destroy",
    "slq_eff_classes", "slq_eff_set_theta", "slq_eff_sweep", "slq_eff_features", "slq_cumulative_step",
    "slq_fit_effective", "slq_group_create", "slq_group_create_flags", "slq_group_batches", "slq_group_batch",
    "slq_group_cumulative_step", "slq_group_destroy", "slq_group_layout", "slq_group_describe",
    "slq_group_weight", "slq_group_green", "slq_magnetization", "slq_net_forward", "slq_net_gradient",
    "slq_net_adam", "slq_eff_set_net", "slq_eff_net_classes", "slq_plan_tune", "slq_plan_set_block_width",
    "slq_bilayer_weight", "slq_bilayer_green", "slq_bilayer_sweep_local", "slq_bilayer_cumulative_step",
    "slq_weight_static", "slq_measure_equal_time", "slq_green_displaced",
)
SLQ_NET_PARAMS = 1969


class SlqError(RuntimeError):
    pass


class slq_model(C.Structure):
    _fields_ = [("lx", C.c_int32), ("ly", C.c_int32), ("n_slices", C.c_int32), ("n_stab", C.c_int32),
                ("t", C.c_double), ("mu", C.c_double), ("dtau", C.c_double), ("xi", C.c_double),
                ("chain_prec", C.c_int32)]

    @classmethod
    def of(cls, m, chain_prec: int = 0) -> "slq_model":
        return cls(m.lx, m.ly, m.n_slices, m.n_stab, m.t, m.mu, m.dtau, m.xi, int(chain_prec))


class slq_bilayer(C.Structure):
    _fields_ = [("J", C.c_double), ("h", C.c_double)]


_lib = None
P = C.c_void_p


def load_library(path: str = LIB_PATH):
    """Load libslq.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise SlqError(f"{path} is missing: build it with `python -m paper_1612_03804_amd.build`")
    lib = C.CDLL(path)
    i32, u64, i64, dbl = C.c_int32, C.c_uint64, C.c_int64, C.c_double
    sig = {
        "slq_version": ([], C.c_char_p),
        "slq_last_error": ([], C.c_char_p),
        "slq_plan_workspace_size": ([C.POINTER(slq_model), i32, i32, C.POINTER(C.c_size_t)], C.c_int),
        "slq_plan_create": ([C.POINTER(slq_model), i32, i32, P, C.c_size_t, C.POINTER(P)], C.c_int),
        "slq_eff_workspace_size": ([P, i32, C.POINTER(C.c_size_t)], C.c_int),
        "slq_plan_destroy": ([P], C.c_int),
        "slq_plan_bytes": ([P, C.POINTER(C.c_size_t)], C.c_int),
        "slq_plan_tune": ([P, i32, C.POINTER(i32), P], C.c_int),
        "slq_plan_set_block_width": ([P, i32], C.c_int),
        "slq_kinetic": ([P, i32, P, P], C.c_int),
        "slq_profile_enable": ([P, i32], C.c_int),
        "slq_profile_read": ([P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)], C.c_int),
        "slq_profile_read_part": ([P, i32, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double)],
                                  C.c_int),
        "slq_weight": ([P, i32, P, P, P, P, P], C.c_int),
        "slq_green": ([P, i32, P, P, P, P, P, P], C.c_int),
        "slq_udv": ([P, i32, P, i32, P, P, P, P, P], C.c_int),
        "slq_sweep_local": ([P, i32, P, P, P, P, i32, u64, u64, u64, P, P, P, P], C.c_int),
        "slq_eff_create": ([P, i32, P, P, dbl, P, C.c_size_t, C.POINTER(P)], C.c_int),
        "slq_eff_destroy": ([P], C.c_int),
        "slq_eff_classes": ([P, C.POINTER(i32)], C.c_int),
        "slq_eff_set_theta": ([P, P, P], C.c_int),
        "slq_eff_sweep": ([P, P, i32, P, i32, u64, u64, u64, P, P, P], C.c_int),
        "slq_eff_features": ([P, P, i32, P, P, P], C.c_int),
        "slq_cumulative_step": ([P, P, i32, P, P, P, i32, u64, u64, u64, P, P, P, P], C.c_int),
        "slq_fit_effective": ([P, P, i64, P, P, P, P, P], C.c_int),
        "slq_group_create": ([P, i32, C.POINTER(P)], C.c_int),
        "slq_group_create_flags": ([P, i32, i32, C.POINTER(P)], C.c_int),
        "slq_group_batches": ([P, C.POINTER(i32)], C.c_int),
        "slq_group_batch": ([P, i32, C.POINTER(P), C.POINTER(i32), P], C.c_int),
        "slq_group_cumulative_step": ([P, P, i32, u64, u64, P, P, P, P, P, P, P], C.c_int),
        "slq_group_destroy": ([P], C.c_int),
        "slq_group_layout": ([P, P, P], C.c_int),
        "slq_group_describe": ([P, C.c_char_p, C.c_size_t], C.c_int),
        "slq_group_weight": ([P, P, P, P, P, P], C.c_int),
        "slq_group_green": ([P, P, P, P, P, P, P], C.c_int),
        "slq_magnetization": ([P, i32, P, P, P], C.c_int),
        "slq_net_forward": ([P, i32, i32, P, P, P, P], C.c_int),
        "slq_net_gradient": ([P, P, i32, i32, P, P, P, P, P, P], C.c_int),
        "slq_net_adam": ([i32, P, P, P, P, i64, dbl, dbl, dbl, dbl, P], C.c_int),
        "slq_eff_set_net": ([P, P, i32, P], C.c_int),
        "slq_eff_net_classes": ([P, C.POINTER(i32)], C.c_int),
        "slq_weight_static": ([C.POINTER(slq_model), i32, P, P, P, P, P], C.c_int),
        "slq_measure_equal_time": ([P, i32, P, P, P], C.c_int),
        "slq_green_displaced": ([P, i32, P, i32, P, P, P], C.c_int),
        "slq_bilayer_weight": ([P, C.POINTER(slq_bilayer), i32, P, P, P, P], C.c_int),
        "slq_bilayer_green": ([P, C.POINTER(slq_bilayer), i32, P, P, P, P, P], C.c_int),
        "slq_bilayer_sweep_local": ([P, C.POINTER(slq_bilayer), i32, P, P, P, i32, u64, u64, u64, P, P, P, P],
                                    C.c_int),
        "slq_bilayer_cumulative_step": ([P, P, C.POINTER(slq_bilayer), i32, P, P, i32, u64, u64, u64, P, P, P, P],
                                        C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != SLQ_OK:
        raise SlqError(f"libslq error {rc}: {load_library().slq_last_error().decode()}")


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise SlqError("libslq takes device tensors only")
    if not t.is_contiguous():
        raise SlqError("libslq takes contiguous tensors only")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _need(t, dtype, shape, name):
    if t.dtype != dtype or tuple(t.shape) != tuple(shape):
        raise SlqError(f"{name}: expected {dtype} {tuple(shape)}, got {t.dtype} {tuple(t.shape)}")


# ------------------------------------------------------------------ plan ----
def slq_plan_workspace_size(model, max_batch: int, chain_prec: int = 0, flags: int = 0) -> int:
    v = C.c_size_t()
    m = slq_model.of(model, chain_prec)
    _check(load_library().slq_plan_workspace_size(C.byref(m), int(max_batch), int(flags), C.byref(v)))
    return v.value


class Plan:
    """Owns an slq_plan (device workspace for one model and max_batch fields).

    sweeps / net add the sections of local sweeps and of the network calls.
    workspace: a caller-owned uint8 device tensor of at least
    slq_plan_workspace_size bytes (256-byte aligned), or None for a plan that
    allocates its own at creation."""

    def __init__(self, model, max_batch: int, chain_prec: int = 0, sweeps: bool = False, net: bool = False,
                 workspace=None):
        lib = load_library()
        self.model = model
        self.n = model.lx * model.ly
        self.L = model.n_slices
        self.max_batch = max_batch
        self.chain_prec = int(chain_prec)
        self.flags = (SLQ_PLAN_SWEEPS if sweeps else 0) | (SLQ_PLAN_NET if net else 0)
        self._m = slq_model.of(model, chain_prec)
        self.workspace = workspace   # kept alive as long as the plan
        ptr, nbytes = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
        h = C.c_void_p()
        _check(lib.slq_plan_create(C.byref(self._m), max_batch, self.flags, ptr, nbytes, C.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load_library().slq_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nbytes(self) -> int:
        v = C.c_size_t()
        _check(load_library().slq_plan_bytes(self.handle, C.byref(v)))
        return v.value


def slq_plan_create(model, max_batch: int, chain_prec: int = 0, sweeps: bool = False, net: bool = False,
                    workspace=None) -> Plan:
    return Plan(model, max_batch, chain_prec, sweeps, net, workspace)


def slq_plan_destroy(plan: Plan):
    plan.close()


def slq_kinetic(plan: Plan, inverse: bool, out, stream=None):
    _need(out, torch.float64, (plan.n, plan.n), "out")
    _check(load_library().slq_kinetic(plan.handle, int(bool(inverse)), _ptr(out), _stream(stream)))


def slq_magnetization(plan: Plan, s, M, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(M, torch.int64, (b,), "M")
    _check(load_library().slq_magnetization(plan.handle, b, _ptr(s), _ptr(M), _stream(stream)))


def slq_plan_tune(plan: Plan, batch: int, stream=None) -> int:
    """Pick the structured chain product's block width on `batch` fields;
    returns it (0 for plans with dense products).  Synchronous."""
    v = C.c_int32()
    _check(load_library().slq_plan_tune(plan.handle, int(batch), C.byref(v), _stream(stream)))
    return v.value


def slq_plan_set_block_width(plan: Plan, width: int):
    """Fix the structured chain product's block width (0: back to the default)."""
    _check(load_library().slq_plan_set_block_width(plan.handle, int(width)))


def slq_profile_enable(plan: Plan, enable: bool = True):
    _check(load_library().slq_profile_enable(plan.handle, int(bool(enable))))


SLQ_PROFILE_CHAIN, SLQ_PROFILE_STAB, SLQ_PROFILE_FINISH = 0, 1, 2


def slq_profile_read(plan: Plan, part: int = SLQ_PROFILE_CHAIN):
    """(summed ms, launch sequences, algorithmic flops) of one profiled part:
    chain products, stabilisations or the final step."""
    ms, n, fl = C.c_double(), C.c_int64(), C.c_double()
    _check(load_library().slq_profile_read_part(plan.handle, int(part), C.byref(ms), C.byref(n), C.byref(fl)))
    return ms.value, n.value, fl.value


def slq_weight(plan: Plan, s, logabs, sign, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(logabs, torch.float64, (b,), "logabs")
    _need(sign, torch.int8, (b,), "sign")
    if status is not None:
        _need(status, torch.int32, (b,), "status")
    _check(load_library().slq_weight(plan.handle, b, _ptr(s), _ptr(logabs), _ptr(sign), _ptr(status),
                                      _stream(stream)))


def slq_green(plan: Plan, s, G, logabs, sign, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(G, torch.float64, (b, plan.n, plan.n), "G")
    _need(logabs, torch.float64, (b,), "logabs")
    _need(sign, torch.int8, (b,), "sign")
    if status is not None:
        _need(status, torch.int32, (b,), "status")
    _check(load_library().slq_green(plan.handle, b, _ptr(s), _ptr(G), _ptr(logabs), _ptr(sign), _ptr(status),
                                     _stream(stream)))


def slq_udv(plan: Plan, s, slice0: int, U, D, V, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(U, torch.float64, (b, plan.n, plan.n), "U")
    _need(D, torch.float64, (b, plan.n), "D")
    _need(V, torch.float64, (b, plan.n, plan.n), "V")
    _check(load_library().slq_udv(plan.handle, b, _ptr(s), int(slice0), _ptr(U), _ptr(D), _ptr(V), _ptr(status),
                                   _stream(stream)))


def slq_sweep_local(plan: Plan, s, G, logabs, sign, n_sweeps: int, seed: int, sweep0: int, chain0: int,
                    accepts, drift, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(G, torch.float64, (b, plan.n, plan.n), "G")
    _need(accepts, torch.int64, (b,), "accepts")
    _need(drift, torch.float64, (b,), "drift")
    _check(load_library().slq_sweep_local(plan.handle, b, _ptr(s), _ptr(G), _ptr(logabs), _ptr(sign),
                                           int(n_sweeps), seed, sweep0, chain0, _ptr(accepts), _ptr(drift),
                                           _ptr(status), _stream(stream)))


# ------------------------------------------------------- effective model ----
class Eff:
    """Owns an slq_eff (terms, couplings and colour classes on the device)."""

    def __init__(self, plan: Plan, terms, lam, c0: float = 0.0, workspace=None):
        import numpy as np
        lib = load_library()
        self.plan = plan
        self.terms = [tuple(int(v) for v in t) for t in terms]
        t = np.ascontiguousarray(np.array(self.terms, dtype=np.int32).reshape(-1, 2))
        lm = np.ascontiguousarray(np.asarray(lam, dtype=np.float64).reshape(-1))
        if len(lm) != len(self.terms):
            raise SlqError("lambda must have one entry per term")
        self.workspace = workspace
        ptr, nbytes = (None, 0) if workspace is None else (_ptr(workspace), workspace.numel() * workspace.element_size())
        h = C.c_void_p()
        _check(lib.slq_eff_create(plan.handle, len(self.terms), t.ctypes.data_as(C.c_void_p),
                                  lm.ctypes.data_as(C.c_void_p), float(c0), ptr, nbytes, C.byref(h)))
        self.handle = h
        self.n_terms = len(self.terms)

    @property
    def n_classes(self) -> int:
        v = C.c_int32()
        _check(load_library().slq_eff_classes(self.handle, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "handle", None):
            load_library().slq_eff_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def slq_eff_workspace_size(plan: Plan, n_terms: int) -> int:
    v = C.c_size_t()
    _check(load_library().slq_eff_workspace_size(plan.handle, int(n_terms), C.byref(v)))
    return v.value


def slq_eff_create(plan: Plan, terms, lam, c0: float = 0.0, workspace=None) -> Eff:
    return Eff(plan, terms, lam, c0, workspace)


def slq_eff_destroy(eff: Eff):
    eff.close()


def slq_eff_set_theta(eff: Eff, theta, stream=None):
    _need(theta, torch.float64, (1 + eff.n_terms,), "theta")
    _check(load_library().slq_eff_set_theta(eff.handle, _ptr(theta), _stream(stream)))


def slq_eff_sweep(plan: Plan, eff: Eff, s, n_moves: int, seed: int, step: int, chain0: int,
                  accepts=None, dS=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _check(load_library().slq_eff_sweep(plan.handle, eff.handle, b, _ptr(s), int(n_moves), seed, step, chain0,
                                         _ptr(accepts), _ptr(dS), _stream(stream)))


def slq_eff_features(plan: Plan, eff: Eff, s, F, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(F, torch.float64, (b, eff.n_terms), "F")
    _check(load_library().slq_eff_features(plan.handle, eff.handle, b, _ptr(s), _ptr(F), _stream(stream)))


def slq_cumulative_step(plan: Plan, eff: Eff, s, logabs, sign, n_moves: int, seed: int, step: int, chain0: int,
                        accepted=None, logA=None, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(logabs, torch.float64, (b,), "logabs")
    _need(sign, torch.int8, (b,), "sign")
    _check(load_library().slq_cumulative_step(plan.handle, eff.handle, b, _ptr(s), _ptr(logabs), _ptr(sign),
                                               int(n_moves), seed, step, chain0, _ptr(accepted), _ptr(logA),
                                               _ptr(status), _stream(stream)))


def slq_fit_effective(plan: Plan, eff: Eff, S, logabs, theta, r2, stream=None):
    n = S.shape[0]
    _need(S, torch.int8, (n, plan.L, plan.n), "S")
    _need(logabs, torch.float64, (n,), "logabs")
    _need(theta, torch.float64, (1 + eff.n_terms,), "theta")
    _need(r2, torch.float64, (1,), "r2")
    _check(load_library().slq_fit_effective(plan.handle, eff.handle, n, _ptr(S), _ptr(logabs), _ptr(theta),
                                             _ptr(r2), _stream(stream)))


# ------------------------------------------------------------------ group ----
class _BatchPlan:
    """A group batch's internal plan (owned by the group), usable wherever a
    Plan is (slq.Eff, slq_fit_effective)."""

    def __init__(self, handle, model, n_chains):
        self.handle = handle
        self.model = model
        self.n = model.lx * model.ly
        self.L = model.n_slices
        self.max_batch = n_chains


class Group:
    """Owns an slq_group: chains of uneven (N, L), one graph launch per evaluation.
    exact_batches: only identical models share a batch (needed by
    slq_group_cumulative_step)."""

    def __init__(self, models, chain_prec: int = 0, exact_batches: bool = False):
        import numpy as np
        lib = load_library()
        self.models = list(models)
        arr = (slq_model * len(self.models))(*[slq_model.of(m, chain_prec) for m in self.models])
        h = C.c_void_p()
        _check(lib.slq_group_create_flags(arr, len(self.models), SLQ_GROUP_EXACT_BATCHES if exact_batches else 0,
                                          C.byref(h)))
        self.handle = h
        n = len(self.models)
        so = np.zeros(n + 1, dtype=np.int64)
        go = np.zeros(n + 1, dtype=np.int64)
        _check(lib.slq_group_layout(h, so.ctypes.data_as(C.c_void_p), go.ctypes.data_as(C.c_void_p)))
        self.s_off, self.g_off = so, go

    def describe(self) -> dict:
        import json
        buf = C.create_string_buffer(1 << 16)
        _check(load_library().slq_group_describe(self.handle, buf, len(buf)))
        return json.loads(buf.value.decode())

    @property
    def n_batches(self) -> int:
        v = C.c_int32()
        _check(load_library().slq_group_batches(self.handle, C.byref(v)))
        return v.value

    def batch(self, k: int):
        """(plan of batch k, chain indices of its positions)."""
        import numpy as np
        h = C.c_void_p()
        n = C.c_int32()
        _check(load_library().slq_group_batch(self.handle, int(k), C.byref(h), C.byref(n), None))
        ids = np.zeros(n.value, dtype=np.int32)
        _check(load_library().slq_group_batch(self.handle, int(k), C.byref(h), C.byref(n),
                                              ids.ctypes.data_as(C.c_void_p)))
        return _BatchPlan(h, self.models[int(ids[0])], n.value), ids

    def pack(self, fields):
        """Pack per-chain int8 [L_c][N_c] arrays into the group's layout (host)."""
        import numpy as np
        out = np.empty(int(self.s_off[-1]), dtype=np.int8)
        for c, f in enumerate(fields):
            out[self.s_off[c]:self.s_off[c + 1]] = np.asarray(f, dtype=np.int8).reshape(-1)
        return out

    def close(self):
        if getattr(self, "handle", None):
            load_library().slq_group_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def slq_group_weight(group: Group, s, logabs, sign, status=None, stream=None):
    n = len(group.models)
    _need(s, torch.int8, (int(group.s_off[-1]),), "s")
    _need(logabs, torch.float64, (n,), "logabs")
    _need(sign, torch.int8, (n,), "sign")
    _check(load_library().slq_group_weight(group.handle, _ptr(s), _ptr(logabs), _ptr(sign), _ptr(status),
                                            _stream(stream)))


def slq_group_cumulative_step(group: Group, effs, eff_sweeps: int, seed: int, step: int, s, logabs, sign,
                              accepted=None, logA=None, status=None, stream=None):
    n = len(group.models)
    _need(s, torch.int8, (int(group.s_off[-1]),), "s")
    _need(logabs, torch.float64, (n,), "logabs")
    _need(sign, torch.int8, (n,), "sign")
    if len(effs) != group.n_batches:
        raise SlqError("one effective model per batch is required")
    arr = (C.c_void_p * len(effs))(*[e.handle for e in effs])
    _check(load_library().slq_group_cumulative_step(group.handle, arr, int(eff_sweeps), int(seed), int(step),
                                                     _ptr(s), _ptr(logabs), _ptr(sign), _ptr(accepted), _ptr(logA),
                                                     _ptr(status), _stream(stream)))


def slq_group_green(group: Group, s, G, logabs, sign, status=None, stream=None):
    n = len(group.models)
    _need(s, torch.int8, (int(group.s_off[-1]),), "s")
    _need(G, torch.float64, (int(group.g_off[-1]),), "G")
    _need(logabs, torch.float64, (n,), "logabs")
    _need(sign, torch.int8, (n,), "sign")
    _check(load_library().slq_group_green(group.handle, _ptr(s), _ptr(G), _ptr(logabs), _ptr(sign), _ptr(status),
                                           _stream(stream)))


# -------------------------------------------------------- learned action ----
def slq_net_forward(plan: Plan, net_prec: int, s, params, S, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(params, torch.float64, (SLQ_NET_PARAMS,), "params")
    _need(S, torch.float64, (b,), "S")
    _check(load_library().slq_net_forward(plan.handle, int(net_prec), b, _ptr(s), _ptr(params), _ptr(S),
                                           _stream(stream)))


def slq_net_gradient(plan: Plan, eff: Eff, net_prec: int, s, y, params, grad, loss=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(y, torch.float64, (b,), "y")
    _need(params, torch.float64, (SLQ_NET_PARAMS,), "params")
    _need(grad, torch.float64, (SLQ_NET_PARAMS,), "grad")
    _check(load_library().slq_net_gradient(plan.handle, eff.handle, int(net_prec), b, _ptr(s), _ptr(y),
                                            _ptr(params), _ptr(grad), _ptr(loss), _stream(stream)))


def slq_net_adam(params, grad, m, v, t: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    n = params.numel()
    _check(load_library().slq_net_adam(n, _ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(t), float(lr),
                                        float(beta1), float(beta2), float(eps), _stream(stream)))


def slq_eff_set_net(eff: Eff, params, net_prec: int = SLQ_PREC_FP32, stream=None):
    if params is not None:
        _need(params, torch.float64, (SLQ_NET_PARAMS,), "params")
    _check(load_library().slq_eff_set_net(eff.handle, _ptr(params), int(net_prec), _stream(stream)))


def slq_eff_net_classes(eff: Eff) -> int:
    v = C.c_int32()
    _check(load_library().slq_eff_net_classes(eff.handle, C.byref(v)))
    return v.value


# ------------------------------------------------------ bilayer workload ----
def _bl(J: float, h: float):
    return C.byref(slq_bilayer(float(J), float(h)))


def slq_bilayer_weight(plan: Plan, J: float, h: float, s, logw, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(logw, torch.float64, (b,), "logw")
    _check(load_library().slq_bilayer_weight(plan.handle, _bl(J, h), b, _ptr(s), _ptr(logw), _ptr(status),
                                             _stream(stream)))


def slq_bilayer_green(plan: Plan, J: float, h: float, s, G, logw, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(G, torch.float64, (2 * b, plan.n, plan.n), "G")
    _need(logw, torch.float64, (b,), "logw")
    _check(load_library().slq_bilayer_green(plan.handle, _bl(J, h), b, _ptr(s), _ptr(G), _ptr(logw), _ptr(status),
                                            _stream(stream)))


def slq_bilayer_sweep_local(plan: Plan, J: float, h: float, s, G, logw, n_sweeps: int, seed: int, sweep0: int,
                            chain0: int, accepts=None, drift=None, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(G, torch.float64, (2 * b, plan.n, plan.n), "G")
    _need(logw, torch.float64, (b,), "logw")
    _check(load_library().slq_bilayer_sweep_local(plan.handle, _bl(J, h), b, _ptr(s), _ptr(G), _ptr(logw),
                                                  int(n_sweeps), seed, sweep0, chain0, _ptr(accepts), _ptr(drift),
                                                  _ptr(status), _stream(stream)))


def slq_bilayer_cumulative_step(plan: Plan, eff: Eff, J: float, h: float, s, logw, n_moves: int, seed: int,
                                step: int, chain0: int, accepted=None, logA=None, status=None, stream=None):
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(logw, torch.float64, (b,), "logw")
    _check(load_library().slq_bilayer_cumulative_step(plan.handle, eff.handle, _bl(J, h), b, _ptr(s), _ptr(logw),
                                                      int(n_moves), seed, step, chain0, _ptr(accepted), _ptr(logA),
                                                      _ptr(status), _stream(stream)))


def slq_measure_equal_time(plan: Plan, G, out, stream=None):
    """out [batch][3] = (density, hopping energy per site, S(pi, pi)) of each G."""
    b = G.shape[0]
    _need(G, torch.float64, (b, plan.n, plan.n), "G")
    _need(out, torch.float64, (b, 3), "out")
    _check(load_library().slq_measure_equal_time(plan.handle, b, _ptr(G), _ptr(out), _stream(stream)))


def slq_green_displaced(plan: Plan, s, slice: int, Gt, status=None, stream=None):
    """Gt [batch][N][N] = G(tau_slice, 0) = B_slice ... B_1 G of each field."""
    b = s.shape[0]
    _need(s, torch.int8, (b, plan.L, plan.n), "s")
    _need(Gt, torch.float64, (b, plan.n, plan.n), "Gt")
    _check(load_library().slq_green_displaced(plan.handle, b, _ptr(s), int(slice), _ptr(Gt), _ptr(status),
                                              _stream(stream)))
