"""Thin ctypes binding of libcredit (include/credit.h).

Argument marshalling only: torch provides device memory and the current HIP
stream; every step of every operator runs in the library's HIP kernels.  If
the shared library is missing the first call raises -- there is no fallback.

Tensor conventions: FP32 tensors are ``torch.float32``; BF16 tensors are
``torch.bfloat16``; FP8 tensors are ``torch.uint8`` (or
``torch.float8_e4m3fn``) OCP e4m3fn codes with one FP32 scale per row.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcredit.so")
# the learned selector's weights; CREDIT_MODEL_PATH overrides the installed file
MODEL_PATH = os.environ.get("CREDIT_MODEL_PATH") or os.path.join(_HERE, "models", "selector_gfx950.txt")

# enums (include/credit.h)
OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP, ERR_TIMEOUT, ERR_MODEL = range(7)
F32, BF16, FP8 = 0, 1, 2
SOFTMAX, LAYERNORM, RMSNORM = 0, 1, 2
SOFTMAX_LOGITS, QUANT_INT8, QUANT_FP8, PEARSON, WVAR, LAYERNORM_FP8_OUT = 3, 4, 5, 6, 7, 8
FWD, BWD = 0, 1
TWO_PASS, ROW_RESIDENT, SPLIT_ROW = 0, 1, 2
SEL_LEARNED, SEL_ANALYTIC, SEL_EXHAUSTIVE, SEL_FIXED, SEL_PEAK, SEL_LEARNED_TIMED = range(6)
OPT_SPIN_LIMIT, OPT_TEST_DROP_PUBLISH, OPT_MAX_GROUPS, OPT_TEST_SKEW, OPT_ROWS = range(5)
NUM_FEATURES, NUM_PLANS, MLP_HIDDEN = 12, 7, 64
DTYPE_NAMES = {"f32": F32, "bf16": BF16, "fp8": FP8}


class CreditError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}")


class Plan(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("k", ctypes.c_int32)]

    def __repr__(self):
        name = {TWO_PASS: "two_pass", ROW_RESIDENT: "resident", SPLIT_ROW: "split"}.get(self.variant, "?")
        return f"Plan({name}, k={self.k})"

    def as_tuple(self):
        return (int(self.variant), int(self.k))


class Workload(ctypes.Structure):
    _fields_ = [("b_base", ctypes.c_float), ("b_staged", ctypes.c_float), ("b_reread", ctypes.c_float),
                ("b_keep", ctypes.c_float), ("stages", ctypes.c_int32), ("q", ctypes.c_int32 * 4)]


class Timing(ctypes.Structure):
    _fields_ = [("median_us", ctypes.c_float), ("min_us", ctypes.c_float), ("p90_us", ctypes.c_float),
                ("mad_us", ctypes.c_float), ("runs", ctypes.c_int32)]


class Instance(ctypes.Structure):
    _fields_ = [("registers", ctypes.c_int32), ("private_bytes", ctypes.c_int32), ("per_cu", ctypes.c_int32),
                ("model_per_cu", ctypes.c_int32), ("coresident_per_cu", ctypes.c_int32)]


class Primitives(ctypes.Structure):
    _fields_ = [("clock_mhz", ctypes.c_float), ("lds_load_ns", ctypes.c_float), ("l2_load_ns", ctypes.c_float),
                ("handoff_same_xcd_ns", ctypes.c_float), ("handoff_cross_xcd_ns", ctypes.c_float),
                ("barrier_ns", ctypes.c_float), ("exchange_ns", ctypes.c_float * 5),
                ("lds_read_bpc", ctypes.c_float), ("lds_write_bpc", ctypes.c_float),
                ("l2_read_bpc", ctypes.c_float), ("global_write_bpc", ctypes.c_float),
                ("xcd_same", ctypes.c_int32 * 2), ("xcd_cross", ctypes.c_int32 * 2), ("errors", ctypes.c_int32)]

    def as_dict(self):
        d = {}
        for name, typ in self._fields_:
            v = getattr(self, name)
            conv = (lambda x: int(x)) if "int" in str(typ) else (lambda x: round(float(x), 3))
            d[name] = [conv(x) for x in v] if hasattr(v, "__len__") else conv(v)
        d["exchange_ns"] = dict(zip(["k2", "k4", "k8", "k16", "k32"], d["exchange_ns"]))
        return d


def plan(variant, k: int = 1) -> Plan:
    if isinstance(variant, str):
        variant = {"two_pass": TWO_PASS, "resident": ROW_RESIDENT, "split": SPLIT_ROW}[variant]
    return Plan(int(variant), int(k))


_lib = None
_lib_lock = threading.Lock()

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_F = ctypes.c_float
_S = ctypes.c_int
_SZ = ctypes.c_size_t
_PP = ctypes.POINTER(Plan)

_SIGS = {
    "credit_status_string": ([_S], ctypes.c_char_p),
    "credit_version": ([], ctypes.c_char_p),
    "credit_create": ([_S, ctypes.POINTER(_P)], _S),
    "credit_destroy": ([_P], _S),
    "credit_set_selector": ([_P, _S], _S),
    "credit_workspace_size": ([_P, _S, _S, _S, _I64, _I64, _PP, ctypes.POINTER(_SZ)], _S),
    "credit_plan_legal": ([_P, _S, _S, _S, _I64, _I64, _PP], _S),
    "credit_select": ([_P, _S, _S, _S, _I64, _I64, _PP, ctypes.POINTER(_F)], _S),
    "credit_softmax_fwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _I64, _P, _PP, _P, _SZ, _P], _S),
    "credit_softmax_bwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _I64, _P, _P, _I64, _P, _PP, _P, _SZ, _P], _S),
    "credit_layernorm_fwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _P, _F, _P, _I64, _P, _P, _P, _PP, _P, _SZ, _P], _S),
    "credit_layernorm_fwd_noalloc": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _P, _F, _P, _I64, _P, _P, _P, _PP,
                                      _P], _S),
    "credit_noalloc_scratch_bytes": ([], _SZ),
    "credit_layernorm_bwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _I64, _P, _P, _P, _P, _F, _P, _I64, _P, _P, _P,
                              _PP, _P, _SZ, _P], _S),
    "credit_rmsnorm_fwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _F, _P, _I64, _P, _P, _PP, _P, _SZ, _P], _S),
    "credit_rmsnorm_bwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _I64, _P, _P, _P, _F, _P, _I64, _P, _P, _PP, _P,
                            _SZ, _P], _S),
    "credit_softmax_logits_bwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _I64, _P, _P, _I64, _P, _PP, _P, _SZ, _P],
                                  _S),
    "credit_quantize_rows": ([_P, _S, _I64, _I64, _S, _P, _I64, _P, _I64, _P, _PP, _P, _SZ, _P], _S),
    "credit_pearson_bwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _I64, _P, _P, _I64, _P, _I64, _PP, _P, _SZ, _P], _S),
    "credit_wvar_bwd": ([_P, _I64, _I64, _S, _P, _I64, _P, _I64, _P, _P, _I64, _P, _I64, _PP, _P, _SZ, _P], _S),
    "credit_layernorm_fwd_fp8_out": ([_P, _I64, _I64, _S, _P, _I64, _P, _P, _F, _P, _I64, _P, _P, _P, _PP, _P, _SZ,
                                      _P], _S),
    "credit_encode": ([_P, _I64, _I64, _S, _P, _P, _P, _P], _S),
    "credit_decode": ([_P, _I64, _I64, _S, _P, _P, _P, _P], _S),
    "credit_check_errors": ([_P, _P], _S),
    "credit_time_plan": ([_P, _S, _S, _S, _I64, _I64, _PP, _S, _S, ctypes.POINTER(_F)], _S),
    "credit_time_plan_stats": ([_P, _S, _S, _S, _I64, _I64, _PP, _S, _S, ctypes.POINTER(Timing)], _S),
    "credit_time_control": ([_P, _S, _S, _S, _I64, _I64, _I32, _S, ctypes.POINTER(_F)], _S),
    "credit_copy_bandwidth": ([_P, _SZ, _S, ctypes.POINTER(_F)], _S),
    "credit_model_delta": ([_P, _S, _S, _S, _I64, _I64, _F, _P, _P], _S),
    "credit_workload_info": ([_S, _S, _S, _S, ctypes.POINTER(Workload)], _S),
    "credit_plan_of_class": ([_I32, _PP], _S),
    "credit_features": ([_S, _S, _S, _I64, _I64, _P], _S),
    "credit_mlp_num_params": ([], _I64),
    "credit_mlp_set": ([_P, _P, _P, _P], _S),
    "credit_mlp_get": ([_P, _P, _P, _P], _S),
    "credit_mlp_grad": ([_P, _P, _P, _P, _I64, ctypes.POINTER(_F), _P], _S),
    "credit_mlp_train": ([_P, _P, _P, _P, _I64, _S, _F, ctypes.c_uint64, ctypes.POINTER(_F)], _S),
    "credit_mlp_predict": ([_P, _P, _I64, _P], _S),
    "credit_save_model": ([_P, ctypes.c_char_p], _S),
    "credit_load_model": ([_P, ctypes.c_char_p], _S),
    "credit_set_option": ([_P, _S, _I64], _S),
    "credit_set_epoch": ([ctypes.c_uint32], _S),
    "credit_probe_primitives": ([_P, _S, ctypes.POINTER(Primitives)], _S),
    "credit_plan_geometry": ([_P, _S, _S, _S, _I64, _I64, _PP, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                              ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)], _S),
    "credit_instance_info": ([_P, _S, _S, _S, _I32, _I32, ctypes.POINTER(Instance)], _S),
}


def lib():
    """The loaded libcredit (ctypes.CDLL).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    f"{LIB_PATH} is missing: build it with `python -m paper_2609_01864_amd.build`")
            # torch's HIP runtime must be in the process before the library
            # binds to one: device pointers and streams come from torch
            import torch  # noqa: F401

            L = ctypes.CDLL(LIB_PATH)
            for name, (args, res) in _SIGS.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = res
            _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().credit_status_string(int(s)).decode()


def check(status: int, where: str) -> None:
    if status != OK:
        raise CreditError(status, where)


def version() -> str:
    return lib().credit_version().decode()


# ------------------------------------------------------------ host helpers
def workload_info(op: int, direction: int, dtype: int, recompute: bool = False) -> Workload:
    w = Workload()
    check(lib().credit_workload_info(op, direction, dtype, int(recompute), ctypes.byref(w)), "credit_workload_info")
    return w


def features(op: int, direction: int, dtype: int, M: int, N: int):
    import numpy as np

    f = np.zeros(NUM_FEATURES, np.float32)
    check(lib().credit_features(op, direction, dtype, M, N, f.ctypes.data), "credit_features")
    return f


def plan_of_class(c: int) -> Plan:
    p = Plan()
    check(lib().credit_plan_of_class(c, ctypes.byref(p)), "credit_plan_of_class")
    return p


def model_delta(handle, op, direction, dtype, M, N, t_base_us, t_ctrl_us):
    import numpy as np

    ctrl = np.ascontiguousarray(t_ctrl_us, np.float32).reshape(-1)
    if ctrl.size != 5:  # the library reads one value per k = 2, 4, 8, 16, 32
        raise ValueError(f"t_ctrl_us needs 5 entries (k = 2, 4, 8, 16, 32), got {ctrl.size}")
    out = np.zeros(5, np.float32)
    h = handle.ptr if handle is not None else None
    check(lib().credit_model_delta(h, op, direction, dtype, M, N, float(t_base_us), ctrl.ctypes.data,
                                   out.ctypes.data), "credit_model_delta")
    return out


def plan_geometry(handle, op, direction, dtype, M, N, p: Plan):
    g, b, v, o, r = _I32(), _I32(), _I32(), _I32(), _I32()
    h = handle.ptr if handle is not None else None
    s = lib().credit_plan_geometry(h, op, direction, dtype, M, N, ctypes.byref(p), ctypes.byref(g), ctypes.byref(b),
                                   ctypes.byref(v), ctypes.byref(o), ctypes.byref(r))
    if s == ERR_UNSUPPORTED:
        return None
    check(s, "credit_plan_geometry")
    return {"grid": g.value, "block": b.value, "vpt": v.value, "per_cu": o.value, "rows": r.value}


def instance_info(handle, op, direction, dtype, vpt: int, rows: int = 1):
    """Registers, private bytes per lane, workgroups per CU (occupancy query,
    register model, verified co-residency; -1 when not probed) of one
    row-resident / split-row instance (rows > 1: the multi-row norm forward),
    or None if it does not exist."""
    out = Instance()
    h = handle.ptr if handle is not None else None
    s = lib().credit_instance_info(h, op, direction, dtype, int(vpt), int(rows), ctypes.byref(out))
    if s == ERR_UNSUPPORTED:
        return None
    check(s, "credit_instance_info")
    return {f: getattr(out, f) for f, _ in Instance._fields_}


def set_epoch(e: int) -> None:
    check(lib().credit_set_epoch(ctypes.c_uint32(e)), "credit_set_epoch")


# ------------------------------------------------------------------ handle
def _mlp_arrays(feats, targets=None, mask=None):
    """Contiguous FP32 features [n, NUM_FEATURES] (and FP32 targets / uint8
    mask [n, NUM_PLANS]); the library reads exactly those sizes, so any other
    shape is refused here."""
    import numpy as np

    f = np.ascontiguousarray(feats, np.float32)
    if f.ndim != 2 or f.shape[1] != NUM_FEATURES:
        raise ValueError(f"features must be [n, {NUM_FEATURES}], got {f.shape}")
    out = [f]
    for a, dt, name in ((targets, np.float32, "targets"), (mask, np.uint8, "mask")):
        if a is None:
            continue
        a = np.ascontiguousarray(a, dt)
        if a.shape != (f.shape[0], NUM_PLANS):
            raise ValueError(f"{name} must be [{f.shape[0]}, {NUM_PLANS}], got {a.shape}")
        out.append(a)
    return out


def _torch():
    import torch

    return torch


def io_dtype(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.bfloat16:
        return BF16
    if t.dtype in (torch.uint8, getattr(torch, "float8_e4m3fn", torch.uint8)):
        return FP8
    raise TypeError(f"unsupported I/O dtype {t.dtype}")


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _ld(t) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("operands must be 2-D with unit inner stride")
    return t.stride(0)


def _validate(M, N, ref, mats=(), vecs=()):
    """Checks what the kernels will read and write before the launch: every
    matrix operand is [M, N] with unit inner stride, on the device of `ref`
    and in its I/O dtype (None entries skipped); every vector operand is FP32
    on that device with at least the given number of contiguous elements.
    The library sees raw pointers only, so a short vector would be read out
    of bounds on the GPU."""
    torch = _torch()
    for t, name in mats:
        if t is None:
            continue
        if tuple(t.shape) != (M, N) or t.dim() != 2 or t.stride(1) != 1:
            raise ValueError(f"{name}: expected [{M}, {N}] with unit inner stride, got {tuple(t.shape)}")
        if t.device != ref.device or t.dtype != ref.dtype:
            raise ValueError(f"{name}: expected {ref.dtype} on {ref.device}, got {t.dtype} on {t.device}")
    for t, n, name in vecs:
        if t is None:
            continue
        if t.dtype != torch.float32 or t.device != ref.device:
            raise ValueError(f"{name}: expected float32 on {ref.device}, got {t.dtype} on {t.device}")
        if t.numel() < n or (t.numel() > 1 and t.dim() == 1 and t.stride(0) != 1) or t.dim() > 1 and not t.is_contiguous():
            raise ValueError(f"{name}: expected at least {n} contiguous elements, got {tuple(t.shape)}")


class Handle:
    """A library handle bound to one HIP device, with per-stream workspaces."""

    def __init__(self, device: int = 0, load_default_model: bool = True):
        torch = _torch()
        self.device = int(device)
        p = _P()
        with torch.cuda.device(self.device):
            check(lib().credit_create(self.device, ctypes.byref(p)), "credit_create")
        self.ptr = p
        self._ws = {}
        # workspaces replaced by a larger one stay allocated until the handle
        # goes away: a launch recorded into a HIP graph keeps the raw address of
        # the workspace it was captured with, and replaying it must not write
        # into memory the caching allocator has handed to someone else
        self._retired = []
        self.model_loaded = False
        if load_default_model and os.path.exists(MODEL_PATH):
            self.model_loaded = lib().credit_load_model(self.ptr, MODEL_PATH.encode()) == OK

    def close(self):
        if self.ptr:
            lib().credit_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- configuration
    def set_selector(self, sel: int) -> None:
        check(lib().credit_set_selector(self.ptr, sel), "credit_set_selector")

    def set_option(self, opt: int, value: int) -> None:
        check(lib().credit_set_option(self.ptr, opt, int(value)), "credit_set_option")

    def load_model(self, path: str) -> int:
        s = lib().credit_load_model(self.ptr, path.encode())
        self.model_loaded = s == OK
        return s

    def save_model(self, path: str) -> None:
        check(lib().credit_save_model(self.ptr, path.encode()), "credit_save_model")

    def check_errors(self, stream=None) -> int:
        s = self._stream(stream)
        return lib().credit_check_errors(self.ptr, s)

    # -- plans
    def workspace_size(self, op, direction, dtype, M, N, p: Optional[Plan] = None) -> int:
        n = _SZ()
        check(lib().credit_workspace_size(self.ptr, op, direction, dtype, M, N, None if p is None else ctypes.byref(p),
                                          ctypes.byref(n)), "credit_workspace_size")
        return n.value

    def plan_legal(self, op, direction, dtype, M, N, p: Plan) -> bool:
        return lib().credit_plan_legal(self.ptr, op, direction, dtype, M, N, ctypes.byref(p)) == OK

    def select(self, op, direction, dtype, M, N) -> Tuple[Plan, float]:
        p = Plan()
        pred = _F()
        check(lib().credit_select(self.ptr, op, direction, dtype, M, N, ctypes.byref(p), ctypes.byref(pred)),
              "credit_select")
        return p, pred.value

    def geometry(self, op, direction, dtype, M, N, p: Plan):
        return plan_geometry(self, op, direction, dtype, M, N, p)

    # -- timing
    def time_plan(self, op, direction, dtype, M, N, p: Plan, reps: int = 15, flush: bool = True) -> float:
        t = _F()
        check(lib().credit_time_plan(self.ptr, op, direction, dtype, M, N, ctypes.byref(p), reps, int(flush),
                                     ctypes.byref(t)), "credit_time_plan")
        return t.value

    def time_plan_stats(self, op, direction, dtype, M, N, p: Plan, reps: int = 15, flush: bool = True) -> dict:
        """Median, minimum, 90th percentile and MAD (microseconds) of `reps` runs."""
        t = Timing()
        check(lib().credit_time_plan_stats(self.ptr, op, direction, dtype, M, N, ctypes.byref(p), reps, int(flush),
                                           ctypes.byref(t)), "credit_time_plan_stats")
        return {f: getattr(t, f) for f, _ in Timing._fields_}

    def time_control(self, op, direction, dtype, M, N, k: int, reps: int = 15) -> float:
        t = _F()
        check(lib().credit_time_control(self.ptr, op, direction, dtype, M, N, k, reps, ctypes.byref(t)),
              "credit_time_control")
        return t.value

    def probe_primitives(self, reps: int = 15) -> dict:
        """MI355X primitive costs (LDS, L2, workgroup handoffs, barrier,
        exchange rounds, per-CU rates); see credit_probe_primitives."""
        out = Primitives()
        check(lib().credit_probe_primitives(self.ptr, int(reps), ctypes.byref(out)), "credit_probe_primitives")
        return out.as_dict()

    def copy_bandwidth(self, nbytes: int = 1 << 30, reps: int = 15) -> float:
        g = _F()
        check(lib().credit_copy_bandwidth(self.ptr, nbytes, reps, ctypes.byref(g)), "credit_copy_bandwidth")
        return g.value

    # -- MLP selector
    def mlp_get(self):
        import numpy as np

        n = lib().credit_mlp_num_params()
        p = np.zeros(n, np.float32)
        mu = np.zeros(NUM_FEATURES, np.float32)
        sd = np.zeros(NUM_FEATURES, np.float32)
        check(lib().credit_mlp_get(self.ptr, p.ctypes.data, mu.ctypes.data, sd.ctypes.data), "credit_mlp_get")
        return p, mu, sd

    def mlp_set(self, params, mu, sd) -> None:
        import numpy as np

        p = np.ascontiguousarray(params, np.float32).reshape(-1)
        m = np.ascontiguousarray(mu, np.float32).reshape(-1)
        s = np.ascontiguousarray(sd, np.float32).reshape(-1)
        if p.size != lib().credit_mlp_num_params() or m.size != NUM_FEATURES or s.size != NUM_FEATURES:
            raise ValueError("mlp_set: wrong number of parameters or standardization entries")
        check(lib().credit_mlp_set(self.ptr, p.ctypes.data, m.ctypes.data, s.ctypes.data), "credit_mlp_set")

    def mlp_grad(self, feats, targets, mask):
        import numpy as np

        f, t, m = _mlp_arrays(feats, targets, mask)
        g = np.zeros(lib().credit_mlp_num_params(), np.float32)
        loss = _F()
        check(lib().credit_mlp_grad(self.ptr, f.ctypes.data, t.ctypes.data, m.ctypes.data, f.shape[0],
                                    ctypes.byref(loss), g.ctypes.data), "credit_mlp_grad")
        return loss.value, g

    def mlp_train(self, feats, targets, mask, epochs: int, lr: float = 1e-3, seed: int = 1) -> float:
        import numpy as np

        f, t, m = _mlp_arrays(feats, targets, mask)
        loss = _F()
        check(lib().credit_mlp_train(self.ptr, f.ctypes.data, t.ctypes.data, m.ctypes.data, f.shape[0], epochs,
                                     lr, seed, ctypes.byref(loss)), "credit_mlp_train")
        self.model_loaded = True
        return loss.value

    def mlp_predict(self, feats):
        import numpy as np

        (f,) = _mlp_arrays(feats)
        out = np.zeros((f.shape[0], NUM_PLANS), np.float32)
        check(lib().credit_mlp_predict(self.ptr, f.ctypes.data, f.shape[0], out.ctypes.data), "credit_mlp_predict")
        return out

    # -- internals
    def _stream(self, stream=None) -> int:
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)

    def workspace(self, nbytes: int, stream: int):
        """A zero-initialised workspace of at least nbytes for this stream."""
        torch = _torch()
        key = int(stream)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            # grow at least twofold, so the retired ones add up to less than
            # the live one
            n = max(nbytes, 1 << 16, 2 * ws.numel() if ws is not None else 0)
            if ws is not None:
                self._retired.append(ws)
            ws = torch.zeros(n, dtype=torch.uint8, device=f"cuda:{self.device}")
            self._ws[key] = ws
        return ws


_handles = {}


def handle(device: Optional[int] = None) -> Handle:
    """The process-wide handle of a device (created on first use)."""
    torch = _torch()
    d = torch.cuda.current_device() if device is None else int(device)
    h = _handles.get(d)
    if h is None:
        h = Handle(d)
        _handles[d] = h
    return h


def _empty_like_out(x, M, N):
    torch = _torch()
    return torch.empty((M, N), dtype=x.dtype, device=x.device)


def _launch(h: Handle, fn_name: str, op, direction, dtype, M, N, p, stream, build_args):
    ws_bytes = h.workspace_size(op, direction, dtype, M, N, p) if M > 0 else 0
    ws = h.workspace(ws_bytes, stream)
    args = build_args(ws.data_ptr(), ws.numel())
    check(getattr(lib(), fn_name)(*args), fn_name)


def _scale_out(x, M):
    torch = _torch()
    return torch.empty(M, dtype=torch.float32, device=x.device)


def softmax_fwd(x, x_scale=None, p: Optional[Plan] = None, out=None, out_scale=None, h: Optional[Handle] = None):
    """Row softmax.  Returns (y, y_scale); y_scale is None unless FP8."""
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(out, "out")], [(x_scale, M, "x_scale"), (out_scale, M, "out_scale")])
    y = out if out is not None else _empty_like_out(x, M, N)
    ys = out_scale if out_scale is not None else (_scale_out(x, M) if dt == FP8 else None)
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_softmax_fwd", SOFTMAX, FWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(x_scale), _ptr(y), _ld(y), _ptr(ys), pp, w, wn, s))
    return y, ys


def softmax_bwd(y, dy, y_scale=None, dy_scale=None, p: Optional[Plan] = None, out=None, h: Optional[Handle] = None):
    """dx = y * (dy - sum(dy * y)).  Returns (dx, dx_scale)."""
    h = h or handle(y.device.index)
    dt = io_dtype(y)
    M, N = y.shape
    _validate(M, N, y, [(dy, "dy"), (out, "out")], [(y_scale, M, "y_scale"), (dy_scale, M, "dy_scale")])
    dx = out if out is not None else _empty_like_out(y, M, N)
    dxs = _scale_out(y, M) if dt == FP8 else None
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_softmax_bwd", SOFTMAX, BWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(y), _ld(y), _ptr(y_scale), _ptr(dy), _ld(dy), _ptr(dy_scale),
                           _ptr(dx), _ld(dx), _ptr(dxs), pp, w, wn, s))
    return dx, dxs


def layernorm_fwd(x, gamma, beta, eps: float = 1e-5, x_scale=None, p: Optional[Plan] = None, out=None,
                  save_stats: bool = True, h: Optional[Handle] = None):
    """Returns (y, y_scale, mean, rstd)."""
    torch = _torch()
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(out, "out")], [(gamma, N, "gamma"), (beta, N, "beta"), (x_scale, M, "x_scale")])
    y = out if out is not None else _empty_like_out(x, M, N)
    ys = _scale_out(x, M) if dt == FP8 else None
    mean = torch.empty(M, dtype=torch.float32, device=x.device) if save_stats else None
    rstd = torch.empty(M, dtype=torch.float32, device=x.device) if save_stats else None
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_layernorm_fwd", LAYERNORM, FWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(x_scale), _ptr(gamma), _ptr(beta), float(eps),
                           _ptr(y), _ld(y), _ptr(ys), _ptr(mean), _ptr(rstd), pp, w, wn, s))
    return y, ys, mean, rstd


def layernorm_bwd(x, dy, gamma, mean=None, rstd=None, eps: float = 1e-5, x_scale=None, dy_scale=None,
                  p: Optional[Plan] = None, need_dgamma: bool = True, need_dbeta: bool = True,
                  h: Optional[Handle] = None):
    """Returns (dx, dx_scale, dgamma, dbeta); mean/rstd None -> recomputed."""
    torch = _torch()
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(dy, "dy")], [(gamma, N, "gamma"), (mean, M, "mean"), (rstd, M, "rstd"),
                                     (x_scale, M, "x_scale"), (dy_scale, M, "dy_scale")])
    dx = _empty_like_out(x, M, N)
    dxs = _scale_out(x, M) if dt == FP8 else None
    dg = torch.empty(N, dtype=torch.float32, device=x.device) if need_dgamma else None
    db = torch.empty(N, dtype=torch.float32, device=x.device) if need_dbeta else None
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_layernorm_bwd", LAYERNORM, BWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(x_scale), _ptr(dy), _ld(dy), _ptr(dy_scale),
                           _ptr(gamma), _ptr(mean), _ptr(rstd), float(eps), _ptr(dx), _ld(dx), _ptr(dxs),
                           _ptr(dg), _ptr(db), pp, w, wn, s))
    return dx, dxs, dg, db


def rmsnorm_fwd(x, gamma, eps: float = 1e-5, x_scale=None, p: Optional[Plan] = None, out=None,
                save_stats: bool = True, h: Optional[Handle] = None):
    """Returns (y, y_scale, rstd)."""
    torch = _torch()
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(out, "out")], [(gamma, N, "gamma"), (x_scale, M, "x_scale")])
    y = out if out is not None else _empty_like_out(x, M, N)
    ys = _scale_out(x, M) if dt == FP8 else None
    rstd = torch.empty(M, dtype=torch.float32, device=x.device) if save_stats else None
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_rmsnorm_fwd", RMSNORM, FWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(x_scale), _ptr(gamma), float(eps), _ptr(y),
                           _ld(y), _ptr(ys), _ptr(rstd), pp, w, wn, s))
    return y, ys, rstd


def rmsnorm_bwd(x, dy, gamma, rstd=None, eps: float = 1e-5, x_scale=None, dy_scale=None,
                p: Optional[Plan] = None, need_dgamma: bool = True, h: Optional[Handle] = None):
    """Returns (dx, dx_scale, dgamma); rstd None -> recomputed."""
    torch = _torch()
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(dy, "dy")], [(gamma, N, "gamma"), (rstd, M, "rstd"), (x_scale, M, "x_scale"),
                                     (dy_scale, M, "dy_scale")])
    dx = _empty_like_out(x, M, N)
    dxs = _scale_out(x, M) if dt == FP8 else None
    dg = torch.empty(N, dtype=torch.float32, device=x.device) if need_dgamma else None
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_rmsnorm_bwd", RMSNORM, BWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(x_scale), _ptr(dy), _ld(dy), _ptr(dy_scale),
                           _ptr(gamma), _ptr(rstd), float(eps), _ptr(dx), _ld(dx), _ptr(dxs), _ptr(dg), pp, w, wn,
                           s))
    return dx, dxs, dg


def softmax_logits_bwd(x, dy, x_scale=None, dy_scale=None, p: Optional[Plan] = None, out=None,
                       h: Optional[Handle] = None):
    """Softmax backward from the logits x: y = softmax(x) is rebuilt inside
    the row, dx = y * (dy - sum(dy * y)).  Returns (dx, dx_scale)."""
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(dy, "dy"), (out, "out")], [(x_scale, M, "x_scale"), (dy_scale, M, "dy_scale")])
    dx = out if out is not None else _empty_like_out(x, M, N)
    dxs = _scale_out(x, M) if dt == FP8 else None
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_softmax_logits_bwd", SOFTMAX_LOGITS, BWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(x_scale), _ptr(dy), _ld(dy), _ptr(dy_scale),
                           _ptr(dx), _ld(dx), _ptr(dxs), pp, w, wn, s))
    return dx, dxs


def _check_codes_out(out, M: int, N: int, fmt: str, device):
    """The code dtype of fmt; a caller-supplied codes tensor must be [M, N] of
    that dtype with unit inner stride on the input's device (its row stride is
    passed to the library in elements of one byte)."""
    torch = _torch()
    code_dt = torch.int8 if fmt == "int8" else torch.uint8
    if out is not None and (out.dim() != 2 or tuple(out.shape) != (M, N) or out.device != device
                            or out.dtype != code_dt or out.stride(1) != 1):
        raise ValueError(f"out: expected [{M}, {N}] {code_dt} codes with unit inner stride on {device}, "
                         f"got {tuple(out.shape)} {out.dtype} on {out.device}")
    return code_dt


def quantize_rows(x, fmt: str = "int8", p: Optional[Plan] = None, out=None, out_scale=None,
                  h: Optional[Handle] = None):
    """Row-wise quantisation of an FP32 / BF16 matrix.  fmt 'int8': codes
    torch.int8 in [-127, 127], scale = amax / 127; fmt 'fp8': e4m3 codes as
    torch.uint8, scale = amax / 448.  Returns (codes, scale)."""
    torch = _torch()
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    op = {"int8": QUANT_INT8, "fp8": QUANT_FP8}[fmt]
    M, N = x.shape
    _validate(M, N, x, [], [(out_scale, M, "out_scale")])
    code_dt = _check_codes_out(out, M, N, fmt, x.device)
    q = out if out is not None else torch.empty((M, N), dtype=code_dt, device=x.device)
    qs = out_scale if out_scale is not None else _scale_out(x, M)
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_quantize_rows", op, FWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, op, M, N, dt, _ptr(x), _ld(x), _ptr(q), _ld(q), _ptr(qs), pp, w, wn, s))
    return q, qs


def layernorm_fwd_fp8_out(x, gamma, beta, eps: float = 1e-5, p: Optional[Plan] = None, save_stats: bool = True,
                          h: Optional[Handle] = None):
    """LayerNorm forward of an FP32 / BF16 matrix fused with row-wise e4m3
    quantisation of y.  Returns (codes uint8, scale, mean, rstd)."""
    torch = _torch()
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [], [(gamma, N, "gamma"), (beta, N, "beta")])
    q = torch.empty((M, N), dtype=torch.uint8, device=x.device)
    qs = _scale_out(x, M)
    mean = torch.empty(M, dtype=torch.float32, device=x.device) if save_stats else None
    rstd = torch.empty(M, dtype=torch.float32, device=x.device) if save_stats else None
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_layernorm_fwd_fp8_out", LAYERNORM_FP8_OUT, FWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(gamma), _ptr(beta), float(eps), _ptr(q), _ld(q),
                           _ptr(qs), _ptr(mean), _ptr(rstd), pp, w, wn, s))
    return q, qs, mean, rstd


def pearson_bwd(x, y, dr, p: Optional[Plan] = None, h: Optional[Handle] = None):
    """Backward of the per-row Pearson correlation r(x, y) given dr [M].
    Returns (dx, dy)."""
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(y, "y")], [(dr, M, "dr")])
    gx, gy = _empty_like_out(x, M, N), _empty_like_out(x, M, N)
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_pearson_bwd", PEARSON, BWD, dt, M, N, p, s,
            lambda w, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(y), _ld(y), _ptr(dr), _ptr(gx), _ld(gx),
                           _ptr(gy), _ld(gy), pp, w, wn, s))
    return gx, gy


def wvar_bwd(x, w, dv, p: Optional[Plan] = None, h: Optional[Handle] = None):
    """Backward of the per-row weighted variance v(x, w) given dv [M].
    Returns (dx, dw)."""
    h = h or handle(x.device.index)
    dt = io_dtype(x)
    M, N = x.shape
    _validate(M, N, x, [(w, "w")], [(dv, M, "dv")])
    gx, gw = _empty_like_out(x, M, N), _empty_like_out(x, M, N)
    s = h._stream()
    pp = None if p is None else ctypes.byref(p)
    _launch(h, "credit_wvar_bwd", WVAR, BWD, dt, M, N, p, s,
            lambda ws, wn: (h.ptr, M, N, dt, _ptr(x), _ld(x), _ptr(w), _ld(w), _ptr(dv), _ptr(gx), _ld(gx),
                            _ptr(gw), _ld(gw), pp, ws, wn, s))
    return gx, gw


def encode(x, dtype: int, row_scale=None, h: Optional[Handle] = None):
    """FP32 [M, N] -> dtype codes (BF16 RNE; FP8 RNE, saturating, / row_scale)."""
    torch = _torch()
    h = h or handle(x.device.index)
    M, N = x.shape
    if x.dtype != torch.float32 or not x.is_contiguous():  # the codec reads M * N packed values
        raise ValueError("encode: x must be a contiguous float32 [M, N] tensor")
    _validate(M, N, x, [], [(row_scale, M, "row_scale")])
    tdt = {F32: torch.float32, BF16: torch.bfloat16, FP8: torch.uint8}[dtype]
    out = torch.empty((M, N), dtype=tdt, device=x.device)
    check(lib().credit_encode(h.ptr, M, N, dtype, _ptr(x), _ptr(row_scale), _ptr(out), h._stream()),
          "credit_encode")
    return out


def decode(codes, row_scale=None, h: Optional[Handle] = None):
    """dtype codes [M, N] -> FP32 values (x row_scale for FP8)."""
    torch = _torch()
    h = h or handle(codes.device.index)
    dt = io_dtype(codes)
    M, N = codes.shape
    if not codes.is_contiguous():  # the codec reads M * N packed codes
        raise ValueError("decode: codes must be a contiguous [M, N] tensor")
    _validate(M, N, codes, [], [(row_scale, M, "row_scale")])
    out = torch.empty((M, N), dtype=torch.float32, device=codes.device)
    check(lib().credit_decode(h.ptr, M, N, dt, _ptr(codes), _ptr(row_scale), _ptr(out), h._stream()),
          "credit_decode")
    return out
