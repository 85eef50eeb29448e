"""FP64 CPU oracle for the wide reduction-reuse row operators.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the CPU-baseline leg of ``bench.py``; never by the product package.  It
shares no code with the HIP path.  The arithmetic lives in ``credit_oracle.c``
(plain double-precision definitions, compiled with gcc); this module only
marshals numpy arrays and decodes the low-precision I/O formats exactly.

Operators (each is the plain definition; the method of the CREDIT paper reaches
it exactly up to rounding order, Sec. III-B, Eq. (1)):

* ``softmax_fwd``   y = exp(x - max x) / sum exp(x - max x)
* ``softmax_bwd``   dx = y * (dy - sum dy*y)
* ``layernorm_fwd`` y = (x - mean) * rstd * gamma + beta, biased variance
* ``layernorm_bwd`` dx, dgamma, dbeta with statistics recomputed in FP64
* ``rmsnorm_fwd`` / ``rmsnorm_bwd``
* codecs: bfloat16 and OCP FP8 e4m3fn, decode and round-to-nearest-even encode
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "credit_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


_NATIVE_PATH = os.path.join(_HERE, "liboracle_native.so")


def build(force: bool = False, native: bool = False) -> str:
    """Compile the oracle with gcc (-O2 -fopenmp, portable).  native=True builds
    the copy the CPU-baseline timing uses, -O3 -march=native, on the machine
    that runs it (never shipped between machines).  Both keep FP64 operations
    uncontracted (-ffp-contract=off), so their results are identical.
    Returns the library path."""
    path = _NATIVE_PATH if native else _LIB_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp%d" % os.getpid()
        opt = ["-O3", "-march=native"] if native else ["-O2"]
        subprocess.check_call(
            ["gcc", *opt, "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC,
             "-lm"]
        )
        os.replace(tmp, path)
    return path


def use_native() -> str:
    """Switches this process to the -O3 -march=native build (built here, now).
    For the CPU-baseline timing only; call before any other oracle function."""
    global _lib
    path = build(force=True, native=True)
    _lib = None
    _load(path)
    return path


def _load(path: str = None):
    global _lib
    if _lib is not None:
        return _lib
    if path is None:
        build()
        path = _LIB_PATH
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    sig = {
        "oracle_num_threads": ([], ctypes.c_int),
        "oracle_set_num_threads": ([ctypes.c_int], None),
        "oracle_sum": ([P, _I64], ctypes.c_double),
        "oracle_decode_bf16": ([P, P, _I64], None),
        "oracle_encode_bf16": ([P, P, _I64], None),
        "oracle_decode_e4m3": ([P, P, _I64], None),
        "oracle_encode_e4m3": ([P, P, _I64], None),
        "oracle_e4m3_step": ([ctypes.c_double], ctypes.c_double),
        "oracle_encode_bf16_f32": ([P, P, _I64], None),
        "oracle_encode_e4m3_f32": ([P, P, _I64], None),
        "oracle_softmax_fwd": ([_I64, _I64, P, P], None),
        "oracle_softmax_bwd": ([_I64, _I64, P, P, P], None),
        "oracle_layernorm_fwd": ([_I64, _I64, P, P, P, ctypes.c_double, P, P, P], None),
        "oracle_layernorm_bwd": ([_I64, _I64, P, P, P, ctypes.c_double, P, P, P, P], None),
        "oracle_rmsnorm_fwd": ([_I64, _I64, P, P, ctypes.c_double, P, P], None),
        "oracle_rmsnorm_bwd": ([_I64, _I64, P, P, P, ctypes.c_double, P, P, P], None),
        "oracle_softmax_logits_bwd": ([_I64, _I64, P, P, P], None),
        "oracle_quantize_rows": ([_I64, _I64, P, ctypes.c_int, P, P], None),
        "oracle_quantize_rows_fp32_product": ([_I64, _I64, P, ctypes.c_int, P], None),
        "oracle_pearson_bwd": ([_I64, _I64, P, P, P, P, P], None),
        "oracle_wvar_bwd": ([_I64, _I64, P, P, P, P, P], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _load().oracle_set_num_threads(int(n))


def fsum(v) -> float:
    """Neumaier-compensated sum of a 1-D array."""
    v = _f64(v).ravel()
    return _load().oracle_sum(_p(v), v.size)


# ------------------------------------------------------------------ codecs
def decode_bf16(bits) -> np.ndarray:
    b = np.ascontiguousarray(bits, dtype=np.uint16)
    out = np.empty(b.shape, np.float64)
    _load().oracle_decode_bf16(_p(b), _p(out), b.size)
    return out


def encode_bf16(v) -> np.ndarray:
    v = _f64(v)
    out = np.empty(v.shape, np.uint16)
    _load().oracle_encode_bf16(_p(v), _p(out), v.size)
    return out


def encode_from_f32(x32, fmt: str) -> np.ndarray:
    """RNE encode of binary32 values ('bf16': bit patterns as uint16; 'fp8':
    e4m3 codes saturating at +-448), the same definitions as encode_bf16 /
    encode_e4m3 applied to exact FP64 conversions of the inputs."""
    x = np.ascontiguousarray(x32, dtype=np.float32)
    out = np.empty(x.shape, np.uint16 if fmt == "bf16" else np.uint8)
    f = _load().oracle_encode_bf16_f32 if fmt == "bf16" else _load().oracle_encode_e4m3_f32
    f(_p(x), _p(out), x.size)
    return out


def decode_e4m3(codes) -> np.ndarray:
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    out = np.empty(c.shape, np.float64)
    _load().oracle_decode_e4m3(_p(c), _p(out), c.size)
    return out


def encode_e4m3(v) -> np.ndarray:
    v = _f64(v)
    out = np.empty(v.shape, np.uint8)
    _load().oracle_encode_e4m3(_p(v), _p(out), v.size)
    return out


def e4m3_step(v: float) -> float:
    return _load().oracle_e4m3_step(float(v))


def decode(raw, dtype: str, row_scale=None) -> np.ndarray:
    """Exact FP64 values of an I/O tensor.  dtype in {"f32", "bf16", "fp8"};
    FP8 codes are multiplied by their per-row FP32 scale (exact in FP64)."""
    if dtype == "f32":
        return np.asarray(raw, dtype=np.float32).astype(np.float64)
    if dtype == "bf16":
        return decode_bf16(np.asarray(raw).view(np.uint16))
    if dtype == "fp8":
        v = decode_e4m3(np.asarray(raw).view(np.uint8))
        s = np.asarray(row_scale, dtype=np.float32).astype(np.float64)
        return v * s.reshape(-1, 1)
    raise ValueError(dtype)


# ---------------------------------------------------------------- operators
def softmax_fwd(x) -> np.ndarray:
    x = _f64(x)
    M, N = x.shape
    y = np.empty_like(x)
    _load().oracle_softmax_fwd(M, N, _p(x), _p(y))
    return y


def softmax_bwd(y, dy) -> np.ndarray:
    y, dy = _f64(y), _f64(dy)
    M, N = y.shape
    dx = np.empty_like(y)
    _load().oracle_softmax_bwd(M, N, _p(y), _p(dy), _p(dx))
    return dx


def layernorm_fwd(x, gamma, beta, eps: float):
    """Returns (y, mean, rstd)."""
    x, g, b = _f64(x), _f64(gamma), _f64(beta)
    M, N = x.shape
    y = np.empty_like(x)
    mu = np.empty(M)
    rs = np.empty(M)
    _load().oracle_layernorm_fwd(M, N, _p(x), _p(g), _p(b), float(eps), _p(y), _p(mu), _p(rs))
    return y, mu, rs


def layernorm_bwd(x, dy, gamma, eps: float):
    """Returns (dx, dgamma, dbeta); statistics recomputed from x in FP64."""
    x, dy, g = _f64(x), _f64(dy), _f64(gamma)
    M, N = x.shape
    dx = np.empty_like(x)
    dg = np.empty(N)
    db = np.empty(N)
    ws = np.empty_like(x)
    _load().oracle_layernorm_bwd(M, N, _p(x), _p(dy), _p(g), float(eps), _p(dx), _p(dg), _p(db), _p(ws))
    return dx, dg, db


def rmsnorm_fwd(x, gamma, eps: float):
    """Returns (y, rstd)."""
    x, g = _f64(x), _f64(gamma)
    M, N = x.shape
    y = np.empty_like(x)
    rs = np.empty(M)
    _load().oracle_rmsnorm_fwd(M, N, _p(x), _p(g), float(eps), _p(y), _p(rs))
    return y, rs


def rmsnorm_bwd(x, dy, gamma, eps: float):
    """Returns (dx, dgamma); statistics recomputed from x in FP64."""
    x, dy, g = _f64(x), _f64(dy), _f64(gamma)
    M, N = x.shape
    dx = np.empty_like(x)
    dg = np.empty(N)
    ws = np.empty_like(x)
    _load().oracle_rmsnorm_bwd(M, N, _p(x), _p(dy), _p(g), float(eps), _p(dx), _p(dg), _p(ws))
    return dx, dg


def softmax_logits_bwd(x, dy) -> np.ndarray:
    """dx = y * (dy - sum(dy * y)) with y = softmax(x) (the softmax-logits workload)."""
    x, dy = _f64(x), _f64(dy)
    M, N = x.shape
    dx = np.empty_like(x)
    _load().oracle_softmax_logits_bwd(M, N, _p(x), _p(dy), _p(dx))
    return dx


def quantize_rows(x, fmt: str):
    """Row-wise quantisation of FP32-representable values (Sec. IV-A workload):
    codes = nearest grid point to x * Q / amax, ties to even, decided exactly
    (Q = 127 for 'int8', 448 for 'fp8'); scale = amax / Q rounded to FP32.
    Returns (int8 codes, FP32 scales) or (uint8 e4m3 codes, scales)."""
    x32 = _fp32_exact(x)
    M, N = x32.shape
    codes = np.empty((M, N), dtype=np.uint8)
    scale = np.empty(M, dtype=np.float32)
    _load().oracle_quantize_rows(M, N, _p(x32), 0 if fmt == "int8" else 1, _p(codes), _p(scale))
    return (codes.view(np.int8) if fmt == "int8" else codes), scale


def quantize_rows_fp32_product(x, fmt: str):
    """The codes an FP32 evaluation gives: v = x * fl32(Q / amax) rounded to
    FP32, then rounded to the grid.  Not the definition: used by the tests to
    show where it departs from it."""
    x32 = _fp32_exact(x)
    M, N = x32.shape
    codes = np.empty((M, N), dtype=np.uint8)
    _load().oracle_quantize_rows_fp32_product(M, N, _p(x32), 0 if fmt == "int8" else 1, _p(codes))
    return codes.view(np.int8) if fmt == "int8" else codes


def _fp32_exact(x):
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    if x32.astype(np.float64).tolist() != np.asarray(x, dtype=np.float64).tolist():
        raise ValueError("quantize_rows takes values exactly representable in FP32")
    return x32


def pearson_bwd(x, y, dr):
    """Backward of the per-row Pearson correlation; returns (dx, dy)."""
    x, y, dr = _f64(x), _f64(y), _f64(dr)
    M, N = x.shape
    gx, gy = np.empty_like(x), np.empty_like(x)
    _load().oracle_pearson_bwd(M, N, _p(x), _p(y), _p(dr), _p(gx), _p(gy))
    return gx, gy


def wvar_bwd(x, w, dv):
    """Backward of the per-row weighted variance; returns (dx, dw)."""
    x, w, dv = _f64(x), _f64(w), _f64(dv)
    M, N = x.shape
    gx, gw = np.empty_like(x), np.empty_like(x)
    _load().oracle_wvar_bwd(M, N, _p(x), _p(w), _p(dv), _p(gx), _p(gw))
    return gx, gw
