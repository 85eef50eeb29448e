"""Softmax over rows with masked (-inf) entries, the form attention scores
take: every legal plan of the forward and of the softmax-from-logits backward
against the FP64 oracle, FP32 and BF16 I/O (e4m3 has no infinity).  Masked
entries carry probability 0 and gradient 0.  The rows exercise what a mask
does to the statistics: slices of a split row, and whole threads, holding
nothing but -inf; a single finite entry; and a row whose largest finite
entry lies far below zero, so the output scale about the row maximum is
large while masked lanes contribute exactly nothing."""
import numpy as np
import pytest

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

from _cases import ALL_PLANS, check_tensor, from_device, to_device, ulp_bf16

pytestmark = pytest.mark.gpu
EPV = {"f32": 4, "bf16": 8}


def masked_rows(N: int, seed: int, epv: int) -> np.ndarray:
    """Eight rows of 4 N(0, 1) logits with masks; epv is the number of
    elements per 16-byte vector of the I/O format."""
    rng = np.random.default_rng([seed, N])
    x = I.softmax_rows(8, N, seed)
    x[0, rng.random(N) < 0.3] = -np.inf                   # scattered mask
    x[1, : (6 * N) // 10] = -np.inf                       # leading 60%: whole slices masked
    x[2, :] = -np.inf                                     # one finite entry: a one-hot output
    x[2, rng.integers(N)] = 1.5
    x[3] = -80.0 + rng.standard_normal(N)                 # row maximum far below zero, and
    x[3, : (6 * N) // 10] = -np.inf                       # whole slices masked
    x[4, :-1] = -np.inf                                   # only the last entry finite
    x[5, 1::2] = -np.inf                                  # every other entry
    x[6] = -80.0 + rng.standard_normal(N)                 # row maximum far below zero, and the
    x[6, (np.arange(N) // epv) % 256 < 128] = -np.inf     # vectors of threads 0-127 masked
    x[6, -1] = -80.0                                      # (short rows keep one finite entry)
    # row 7: no mask (control)
    return x


def plans(h, op, dt, M, N):
    o, d = {"fwd": (C.SOFTMAX, C.FWD), "smxl": (C.SOFTMAX_LOGITS, C.BWD)}[op]
    return [C.plan(v, k) for v, k in ALL_PLANS if h.plan_legal(o, d, C.DTYPE_NAMES[dt], M, N, C.plan(v, k))]


@pytest.mark.parametrize("N", [1000, 5003, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_masked_softmax_forward(gpu_handle, dtype, N):
    h = gpu_handle
    raw, _ = I.store(masked_rows(N, 31, EPV[dtype]), dtype)
    xv = oracle.decode(raw, dtype)
    ref = oracle.softmax_fwd(xv)
    assert np.all(np.isfinite(ref))
    x = to_device(raw, dtype)
    for p in plans(h, "fwd", dtype, 8, N):
        print(f"[masked] softmax fwd {dtype} N={N} {p}", flush=True)
        y, _ = C.softmax_fwd(x, p=p, h=h)
        got = from_device(y, dtype)
        try:
            check_tensor("y", "softmax_fwd", dtype, got, ref, np.abs(ref))
        except AssertionError as e:
            raise AssertionError(f"{p}: {e}") from None
        assert np.all(got[np.isneginf(xv)] == 0.0), f"{p}: masked entries not 0"
    assert h.check_errors() == C.OK


@pytest.mark.parametrize("N", [1000, 5003, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_masked_softmax_logits_backward(gpu_handle, dtype, N):
    h = gpu_handle
    raw, _ = I.store(masked_rows(N, 32, EPV[dtype]), dtype)
    draw, _ = I.store(I.normal_rows(8, N, 32, 1), dtype)
    xv, dyv = oracle.decode(raw, dtype), oracle.decode(draw, dtype)
    ref = oracle.softmax_logits_bwd(xv, dyv)
    assert np.all(np.isfinite(ref))
    y = oracle.softmax_fwd(xv)
    mag = y * (np.abs(dyv) + np.sum(y * np.abs(dyv), 1, keepdims=True))
    x, dy = to_device(raw, dtype), to_device(draw, dtype)
    for p in plans(h, "smxl", dtype, 8, N):
        print(f"[masked] softmax-logits bwd {dtype} N={N} {p}", flush=True)
        dx, _ = C.softmax_logits_bwd(x, dy, p=p, h=h)
        got = from_device(dx, dtype)
        assert np.all(np.isfinite(got)), f"{p}: non-finite gradient"
        if dtype == "f32":
            worst = float((np.abs(got - ref) / (1e-5 * mag + 1e-30)).max())
            assert worst <= 1.0, f"{p}: {worst:.3f} of the FP32 bound"
        else:
            allow = ulp_bf16(np.maximum(np.abs(ref), mag / 256.0))
            worst = float((np.abs(got - ref) / allow).max())
            assert worst <= 1.0, f"{p}: {worst:.3f} bf16 ulp"
        assert np.all(got[np.isneginf(xv)] == 0.0), f"{p}: masked entries have a gradient"
    assert h.check_errors() == C.OK


@pytest.mark.parametrize("N", [1000, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_fully_masked_row_is_nan_like_the_oracle(gpu_handle, dtype, N):
    # softmax of a row of -inf is 0/0: the oracle (and torch) give NaN; every
    # plan gives NaN on that row and leaves the neighbouring rows intact
    h = gpu_handle
    x64 = I.softmax_rows(3, N, 33)
    x64[1, :] = -np.inf
    raw, _ = I.store(x64, dtype)
    xv = oracle.decode(raw, dtype)
    with np.errstate(invalid="ignore"):
        ref = oracle.softmax_fwd(xv)
    assert np.all(np.isnan(ref[1])) and np.all(np.isfinite(ref[[0, 2]]))
    x = to_device(raw, dtype)
    for p in plans(h, "fwd", dtype, 3, N):
        print(f"[masked] fully masked row {dtype} N={N} {p}", flush=True)
        y, _ = C.softmax_fwd(x, p=p, h=h)
        got = from_device(y, dtype)
        assert np.all(np.isnan(got[1])), f"{p}: fully masked row not NaN"
        check_tensor("y", "softmax_fwd", dtype, got[[0, 2]], ref[[0, 2]], np.abs(ref[[0, 2]]))
    assert h.check_errors() == C.OK
