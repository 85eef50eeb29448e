"""Row-wise int8 and e4m3 quantisation on rows built to hit exact rounding
ties, bit-exact against the FP64 oracle on every legal plan: each row's
amax makes the scale a power of two (int8: amax = 127/8, multiplier 8;
e4m3: amax = 112, multiplier 4), so value * multiplier lands exactly halfway
between two codes and round-to-nearest-even decides.  Also an all-zero row
(scale 1, codes 0) and a row with a single nonzero value.  Then rows whose
reciprocal Q / amax is inexact in FP32: exact ties of x * Q / amax, and
values next to a decision boundary where an FP32 evaluation of
x * fl32(Q / amax) rounds to another code than the definition (the kernel
must decide those exactly, as the oracle does)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

from _cases import ALL_PLANS, to_device
from _quant_rows import fp32_departure_rows, fp32_product_codes, tie_rows as exact_tie_rows

pytestmark = pytest.mark.gpu


def tie_rows(N: int, fmt: str) -> np.ndarray:
    rng = np.random.default_rng([51, N, fmt == "int8"])
    x = np.zeros((4, N))
    if fmt == "int8":
        mult = 8.0
        for r in (1, 2):
            k = rng.integers(-127, 127, N)           # (k + 0.5) lies in [-126.5, 126.5]
            x[r] = (k + 0.5) / mult
            x[r, rng.integers(N)] = (127.0 if r == 1 else -127.0) / mult   # the row's amax
    else:
        mult = 4.0
        for r in (1, 2):
            e = rng.integers(-6, 8, N)               # normal binades up to 2^8
            m = rng.integers(0, 8, N)                # halfway above mantissa m (m = 7: below the next power)
            v = np.ldexp(1.0 + (m + 0.5) / 8.0, e)
            sub = rng.random(N) < 0.1                # subnormal midpoints (j + 1/2) 2^-9
            v[sub] = (rng.integers(0, 7, sub.sum()) + 0.5) * 2.0 ** -9
            x[r] = np.where(rng.random(N) < 0.5, -v, v) / mult
            x[r, rng.integers(N)] = (448.0 if r == 1 else -448.0) / mult
    x[3, rng.integers(N)] = -3.0                     # one nonzero value; row 0 stays zero
    return x.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("N", [3001, 65536])
@pytest.mark.parametrize("fmt", ["int8", "fp8"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_quantisation_ties_zero_and_single_value_rows(gpu_handle, dtype, fmt, N):
    # every value of these rows has at most 8 significant bits, so BF16 input
    # holds them exactly and the expected codes are the same
    h = gpu_handle
    x = tie_rows(N, fmt)
    raw, _ = I.store(x, dtype)
    assert np.array_equal(oracle.decode(raw, dtype), x)
    mult = 8.0 if fmt == "int8" else 4.0
    assert np.all(np.abs(x[1:3]).max(axis=1) * mult == (127.0 if fmt == "int8" else 448.0))
    codes_ref, scale_ref = oracle.quantize_rows(x.astype(np.float32), fmt)
    assert scale_ref[0] == 1.0 and np.all(codes_ref[0] == 0)
    op = C.QUANT_INT8 if fmt == "int8" else C.QUANT_FP8
    xd = to_device(raw, dtype)
    for v, k in ALL_PLANS:
        p = C.plan(v, k)
        if not h.plan_legal(op, C.FWD, C.DTYPE_NAMES[dtype], 4, N, p):
            continue
        print(f"[quant ties] {dtype} -> {fmt} N={N} {p}", flush=True)
        q, qs = C.quantize_rows(xd, fmt, p=p, h=h)
        torch.cuda.synchronize()
        assert np.array_equal(qs.cpu().numpy().view(np.uint32), scale_ref.view(np.uint32)), f"{p}: scale"
        bad = np.flatnonzero(q.cpu().numpy().view(np.uint8) != codes_ref.view(np.uint8))
        assert bad.size == 0, f"{p}: {bad.size} codes differ, first at {bad[0]}"
    assert h.check_errors() == C.OK


def _check_all_plans(h, x, dtype, fmt, tag):
    raw, _ = I.store(x, dtype)
    assert np.array_equal(oracle.decode(raw, dtype), x)
    codes_ref, scale_ref = oracle.quantize_rows(x.astype(np.float32), fmt)
    op = C.QUANT_INT8 if fmt == "int8" else C.QUANT_FP8
    M, N = x.shape
    xd = to_device(raw, dtype)
    ran = 0
    for v, k in ALL_PLANS:
        p = C.plan(v, k)
        if not h.plan_legal(op, C.FWD, C.DTYPE_NAMES[dtype], M, N, p):
            continue
        print(f"[quant {tag}] {dtype} -> {fmt} {M}x{N} {p}", flush=True)
        q, qs = C.quantize_rows(xd, fmt, p=p, h=h)
        torch.cuda.synchronize()
        assert np.array_equal(qs.cpu().numpy().view(np.uint32), scale_ref.view(np.uint32)), f"{p}: scale"
        bad = np.flatnonzero(q.cpu().numpy().view(np.uint8) != codes_ref.view(np.uint8))
        assert bad.size == 0, f"{p}: {bad.size} codes differ, first at {bad[0]}"
        ran += 1
    assert ran >= 3
    assert h.check_errors() == C.OK
    return codes_ref


@pytest.mark.parametrize("N", [4099, 65536])
@pytest.mark.parametrize("fmt", ["int8", "fp8"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_quantisation_exact_ties_with_inexact_reciprocal(gpu_handle, dtype, fmt, N):
    x = exact_tie_rows(N, fmt)
    _check_all_plans(gpu_handle, x, dtype, fmt, "exact ties")


@pytest.mark.parametrize("N", [4099, 65536])
@pytest.mark.parametrize("fmt", ["int8", "fp8"])
def test_quantisation_where_the_fp32_product_departs(gpu_handle, fmt, N):
    x = fp32_departure_rows(N, fmt, per_row=24)
    codes = _check_all_plans(gpu_handle, x, "f32", fmt, "fp32 departures")
    fp32 = np.stack([fp32_product_codes(r, fmt) for r in x])
    assert int((fp32 != codes.view(np.uint8)).sum()) >= 4 * 24
