"""LayerNorm and RMSNorm, forward and backward, on the degenerate rows of the
method (Sec. III-B: the statistics of a row): a constant row (variance 0, so
rstd = 1/sqrt(eps) and LayerNorm returns beta), a row of zeros (RMSNorm
returns 0) and a row of two values.  Every legal plan against the FP64
oracle, in FP32, BF16 and FP8-e4m3, with the tolerance rules of the other
parity tests."""
import numpy as np
import pytest

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

from _cases import ALL_PLANS, OPNUM, Case, check_case

pytestmark = pytest.mark.gpu


def degenerate_rows(N: int) -> np.ndarray:
    return np.stack([np.full(N, 7.25),                               # constant
                     np.zeros(N),                                     # zeros
                     np.where(np.arange(N) % 2 == 0, 3.0, -1.0)])     # two values


@pytest.mark.parametrize("N", [3001, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("op", ["layernorm_fwd", "rmsnorm_fwd", "layernorm_bwd", "rmsnorm_bwd"])
def test_degenerate_rows(gpu_handle, op, dtype, N):
    h = gpu_handle
    x = degenerate_rows(N)
    M = x.shape[0]
    case = Case(op, dtype, M, N, seed=41)
    case.raw["x"] = I.store(x, dtype)
    case.vals = {k: oracle.decode(r, dtype, s) for k, (r, s) in case.raw.items()}
    ref = case.reference()
    for k in ("y", "dx", "rstd", "mean"):
        if k in ref:
            assert np.all(np.isfinite(ref[k]))
    o, d = OPNUM[op]
    for v, kk in ALL_PLANS:
        p = C.plan(v, kk)
        if not h.plan_legal(o, d, C.DTYPE_NAMES[dtype], M, N, p):
            continue
        print(f"[degenerate] {op} {dtype} N={N} {p}", flush=True)
        try:
            check_case(case, case.run(h, p, ref=ref), ref)
        except AssertionError as e:
            raise AssertionError(f"{p}: {e}") from None


@pytest.mark.parametrize("N", [3001, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_softmax_backward_of_one_hot_and_uniform_rows(gpu_handle, dtype, N):
    # y one-hot: dx = 0 exactly (in FP8 the stored 1 is 448 times the FP32
    # scale 1/448, a hair off 1, so dx is tiny there instead);
    # y uniform 1/N: dx = (dy - mean dy) / N; y with two equal halves
    h = gpu_handle
    y = np.zeros((3, N))
    y[0, N // 3] = 1.0
    y[1] = 1.0 / N
    y[2, : N // 2] = 1.0 / (2 * (N // 2))
    case = Case("softmax_bwd", dtype, 3, N, seed=42)
    case.raw["y"] = I.store(y, dtype)
    case.vals = {k: oracle.decode(r, dtype, s) for k, (r, s) in case.raw.items()}
    ref = case.reference()
    exact = dtype != "fp8"
    assert np.all(ref["dx"][0] == 0.0) or not exact
    o, d = OPNUM["softmax_bwd"]
    for v, kk in ALL_PLANS:
        p = C.plan(v, kk)
        if not h.plan_legal(o, d, C.DTYPE_NAMES[dtype], 3, N, p):
            continue
        print(f"[degenerate] softmax_bwd {dtype} N={N} {p}", flush=True)
        out = case.run(h, p, ref=ref)
        assert np.all(out["dx"][0] == 0.0) or not exact, f"{p}: one-hot row has a gradient"
        try:
            check_case(case, out, ref)
        except AssertionError as e:
            raise AssertionError(f"{p}: {e}") from None
