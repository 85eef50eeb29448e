"""Degenerate rows of the other reduction-reuse workloads, every legal plan
against the FP64 oracle with the tolerance rules of the workload tests:

* weighted-variance backward: a constant row (variance 0: both gradients
  vanish), equal weights, and a single nonzero weight (the mean is that
  element, so dx = 0 and dw = (x - x_j)^2 / W);
* Pearson backward: y = 2x and y = -x (r = +-1 exactly, where the gradient
  vanishes and what remains is cancellation, bounded by the magnitude rule);
* LayerNorm -> e4m3 with beta = 0 on a constant row: y = 0, so amax = 0, the
  scale is 1 and every code is 0.
"""
import numpy as np
import pytest

import oracle
from paper_2609_01864_amd import inputs as I

from test_workloads_gpu import WCase, check, legal_plans

pytestmark = pytest.mark.gpu


def _set(case, **rows):
    for k, v in rows.items():
        case.raw[k] = I.store(v, case.dtype)
    case.vals = {k: oracle.decode(r, case.dtype, s) for k, (r, s) in case.raw.items()}


def _run_all(h, case, tag):
    with np.errstate(divide="ignore", invalid="ignore"):  # undefined rows are 0/0
        ref = case.reference()
    for p in legal_plans(h, case.op, case.dtype, case.M, case.N):
        print(f"[degenerate] {tag} {case.dtype} N={case.N} {p}", flush=True)
        try:
            check(case, case.run(h, p), ref)
        except AssertionError as e:
            raise AssertionError(f"{p}: {e}") from None


@pytest.mark.parametrize("N", [3001, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_weighted_variance_degenerate_rows(gpu_handle, dtype, N):
    case = WCase("wvar", dtype, 3, N, seed=61)
    x = I.normal_rows(3, N, 61, 0, mean=2.0)
    x[0] = 2.5
    w = I.uniform_rows(3, N, 61, 1)
    w[1] = 0.5
    w[2] = 0.0
    w[2, N // 2] = 0.75
    _set(case, x=x, w=w)
    _run_all(gpu_handle, case, "wvar")


@pytest.mark.parametrize("N", [3001, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_pearson_exactly_correlated_rows(gpu_handle, dtype, N):
    case = WCase("pearson", dtype, 2, N, seed=62)
    x = oracle.decode(I.store(I.normal_rows(2, N, 62, 0), dtype)[0], dtype)
    y = np.stack([2.0 * x[0], -x[1]])  # exact in the I/O format
    _set(case, x=x, y=y)
    _run_all(gpu_handle, case, "pearson")


@pytest.mark.parametrize("N", [3001, 65536])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_layernorm_fp8_out_of_a_zero_output_row(gpu_handle, dtype, N):
    case = WCase("lnq", dtype, 2, N, seed=63)
    x = I.norm_rows(2, N, 63)
    x[0] = 7.25
    _set(case, x=x)
    case.beta = np.zeros_like(case.beta)
    _run_all(gpu_handle, case, "lnq")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_undefined_statistics_are_non_finite_like_the_oracle(gpu_handle, dtype):
    # Pearson with a constant x (S_xx = 0) and weighted variance with all
    # weights 0 (W = 0) are 0/0: the oracle's plain definitions give
    # non-finite gradients there, and so must every plan, with the other
    # rows intact (the finiteness rule of the workload checks)
    N = 5003
    case = WCase("pearson", dtype, 3, N, seed=64)
    x, y = I.correlated_rows(3, N, 64)
    x[1] = 1.5
    _set(case, x=x, y=y)
    _run_all(gpu_handle, case, "pearson undefined")
    case = WCase("wvar", dtype, 3, N, seed=65)
    w = I.uniform_rows(3, N, 65, 1)
    w[1] = 0.0
    _set(case, w=w)
    _run_all(gpu_handle, case, "wvar undefined")
