"""Pins of the oracle for the other reduction-reuse workloads of the paper's
evaluation suite (Sec. IV-A): softmax backward from the logits, row-wise
int8 / e4m3 quantisation, Pearson-correlation backward and weighted-variance
backward.  Each pin comes from outside the oracle's own formula: finite
differences of an independently computed forward, library routines (numpy,
torch autograd), closed forms, invariances and brute force on tiny inputs."""
import numpy as np
import pytest
import torch

import oracle

RNG = np.random.default_rng(20240607)


# ------------------------------------------------------------ softmax-logits
def _softmax_np(x):
    e = np.exp(x - x.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def test_softmax_logits_bwd_finite_differences():
    # gradient of L(x) = sum_i dy_i softmax(x)_i, central differences in FP64
    x = RNG.standard_normal((3, 9)) * 2
    dy = RNG.standard_normal((3, 9))
    dx = oracle.softmax_logits_bwd(x, dy)
    h = 1e-6
    fd = np.empty_like(x)
    for i in range(x.shape[1]):
        xp, xm = x.copy(), x.copy()
        xp[:, i] += h
        xm[:, i] -= h
        fd[:, i] = ((_softmax_np(xp) * dy).sum(1) - (_softmax_np(xm) * dy).sum(1)) / (2 * h)
    assert np.max(np.abs(dx - fd)) <= 1e-8 * max(1.0, np.max(np.abs(fd)))


def test_softmax_logits_bwd_against_torch_autograd():
    x = torch.from_numpy(RNG.standard_normal((4, 33)) * 3).requires_grad_(True)
    dy = torch.from_numpy(RNG.standard_normal((4, 33)))
    (torch.softmax(x, dim=1) * dy).sum().backward()
    dx = oracle.softmax_logits_bwd(x.detach().numpy(), dy.numpy())
    assert np.max(np.abs(dx - x.grad.numpy())) <= 1e-14


def test_softmax_logits_bwd_invariances():
    x = RNG.standard_normal((5, 40)) * 4
    dy = RNG.standard_normal((5, 40))
    dx = oracle.softmax_logits_bwd(x, dy)
    # the rows of dx sum to zero (softmax sums to one)
    assert np.max(np.abs(dx.sum(1))) <= 1e-15 * 40
    # a constant added to the logits or to the upstream gradient changes nothing
    assert np.max(np.abs(oracle.softmax_logits_bwd(x + 3.0, dy) - dx)) <= 1e-15
    assert np.max(np.abs(oracle.softmax_logits_bwd(x, dy - 1.25) - dx)) <= 1e-15


def test_softmax_logits_bwd_two_elements_closed_form():
    # N = 2: y0 = logistic(x0 - x1), dx0 = y0 y1 (dy0 - dy1) = -dx1
    x = RNG.standard_normal((6, 2)) * 3
    dy = RNG.standard_normal((6, 2))
    y0 = 1.0 / (1.0 + np.exp(x[:, 1] - x[:, 0]))
    ref0 = y0 * (1 - y0) * (dy[:, 0] - dy[:, 1])
    dx = oracle.softmax_logits_bwd(x, dy)
    assert np.max(np.abs(dx[:, 0] - ref0)) <= 1e-15
    assert np.max(np.abs(dx[:, 1] + ref0)) <= 1e-15


# ---------------------------------------------------------- quantisation
# The code is the grid point nearest to x * Q / amax, ties to even; the pins
# compare the oracle with brute force over the whole grid in rational
# arithmetic (tests/_quant_rows.py), on random rows, on exact ties whose
# reciprocal Q / amax is inexact in FP32, and on values where an FP32
# evaluation of the same formula departs from the definition.
from _quant_rows import exact_codes, fp32_departure_rows, fp32_product_codes, tie_rows  # noqa: E402


def _quant_inputs():
    x = (RNG.standard_normal((5, 37)) * 3).astype(np.float32)
    x[1, 3] = 40.0
    x[2, :] = 0.0  # all-zero row
    x[3, 5] = -7.5
    x[4, 7] = -0.0
    return x


def _scale_is_nearest_fp32(scale: np.float32, amax: np.float32, q: int) -> bool:
    from fractions import Fraction
    exact = Fraction(float(amax)) / q
    s = np.float32(scale)
    lo, hi = np.nextafter(s, np.float32(-np.inf)), np.nextafter(s, np.float32(np.inf))
    ds = abs(Fraction(float(s)) - exact)
    return ds <= abs(Fraction(float(lo)) - exact) and ds <= abs(Fraction(float(hi)) - exact)


@pytest.mark.parametrize("fmt", ["int8", "fp8"])
def test_quantize_codes_brute_force_exact_definition(fmt):
    x = np.concatenate([_quant_inputs(), tie_rows(37, fmt).astype(np.float32),
                        fp32_departure_rows(37, fmt, per_row=6).astype(np.float32)])
    codes, scale = oracle.quantize_rows(x, fmt)
    q = 127 if fmt == "int8" else 448
    for m in range(x.shape[0]):
        assert np.array_equal(codes[m].view(np.uint8), exact_codes(x[m], fmt)), m
        amax = np.float32(np.max(np.abs(x[m])))
        if amax == 0:
            assert scale[m] == np.float32(1.0)
            continue
        assert _scale_is_nearest_fp32(scale[m], amax, q), m
        # the largest magnitude lands on the end of the grid
        got = codes[m].view(np.int8).astype(np.int64) if fmt == "int8" else oracle.decode_e4m3(codes[m])
        assert np.max(np.abs(got)) == q


@pytest.mark.parametrize("fmt", ["int8", "fp8"])
def test_quantize_is_not_the_fp32_product(fmt):
    # values next to decision boundaries where x * fl32(Q / amax) rounds to
    # another code: the oracle takes the definition's code at every one of them
    x = fp32_departure_rows(101, fmt, per_row=12).astype(np.float32)
    codes, _ = oracle.quantize_rows(x, fmt)
    fp32 = oracle.quantize_rows_fp32_product(x, fmt)
    departs = np.stack([fp32_product_codes(r, fmt) for r in x]) != np.stack([exact_codes(r, fmt) for r in x])
    assert departs.sum() >= 4 * 12
    assert np.array_equal(fp32.view(np.uint8) != codes.view(np.uint8), departs)


def test_quantize_int8_error_bound_and_symmetry():
    x = (RNG.standard_normal((8, 300)) * 2).astype(np.float32)
    codes, scale = oracle.quantize_rows(x, "int8")
    amax = np.max(np.abs(x), axis=1).astype(np.float64)
    step = amax / 127.0
    # the code is the nearest integer to x * 127 / amax: within half a step
    assert np.all(np.abs(codes.astype(np.float64) * step[:, None] - x) <= 0.5 * step[:, None] * (1 + 1e-12))
    ncodes, nscale = oracle.quantize_rows(-x, "int8")
    assert np.array_equal(ncodes.astype(np.int64), -codes.astype(np.int64))
    assert np.array_equal(nscale, scale)


def test_quantize_fp8_error_bound_and_symmetry():
    x = (RNG.standard_normal((8, 300)) * 3).astype(np.float32)
    codes, scale = oracle.quantize_rows(x, "fp8")
    amax = np.max(np.abs(x), axis=1).astype(np.float64)
    v = x * 448.0 / amax[:, None]
    got = oracle.decode_e4m3(codes)
    steps = np.vectorize(oracle.e4m3_step)(np.abs(v))
    assert np.all(np.abs(got - v) <= 0.5 * steps * (1 + 1e-12))
    ncodes, nscale = oracle.quantize_rows(-x, "fp8")
    assert np.array_equal(ncodes ^ 0x80, codes) and np.array_equal(nscale, scale)


# ------------------------------------------------------------ Pearson
def _pearson_np(x, y):
    return np.array([np.corrcoef(x[m], y[m])[0, 1] for m in range(x.shape[0])])


def _pearson_inputs(M, N):
    x = RNG.standard_normal((M, N))
    y = 0.6 * x + 0.8 * RNG.standard_normal((M, N))
    return x, y, RNG.standard_normal(M)


def test_pearson_bwd_finite_differences():
    x, y, dr = _pearson_inputs(3, 8)
    gx, gy = oracle.pearson_bwd(x, y, dr)
    h = 1e-6
    for i in range(8):
        xp, xm, yp, ym = x.copy(), x.copy(), y.copy(), y.copy()
        xp[:, i] += h
        xm[:, i] -= h
        yp[:, i] += h
        ym[:, i] -= h
        fdx = dr * (_pearson_np(xp, y) - _pearson_np(xm, y)) / (2 * h)
        fdy = dr * (_pearson_np(x, yp) - _pearson_np(x, ym)) / (2 * h)
        assert np.max(np.abs(gx[:, i] - fdx)) <= 1e-8
        assert np.max(np.abs(gy[:, i] - fdy)) <= 1e-8


def test_pearson_bwd_against_torch_autograd():
    x, y, dr = _pearson_inputs(4, 50)
    xt = torch.from_numpy(x).requires_grad_(True)
    yt = torch.from_numpy(y).requires_grad_(True)
    r = torch.stack([torch.corrcoef(torch.stack([xt[m], yt[m]]))[0, 1] for m in range(4)])
    (r * torch.from_numpy(dr)).sum().backward()
    gx, gy = oracle.pearson_bwd(x, y, dr)
    assert np.max(np.abs(gx - xt.grad.numpy())) <= 1e-13
    assert np.max(np.abs(gy - yt.grad.numpy())) <= 1e-13


def test_pearson_bwd_invariances_and_special_cases():
    x, y, dr = _pearson_inputs(5, 60)
    gx, gy = oracle.pearson_bwd(x, y, dr)
    # r is invariant under a shift of x: the gradient sums to zero, and under
    # a positive scaling of x: the gradient is orthogonal to x - mean(x)
    assert np.max(np.abs(gx.sum(1))) <= 1e-14
    assert np.max(np.abs((gx * (x - x.mean(1, keepdims=True))).sum(1))) <= 1e-13
    # affine change of x: dx scales by 1 / a
    gx2, gy2 = oracle.pearson_bwd(2.5 * x - 4.0, y, dr)
    assert np.max(np.abs(gx2 * 2.5 - gx)) <= 1e-13
    assert np.max(np.abs(gy2 - gy)) <= 1e-13
    # symmetry in (x, y)
    hy, hx = oracle.pearson_bwd(y, x, dr)
    assert np.max(np.abs(hx - gx)) <= 1e-15 and np.max(np.abs(hy - gy)) <= 1e-15
    # exactly correlated rows (y = 3x + 1): r = 1 is a maximum, the gradient vanishes
    gxe, gye = oracle.pearson_bwd(x, 3.0 * x + 1.0, dr)
    assert np.max(np.abs(gxe)) <= 1e-13 and np.max(np.abs(gye)) <= 1e-13


# ------------------------------------------------------- weighted variance
def _wvar_np(x, w):
    return np.array([np.cov(x[m], aweights=w[m], bias=True) for m in range(x.shape[0])])


def test_wvar_bwd_finite_differences():
    x = RNG.standard_normal((3, 8)) + 2
    w = RNG.uniform(0.2, 1.0, (3, 8))
    dv = RNG.standard_normal(3)
    gx, gw = oracle.wvar_bwd(x, w, dv)
    h = 1e-6
    for i in range(8):
        xp, xm, wp, wm = x.copy(), x.copy(), w.copy(), w.copy()
        xp[:, i] += h
        xm[:, i] -= h
        wp[:, i] += h
        wm[:, i] -= h
        fdx = dv * (_wvar_np(xp, w) - _wvar_np(xm, w)) / (2 * h)
        fdw = dv * (_wvar_np(x, wp) - _wvar_np(x, wm)) / (2 * h)
        assert np.max(np.abs(gx[:, i] - fdx)) <= 1e-8
        assert np.max(np.abs(gw[:, i] - fdw)) <= 1e-8


def test_wvar_bwd_against_torch_autograd():
    x = RNG.standard_normal((4, 45))
    w = RNG.uniform(0.0, 1.0, (4, 45))
    dv = RNG.standard_normal(4)
    xt = torch.from_numpy(x).requires_grad_(True)
    wt = torch.from_numpy(w).requires_grad_(True)
    v = torch.stack([torch.cov(xt[m], aweights=wt[m], correction=0) for m in range(4)])
    (v * torch.from_numpy(dv)).sum().backward()
    gx, gw = oracle.wvar_bwd(x, w, dv)
    assert np.max(np.abs(gx - xt.grad.numpy())) <= 1e-14
    assert np.max(np.abs(gw - wt.grad.numpy())) <= 1e-14


def test_wvar_bwd_uniform_weights_and_invariances():
    x = RNG.standard_normal((4, 64)) * 2 + 5
    dv = RNG.standard_normal(4)
    c = 0.7
    gx, gw = oracle.wvar_bwd(x, np.full_like(x, c), dv)
    mu = x.mean(1, keepdims=True)
    var = ((x - mu) ** 2).mean(1, keepdims=True)
    # uniform weights: the textbook gradient of the population variance
    assert np.max(np.abs(gx - dv[:, None] * 2 * (x - mu) / 64)) <= 1e-14
    assert np.max(np.abs(gw - dv[:, None] * ((x - mu) ** 2 - var) / (64 * c))) <= 1e-14
    w = RNG.uniform(0.1, 1.0, x.shape)
    gx, gw = oracle.wvar_bwd(x, w, dv)
    # shift of x: gradient sums to zero; scaling all weights: v unchanged
    assert np.max(np.abs(gx.sum(1))) <= 1e-13
    assert np.max(np.abs((gw * w).sum(1))) <= 1e-13
    # a weight-scaled copy gives gradients scaled by 1 / a in w
    gx2, gw2 = oracle.wvar_bwd(x, 4.0 * w, dv)
    assert np.max(np.abs(gx2 - gx)) <= 1e-14 and np.max(np.abs(gw2 * 4.0 - gw)) <= 1e-14


@pytest.mark.parametrize("fmt", ["int8", "fp8"])
def test_quantize_rejects_non_fp32_values(fmt):
    with pytest.raises(ValueError):
        oracle.quantize_rows(np.array([[0.1, 0.2]]), fmt)
