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
def _brute_int8(v32: np.ndarray) -> np.ndarray:
    # nearest integer code in [-127, 127] to each FP32 value; ties to the even code
    codes = np.arange(-127, 128, dtype=np.float64)
    out = np.empty(v32.shape, dtype=np.int64)
    for idx, v in np.ndenumerate(v32.astype(np.float64)):
        d = np.abs(codes - v)
        best = np.flatnonzero(d == d.min())
        out[idx] = int(codes[best[0]] if len(best) == 1 else [c for c in codes[best] if int(c) % 2 == 0][0])
    return out


def _quant_inputs():
    x = (RNG.standard_normal((5, 37)) * 3).astype(np.float32)
    x[1, 3] = 40.0
    x[2, :] = 0.0  # all-zero row
    x[3, 5] = -7.5
    return x


def _tie_rows(q: float):
    # exact ties of the decision variable: amax = 127 (int8) or 448 (e4m3)
    # makes the reciprocal scale exactly 1, so v = x
    row = np.zeros(37, dtype=np.float32)
    if q == 127.0:
        row[:9] = [127.0, 0.5, 1.5, 2.5, -0.5, -2.5, 3.5, -126.5, 100.5]
        # a row with amax = 3 and two values where x * fl(127 / amax) and
        # x / fl(amax / 127) round to different integers (the decision is the
        # product with the FP32 reciprocal scale)
        row2 = np.zeros(37, dtype=np.float32)
        row2[:3] = [3.0] + np.array([1074418857, 1074220701], dtype=np.uint32).view(np.float32).tolist()
        return np.stack([row, row2])
    else:  # e4m3 steps are 1/8 in [1, 2) and 16 in [256, 448]
        row[:9] = [448.0, 1.0625, 1.1875, -1.0625, -1.1875, 264.0, 280.0, -296.0, 0.5 + 1.0 / 32]
    return row[None, :]


def test_quantize_int8_brute_force_nearest_code():
    x = np.concatenate([_quant_inputs(), _tie_rows(127.0)])
    codes, scale = oracle.quantize_rows(x, "int8")
    for m in range(x.shape[0]):
        amax = np.float32(np.max(np.abs(x[m])))
        if amax == 0:
            assert scale[m] == np.float32(1.0) and np.all(codes[m] == 0)
            continue
        # the decision variable: FP32 product of x with the FP32 reciprocal scale
        inv = np.float32(np.float32(127.0) / amax)
        v = (x[m] * inv).astype(np.float32)
        assert np.array_equal(codes[m].astype(np.int64), _brute_int8(v))
        assert scale[m] == np.float32(amax / np.float32(127.0))
        # the largest magnitude lands on +-127
        assert np.max(np.abs(codes[m].astype(np.int64))) == 127


def test_quantize_int8_error_bound_and_symmetry():
    x = (RNG.standard_normal((8, 300)) * 2).astype(np.float32)
    codes, scale = oracle.quantize_rows(x, "int8")
    deq = codes.astype(np.float64) * scale[:, None].astype(np.float64)
    # half a quantisation step, plus the FP32 rounding of scale and product
    assert np.all(np.abs(deq - x) <= 0.5 * scale[:, None] * (1 + 1e-5))
    ncodes, nscale = oracle.quantize_rows(-x, "int8")
    assert np.array_equal(ncodes.astype(np.int64), -codes.astype(np.int64))
    assert np.array_equal(nscale, scale)


def test_quantize_fp8_brute_force_nearest_e4m3():
    x = np.concatenate([_quant_inputs(), _tie_rows(448.0)])
    codes, scale = oracle.quantize_rows(x, "fp8")
    allc = np.arange(256, dtype=np.uint8)
    vals = torch.from_numpy(allc).view(torch.float8_e4m3fn).double().numpy()
    finite = np.isfinite(vals)
    fc, fv = allc[finite], vals[finite]
    for m in range(x.shape[0]):
        amax = np.float32(np.max(np.abs(x[m])))
        if amax == 0:
            assert scale[m] == np.float32(1.0) and np.all(oracle.decode_e4m3(codes[m]) == 0)
            continue
        inv = np.float32(np.float32(448.0) / amax)
        v = (x[m] * inv).astype(np.float32).astype(np.float64)
        got = oracle.decode_e4m3(codes[m])
        for i, vi in enumerate(v):
            vi = min(448.0, max(-448.0, vi))
            d = np.abs(fv - vi)
            cand = fv[d == d.min()]
            if len(set(cand.tolist())) == 1:
                assert got[i] == cand[0]
            else:  # tie: the even mantissa (lowest code bit 0)
                even = [fv[j] for j in np.flatnonzero(d == d.min()) if fc[j] % 2 == 0]
                assert got[i] == even[0]
        assert np.max(np.abs(got)) == 448.0
        assert scale[m] == np.float32(amax / np.float32(448.0))


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
