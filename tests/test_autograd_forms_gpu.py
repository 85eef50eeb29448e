"""The differentiation form through torch.autograd.Function (Sec. III-B, the
backward passes as reduction-reuse operators):

* FP32 gradients at M = 4, N = 16 against central finite differences in FP64
  of the oracle's forward definitions, with the loss L = sum(dy * f(x)).  The
  finite differences never touch the oracle's backward formulas, so this pins
  the GPU backward to the derivative itself.  A central difference with step
  h has error O(h^2 f''') + O(eps_64 |L| / h), about 1e-9 here, far below the
  FP32 bounds of the library's backward (dx: 1e-5 * max(1, |dx|_inf); dgamma
  / dbeta per column: 1e-5 of the summed magnitudes of the terms + 1e-6).
* BF16 tensors through the same autograd functions, against the FP64 oracle
  on the decoded BF16 inputs, to the one-BF16-ulp rules of the core
  operators.  With save="output" the backward consumes the forward's BF16 y,
  so it is compared with the exact gradient at x under a bound derived from
  that rounding: dx_i = y_i (dy_i - c), c = sum_j y_j dy_j; each y_j within
  one BF16 ulp (relative 2^-7) perturbs dx_i by at most
  2^-7 (1 + 2^-7) |y_i| (|dy_i| + |c| + sum_j |y_j dy_j|), on top of the one
  ulp of the result (taken at |dx| plus that perturbation).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import autograd as A
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

from _cases import EPS, ulp_bf16

pytestmark = pytest.mark.gpu


def _central(loss, v: np.ndarray, h: float) -> np.ndarray:
    """Central finite differences of a scalar function of the array v."""
    g = np.empty_like(v)
    flat, gf = v.reshape(-1), g.reshape(-1)
    for i in range(flat.size):
        keep = flat[i]
        flat[i] = keep + h
        up = loss()
        flat[i] = keep - h
        dn = loss()
        flat[i] = keep
        gf[i] = (up - dn) / (2.0 * h)
    return g


def _dx_bound(ref: np.ndarray) -> float:
    return 1e-5 * max(1.0, float(np.abs(ref).max()))


@pytest.mark.parametrize("save", ["output", "logits"])
def test_softmax_gradient_matches_fp64_finite_differences(lib_built, save):
    M, N = 4, 16
    x32 = I.softmax_rows(M, N, 11).astype(np.float32)
    dy32 = I.normal_rows(M, N, 11, 1).astype(np.float32)
    x = torch.from_numpy(x32).cuda().requires_grad_(True)
    A.softmax(x, save=save).backward(torch.from_numpy(dy32).cuda())
    got = x.grad.double().cpu().numpy()

    xv, dy = x32.astype(np.float64), dy32.astype(np.float64)
    fd = _central(lambda: float(np.sum(dy * oracle.softmax_fwd(xv))), xv, 1e-6)
    assert np.max(np.abs(got - fd)) <= _dx_bound(fd)
    assert np.all(np.abs(got.sum(1)) <= 1e-5 * np.abs(got).sum(1) + 1e-7)  # softmax's dx rows sum to 0


def test_layernorm_gradients_match_fp64_finite_differences(lib_built):
    M, N = 4, 16
    x32 = I.norm_rows(M, N, 12).astype(np.float32)
    dy32 = I.normal_rows(M, N, 12, 1).astype(np.float32)
    g32, b32 = I.norm_params(N, 12)
    x = torch.from_numpy(x32).cuda().requires_grad_(True)
    g = torch.from_numpy(g32).cuda().requires_grad_(True)
    b = torch.from_numpy(b32).cuda().requires_grad_(True)
    A.layer_norm(x, g, b, EPS).backward(torch.from_numpy(dy32).cuda())

    xv, dy = x32.astype(np.float64), dy32.astype(np.float64)
    gv, bv = g32.astype(np.float64), b32.astype(np.float64)
    loss = lambda: float(np.sum(dy * oracle.layernorm_fwd(xv, gv, bv, EPS)[0]))  # noqa: E731
    fd_x = _central(loss, xv, 1e-5)
    fd_g = _central(loss, gv, 1e-6)
    fd_b = _central(loss, bv, 1e-6)

    _, mu, rs = oracle.layernorm_fwd(xv, gv, bv, EPS)
    assert np.max(np.abs(x.grad.double().cpu().numpy() - fd_x)) <= _dx_bound(fd_x)
    # x_hat = (x - mean) * rstd cancels: its FP32 resolution is set by |x| + |mean|
    dg_tol = 1e-5 * (np.abs(dy) * (np.abs(xv) + np.abs(mu[:, None])) * rs[:, None]).sum(0) + 1e-6
    assert np.all(np.abs(g.grad.double().cpu().numpy() - fd_g) <= dg_tol)
    assert np.all(np.abs(b.grad.double().cpu().numpy() - fd_b) <= 1e-5 * np.abs(dy).sum(0) + 1e-6)


def test_rmsnorm_gradients_match_fp64_finite_differences(lib_built):
    M, N = 4, 16
    x32 = (I.normal_rows(M, N, 13, 0) + 0.5).astype(np.float32)
    dy32 = I.normal_rows(M, N, 13, 1).astype(np.float32)
    g32, _ = I.norm_params(N, 13)
    x = torch.from_numpy(x32).cuda().requires_grad_(True)
    g = torch.from_numpy(g32).cuda().requires_grad_(True)
    A.rms_norm(x, g, EPS).backward(torch.from_numpy(dy32).cuda())

    xv, dy, gv = x32.astype(np.float64), dy32.astype(np.float64), g32.astype(np.float64)
    loss = lambda: float(np.sum(dy * oracle.rmsnorm_fwd(xv, gv, EPS)[0]))  # noqa: E731
    fd_x = _central(loss, xv, 1e-6)
    fd_g = _central(loss, gv, 1e-6)

    _, rs = oracle.rmsnorm_fwd(xv, gv, EPS)
    assert np.max(np.abs(x.grad.double().cpu().numpy() - fd_x)) <= _dx_bound(fd_x)
    dg_tol = 1e-5 * np.abs(dy * xv * rs[:, None]).sum(0) + 1e-6
    assert np.all(np.abs(g.grad.double().cpu().numpy() - fd_g) <= dg_tol)


# ------------------------------------------------------------------ BF16
def _bf16(x64: np.ndarray, shape):
    """(device BF16 tensor of the given shape, exact FP64 values as [M, N])."""
    bits = I.store(x64, "bf16")[0]
    t = torch.from_numpy(bits.view(np.int16).reshape(shape)).view(torch.bfloat16).cuda()
    return t, oracle.decode(bits, "bf16")


def _bf16_values(t) -> np.ndarray:
    return oracle.decode_bf16(t.detach().contiguous().view(torch.int16).cpu().numpy().view(np.uint16))


def _ulps(got, ref, mag) -> float:
    return float((np.abs(got - ref) / ulp_bf16(np.maximum(np.abs(ref), mag / 256.0))).max())


SHAPES = [(3, 5, 1000), (3, 5, 40000)]


@pytest.mark.parametrize("save", ["output", "logits"])
@pytest.mark.parametrize("shape", SHAPES)
def test_softmax_autograd_bf16(lib_built, save, shape):
    N = shape[-1]
    M = int(np.prod(shape[:-1]))
    x, xv = _bf16(I.outlier_rows(M, N, 21), shape)
    dy, dyv = _bf16(I.normal_rows(M, N, 21, 1), shape)
    x.requires_grad_(True)
    y = A.softmax(x, save=save)
    assert y.dtype == torch.bfloat16
    y.backward(dy)
    assert x.grad.dtype == torch.bfloat16

    yr = oracle.softmax_fwd(xv)
    assert _ulps(_bf16_values(y).reshape(M, N), yr, np.abs(yr)) <= 1.0
    dxr = oracle.softmax_logits_bwd(xv, dyv)
    got = _bf16_values(x.grad).reshape(M, N)
    c = np.sum(yr * dyv, 1, keepdims=True)
    s_abs = np.sum(np.abs(yr * dyv), 1, keepdims=True)
    if save == "logits":  # y rebuilt inside the row: the one-ulp rule
        assert _ulps(got, dxr, np.abs(yr) * (np.abs(dyv) + s_abs)) <= 1.0
    else:
        from_y = 2.0 ** -7 * (1 + 2.0 ** -7) * np.abs(yr) * (np.abs(dyv) + np.abs(c) + s_abs)
        # the ulp is taken at |dx| + from_y: the result may sit one binade up
        allow = from_y + ulp_bf16(np.maximum(np.abs(dxr) + from_y, np.abs(yr) * (np.abs(dyv) + s_abs) / 256.0))
        worst = float((np.abs(got - dxr) / allow).max())
        assert worst <= 1.0, f"{worst:.3f} of the bound"


@pytest.mark.parametrize("op", ["layer_norm", "rms_norm"])
@pytest.mark.parametrize("shape", SHAPES)
def test_norm_autograd_bf16(lib_built, op, shape):
    N = shape[-1]
    M = int(np.prod(shape[:-1]))
    x, xv = _bf16(I.norm_rows(M, N, 22), shape)
    dy, dyv = _bf16(I.normal_rows(M, N, 22, 1), shape)
    g32, b32 = I.norm_params(N, 22)
    gv, bv = g32.astype(np.float64), b32.astype(np.float64)
    x.requires_grad_(True)
    g = torch.from_numpy(g32).cuda().requires_grad_(True)
    b = torch.from_numpy(b32).cuda().requires_grad_(True)
    y = A.layer_norm(x, g, b, EPS) if op == "layer_norm" else A.rms_norm(x, g, EPS)
    assert y.dtype == torch.bfloat16
    y.backward(dy)
    got_y = _bf16_values(y).reshape(M, N)
    got_dx = _bf16_values(x.grad).reshape(M, N)
    gg = dyv * gv
    if op == "layer_norm":
        yr, mu, rs = oracle.layernorm_fwd(xv, gv, bv, EPS)
        dxr, dgr, dbr = oracle.layernorm_bwd(xv, dyv, gv, EPS)
        # y: x - mean cancels, judged at |x| rstd |gamma| + |beta|
        assert _ulps(got_y, yr, np.abs(xv) * rs[:, None] * gv + np.abs(bv)) <= 1.0
        xh = (xv - mu[:, None]) * rs[:, None]
        c1 = gg.mean(1, keepdims=True)
        c2 = (gg * xh).mean(1, keepdims=True)
        mag = rs[:, None] * (np.abs(gg) + np.abs(c1) + np.abs(xv) * rs[:, None] * np.abs(c2))
        dg_mag = (np.abs(dyv) * (np.abs(xv) + np.abs(mu[:, None])) * rs[:, None]).sum(0)
        assert np.all(np.abs(b.grad.double().cpu().numpy() - dbr) <= 1e-5 * np.abs(dyv).sum(0) + 1e-6)
    else:
        yr, rs = oracle.rmsnorm_fwd(xv, gv, EPS)
        dxr, dgr = oracle.rmsnorm_bwd(xv, dyv, gv, EPS)
        assert _ulps(got_y, yr, np.abs(yr)) <= 1.0
        xh = xv * rs[:, None]
        c = (gg * xh).mean(1, keepdims=True)
        mag = rs[:, None] * (np.abs(gg) + np.abs(xh * c))
        dg_mag = np.abs(dyv * xh).sum(0)
    assert _ulps(got_dx, dxr, mag) <= 1.0
    assert g.grad.dtype == torch.float32
    assert np.all(np.abs(g.grad.double().cpu().numpy() - dgr) <= 1e-5 * dg_mag + 1e-6)
    assert C.handle().check_errors() == C.OK
