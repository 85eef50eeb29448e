"""The autograd layer over the C ABI: forward and backward of softmax (saving
y, or the logits), LayerNorm and RMSNorm on a 3-D FP32 input, against the FP64
oracle on the same values."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import autograd as A
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

pytestmark = pytest.mark.gpu
EPS = 1e-5


def _vals(shape, seed, tensor=0, kind="softmax"):
    M = int(np.prod(shape[:-1]))
    N = shape[-1]
    if kind == "softmax":
        v = I.softmax_rows(M, N, seed, tensor)
    elif kind == "norm":
        v = I.norm_rows(M, N, seed, tensor)
    else:
        v = I.normal_rows(M, N, seed, tensor)
    return v.astype(np.float32)


@pytest.mark.parametrize("save", ["output", "logits"])
@pytest.mark.parametrize("N", [1000, 40000])
def test_softmax_autograd(lib_built, save, N):
    shape = (3, 5, N)
    x32, dy32 = _vals(shape, 1), _vals(shape, 1, 1, "normal")
    x = torch.from_numpy(x32.reshape(shape)).cuda().requires_grad_(True)
    y = A.softmax(x, save=save)
    y.backward(torch.from_numpy(dy32.reshape(shape)).cuda())
    yr = oracle.softmax_fwd(x32.astype(np.float64))
    dxr = oracle.softmax_logits_bwd(x32.astype(np.float64), dy32.astype(np.float64))
    assert np.max(np.abs(y.detach().reshape(-1, N).double().cpu().numpy() - yr)) <= 2e-6
    c_mag = np.sum(yr * np.abs(dy32), 1, keepdims=True)
    err = np.abs(x.grad.reshape(-1, N).double().cpu().numpy() - dxr)
    # the saved-y backward sees y rounded to FP32: one more rounding per element
    assert np.all(err <= 1e-5 * np.abs(yr) * (np.abs(dy32) + c_mag) + 1e-12)


def test_softmax_autograd_rejects_unknown_save(lib_built):
    with pytest.raises(ValueError):
        A.softmax(torch.zeros((2, 4), device="cuda"), save="both")


@pytest.mark.parametrize("op", ["layer_norm", "rms_norm"])
def test_norm_autograd(lib_built, op):
    shape, N = (4, 3, 5000), 5000
    x32, dy32 = _vals(shape, 2, 0, "norm"), _vals(shape, 2, 1, "normal")
    g32, b32 = I.norm_params(N, 2)
    x = torch.from_numpy(x32.reshape(shape)).cuda().requires_grad_(True)
    g = torch.from_numpy(g32).cuda().requires_grad_(True)
    b = torch.from_numpy(b32).cuda().requires_grad_(True)
    if op == "layer_norm":
        y = A.layer_norm(x, g, b, EPS)
    else:
        y = A.rms_norm(x, g, EPS)
    y.backward(torch.from_numpy(dy32.reshape(shape)).cuda())
    x64, dy64, g64 = x32.astype(np.float64), dy32.astype(np.float64), g32.astype(np.float64)
    if op == "layer_norm":
        yr, mu, rs = oracle.layernorm_fwd(x64, g64, b32.astype(np.float64), EPS)
        dxr, dgr, dbr = oracle.layernorm_bwd(x64, dy64, g64, EPS)
        xh = (x64 - mu[:, None]) * rs[:, None]
        db_tol = 1e-5 * np.abs(dy64).sum(0) + 1e-6
        assert np.all(np.abs(b.grad.double().cpu().numpy() - dbr) <= db_tol)
    else:
        yr, rs = oracle.rmsnorm_fwd(x64, g64, EPS)
        dxr, dgr = oracle.rmsnorm_bwd(x64, dy64, g64, EPS)
        xh = x64 * rs[:, None]
    assert np.max(np.abs(y.detach().reshape(-1, N).double().cpu().numpy() - yr)) <= 1e-5
    assert np.max(np.abs(x.grad.reshape(-1, N).double().cpu().numpy() - dxr)) <= 1e-5 * max(1.0, np.abs(dxr).max())
    # dgamma per column: 1e-5 of the summed magnitudes (FP32 sums over the rows)
    dg_tol = 1e-5 * np.abs(dy64 * xh).sum(0) + 1e-6
    assert np.all(np.abs(g.grad.double().cpu().numpy() - dgr) <= dg_tol)
    assert A is not None and C.handle().check_errors() == C.OK
