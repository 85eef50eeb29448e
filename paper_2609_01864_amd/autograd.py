"""torch.autograd.Function wrappers over the library's forward and backward
kernels (FP32 and BF16 I/O).  The forward saves y (softmax), or the logits x
when asked to (the backward then rebuilds y inside the row: the
softmax-logits backward of the evaluation suite, Sec. IV-A), or x with the
FP32 row statistics (normalisations); the backward is itself a
reduction-reuse pass computed by the library (dx; dgamma / dbeta by column
reduction)."""
from __future__ import annotations

import torch

from . import credit as C


def _rows(t):
    return t.reshape(-1, t.shape[-1])


class SoftmaxFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan=None):
        x2 = _rows(x.contiguous())
        y, _ = C.softmax_fwd(x2, p=plan)
        ctx.save_for_backward(y)
        ctx.plan_bwd = None
        return y.view_as(x)

    @staticmethod
    def backward(ctx, dy):
        (y,) = ctx.saved_tensors
        dx, _ = C.softmax_bwd(y, _rows(dy.contiguous().to(y.dtype)), p=ctx.plan_bwd)
        return dx.view(dy.shape), None


class SoftmaxLogitsFn(torch.autograd.Function):
    """Softmax that saves its input instead of its output; the backward
    recomputes y = softmax(x) in the same pass that forms dx."""

    @staticmethod
    def forward(ctx, x, plan=None):
        x2 = _rows(x.contiguous())
        y, _ = C.softmax_fwd(x2, p=plan)
        ctx.save_for_backward(x2)
        return y.view_as(x)

    @staticmethod
    def backward(ctx, dy):
        (x2,) = ctx.saved_tensors
        dx, _ = C.softmax_logits_bwd(x2, _rows(dy.contiguous().to(x2.dtype)))
        return dx.view(dy.shape), None


class LayerNormFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, gamma, beta, eps=1e-5, plan=None):
        x2 = _rows(x.contiguous())
        y, _, mean, rstd = C.layernorm_fwd(x2, gamma.contiguous(), beta.contiguous(), eps, p=plan)
        ctx.save_for_backward(x2, gamma, mean, rstd)
        ctx.eps = eps
        return y.view_as(x)

    @staticmethod
    def backward(ctx, dy):
        x2, gamma, mean, rstd = ctx.saved_tensors
        dx, _, dg, db = C.layernorm_bwd(x2, _rows(dy.contiguous().to(x2.dtype)), gamma.contiguous(), mean, rstd,
                                        ctx.eps, need_dgamma=ctx.needs_input_grad[1],
                                        need_dbeta=ctx.needs_input_grad[2])
        return dx.view(dy.shape), dg, db, None, None


class RMSNormFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, gamma, eps=1e-5, plan=None):
        x2 = _rows(x.contiguous())
        y, _, rstd = C.rmsnorm_fwd(x2, gamma.contiguous(), eps, p=plan)
        ctx.save_for_backward(x2, gamma, rstd)
        ctx.eps = eps
        return y.view_as(x)

    @staticmethod
    def backward(ctx, dy):
        x2, gamma, rstd = ctx.saved_tensors
        dx, _, dg = C.rmsnorm_bwd(x2, _rows(dy.contiguous().to(x2.dtype)), gamma.contiguous(), rstd, ctx.eps,
                                  need_dgamma=ctx.needs_input_grad[1])
        return dx.view(dy.shape), dg, None, None


def softmax(x, plan=None, save: str = "output"):
    """Softmax over the last dimension.  save="logits" keeps x for the
    backward instead of y (same memory, and x is often kept anyway)."""
    if save == "logits":
        return SoftmaxLogitsFn.apply(x, plan)
    if save != "output":
        raise ValueError(f"save must be 'output' or 'logits', not {save!r}")
    return SoftmaxFn.apply(x, plan)


def layer_norm(x, gamma, beta, eps: float = 1e-5, plan=None):
    """LayerNorm over the last dimension (biased variance, eps inside the root)."""
    return LayerNormFn.apply(x, gamma, beta, eps, plan)


def rms_norm(x, gamma, eps: float = 1e-5, plan=None):
    """RMSNorm over the last dimension."""
    return RMSNormFn.apply(x, gamma, eps, plan)
