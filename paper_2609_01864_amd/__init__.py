"""MI355X (gfx950) wide reduction-reuse row kernels: row softmax, LayerNorm
and RMSNorm, forward and backward, in FP32 / BF16 / FP8-e4m3 I/O, each with a
two-pass, a register-resident and a split-row variant chosen per shape by the
CREDIT profitability model, a learned selector or exhaustive timing.

``credit`` is the ctypes binding of libcredit (include/credit.h);
``autograd`` holds the torch.autograd.Function layer.  Importing the package
loads nothing: the shared library is opened on first use and its absence is an
error, never a fallback."""

__all__ = ["credit", "autograd", "inputs", "build"]
