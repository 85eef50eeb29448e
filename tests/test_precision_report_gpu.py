"""Error of the precision forms against the FP64 oracle, per result, next to
the plain FP32 two-pass kernel: softmax and LayerNorm forward, M = 4096 rows,
N in {65536, 262144}, x = 3 N(0, 1) with 1% outliers at +-40 (the FP32 values
are the common input; BF16 stores them rounded to nearest even, FP8-e4m3 as
codes with the per-row scale amax / 448).  Every reduction is FP32 inside the
kernels.  For each result two errors are measured on sampled rows:

* kernel: against the oracle on exactly the values the kernel consumed (the
  parity bound: FP32 max abs error, BF16 ulps, FP8 e4m3 steps of the bound);
* end to end: against the oracle on the FP32 input, so the rounding of the
  input to the narrower format is included; reported as max |err| / max |y|
  over the row and as the relative RMS error.

The table is printed; with CREDIT_REPORT_DIR set it is also written there as
precision_errors.md.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

from _cases import EPS, check_tensor

pytestmark = pytest.mark.gpu
M = 4096
ROWS = np.array([0, 1, 517, 1024, 2047, 2048, 3001, 4094, 4095])
TDT = {"f32": torch.float32, "bf16": torch.bfloat16, "fp8": torch.uint8}
NUM = {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}


def _upload(N, seed):
    """x in FP32, BF16 and FP8 on the device, filled row block by row block
    from one generation of the FP32 values."""
    dev = {d: torch.empty((M, N), dtype=TDT[d], device="cuda") for d in TDT}
    scale = torch.empty(M, dtype=torch.float32, device="cuda")
    for r0 in range(0, M, 256):
        rows = np.arange(r0, min(M, r0 + 256))
        x32 = I.outlier_rows(M, N, seed, 0, rows=rows).astype(np.float32).astype(np.float64)
        for d in TDT:
            raw, s = I.store(x32, d)
            host = torch.from_numpy(raw.view(np.int16)).view(torch.bfloat16) if d == "bf16" else torch.from_numpy(raw)
            dev[d][r0:r0 + len(rows)].copy_(host.to("cuda"))
            if s is not None:
                scale[r0:r0 + len(rows)].copy_(torch.from_numpy(s).cuda())
    return dev, scale


def _consumed(N, seed, dtype):
    x32 = I.outlier_rows(M, N, seed, 0, rows=ROWS).astype(np.float32).astype(np.float64)
    raw, s = I.store(x32, dtype)
    return x32, oracle.decode(raw, dtype, s)


def _values(t, dtype, scale=None):
    sub = t[torch.from_numpy(ROWS).cuda()]
    if dtype == "f32":
        return sub.double().cpu().numpy()
    if dtype == "bf16":
        return oracle.decode_bf16(sub.view(torch.int16).cpu().numpy().view(np.uint16))
    return oracle.decode(sub.cpu().numpy(), "fp8", scale[torch.from_numpy(ROWS).cuda()].cpu().numpy())


def _end_to_end(got, truth):
    e = got - truth
    norm = np.abs(truth).max(axis=1, keepdims=True)
    return float((np.abs(e) / norm).max()), float(np.sqrt((e * e).sum() / (truth * truth).sum()))


@pytest.fixture(scope="module")
def hsel(lib_built):
    h = C.Handle(0)
    yield h
    h.close()


REPORT = []


@pytest.mark.parametrize("N", [65536, 262144])
def test_precision_errors_against_fp64_oracle(hsel, N):
    seed = 7
    print(f"[prec] uploading M={M} N={N}", flush=True)
    dev, x_scale = _upload(N, seed)
    g32, b32 = I.norm_params(N, seed)
    g, b = torch.from_numpy(g32).cuda(), torch.from_numpy(b32).cuda()
    g64, b64 = g32.astype(np.float64), b32.astype(np.float64)
    truth_s = truth_l = None
    runs = [("f32", C.plan("two_pass"), "FP32 two-pass (plain)"), ("f32", None, "FP32"),
            ("bf16", None, "BF16"), ("fp8", None, "FP8-e4m3")]
    for op in ("softmax", "layernorm"):
        for dtype, plan, label in runs:
            x32, xv = _consumed(N, seed, dtype)
            sc = x_scale if dtype == "fp8" else None
            o = C.SOFTMAX if op == "softmax" else C.LAYERNORM
            used = plan if plan is not None else hsel.select(o, C.FWD, NUM[dtype], M, N)[0]
            if op == "softmax":
                ref = oracle.softmax_fwd(xv)
                mag = np.abs(ref)
                truth_s = oracle.softmax_fwd(x32) if truth_s is None else truth_s
                truth = truth_s
                y, ysc = C.softmax_fwd(dev[dtype], sc, p=used, h=hsel)
            else:
                ref, mu, rs = oracle.layernorm_fwd(xv, g64, b64, EPS)
                mag = np.abs(xv) * rs[:, None] * g64 + np.abs(b64)
                truth_l = oracle.layernorm_fwd(x32, g64, b64, EPS)[0] if truth_l is None else truth_l
                truth = truth_l
                y, ysc, _, _ = C.layernorm_fwd(dev[dtype], g, b, EPS, sc, p=used, h=hsel)
            torch.cuda.synchronize()
            got = _values(y, dtype, ysc)
            bound = check_tensor("y", op + "_fwd", dtype, got, ref, mag, ysc, rows=ROWS)
            worst_abs = float(np.abs(got - ref).max())
            if dtype == "f32":  # as a fraction of the FP32 bound
                bound = worst_abs / (2e-6 if op == "softmax" else 1e-5)
            e2e_max, e2e_rms = _end_to_end(got, truth)
            REPORT.append((op, N, label, str(used), worst_abs, bound, e2e_max, e2e_rms, dtype))
            print(f"[prec] {op} N={N} {label} {used}: kernel max abs {worst_abs:.3e} "
                  f"({bound:.3f} of the bound), end to end max/rowmax {e2e_max:.3e}, rel rms {e2e_rms:.3e}",
                  flush=True)
            del y
    assert hsel.check_errors() == C.OK


def test_write_precision_report():
    if not REPORT:
        pytest.skip("no precision results in this session")
    unit = {"f32": "of the FP32 bound", "bf16": "BF16 ulps", "fp8": "of the e4m3 bound"}
    lines = ["| op | N | form | plan | kernel max abs err | kernel worst (unit) | end-to-end max err / row max |"
             " end-to-end rel. RMS |", "|---|---:|---|---|---:|---|---:|---:|"]
    for op, N, label, plan, wa, bd, em, er, dt in REPORT:
        lines.append(f"| {op} | {N} | {label} | {plan} | {wa:.2e} | {bd:.3g} ({unit[dt]}) | {em:.2e} | {er:.2e} |")
    text = "\n".join(lines)
    print(text)
    out = os.environ.get("CREDIT_REPORT_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        with open(os.path.join(out, "precision_errors.md"), "w") as f:
            f.write(text + "\n")
