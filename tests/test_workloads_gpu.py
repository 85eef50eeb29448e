"""GPU parity of the other reduction-reuse workloads of the evaluation suite
(Sec. IV-A) -- softmax backward from the logits, row-wise int8 / e4m3
quantisation, Pearson-correlation backward, weighted-variance backward --
through the C ABI, against the FP64 oracle on the values the GPU consumed.

Tolerances:
* quantisation: bit-exact codes and scales (the code nearest to
  x * Q / amax, decided exactly on both sides; the scale amax / Q rounded
  once to FP32);
* FP32 gradients: |got - ref| <= 1e-5 * m elementwise, with m the magnitude
  of the terms of the last operation, each statistic that cancels counted at
  the size of its summands (e.g. Pearson |dr / sqrt(Sxx Syy)| |y - mean y|
  + |dr / Sxx| |x - mean x|: |r| <= 1 stands for the resolution of Sxy, and
  |x| + |mean| for that of the centring; softmax-logits |y| (|dy| + sum |dy| y)).  The statistics are FP32 sums over up to
  N = 262144 elements; 1e-5 is about 170 FP32 ulps of the terms;
* BF16 / FP8 outputs: the one-ulp / one-step rules of the core operators.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

from _cases import ALL_PLANS, EPS, check_tensor, from_device, scale_dev, to_device, ulp_bf16

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1), (3, 7), (5, 17), (2, 33), (37, 1000), (4, 4097), (3, 20011)]
OPS = {"smxl": (C.SOFTMAX_LOGITS, C.BWD, ["f32", "bf16", "fp8"]),
       "quant_int8": (C.QUANT_INT8, C.FWD, ["f32", "bf16"]),
       "quant_fp8": (C.QUANT_FP8, C.FWD, ["f32", "bf16"]),
       "pearson": (C.PEARSON, C.BWD, ["f32", "bf16"]),
       "wvar": (C.WVAR, C.BWD, ["f32", "bf16"]),
       "lnq": (C.LAYERNORM_FP8_OUT, C.FWD, ["f32", "bf16"])}
DTN = {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}


class WCase:
    """Seeded inputs, oracle reference and GPU call of one workload."""

    def __init__(self, op, dtype, M, N, seed=0, rows=None):
        self.op, self.dtype, self.M, self.N = op, dtype, M, N
        if op == "smxl":
            x = I.outlier_rows(M, N, seed, 0, rows) if dtype != "f32" else I.softmax_rows(M, N, seed, 0, rows=rows)
            self.raw = {"x": I.store(x, dtype), "dy": I.store(I.normal_rows(M, N, seed, 1, rows=rows), dtype)}
        elif op.startswith("quant"):
            self.raw = {"x": I.store(I.outlier_rows(M, N, seed, 0, rows), dtype)}
        elif op == "lnq":
            self.raw = {"x": I.store(I.norm_rows(M, N, seed, 0, rows), dtype)}
            self.gamma, self.beta = I.norm_params(N, seed)
        elif op == "pearson":
            x, y = I.correlated_rows(M, N, seed, rows=rows)
            self.raw = {"x": I.store(x, dtype), "y": I.store(y, dtype)}
        else:
            self.raw = {"x": I.store(I.normal_rows(M, N, seed, 0, mean=2.0, rows=rows), dtype),
                        "w": I.store(I.uniform_rows(M, N, seed, 1, rows=rows), dtype)}
        self.vals = {k: oracle.decode(r, dtype, s) for k, (r, s) in self.raw.items()}
        g = I.row_vector(max(M, 1), seed)
        self.g = g[:M] if rows is None else g[np.asarray(rows)]

    def reference(self):
        v, g = self.vals, self.g.astype(np.float64)[:, None]
        if self.op == "smxl":
            dx = oracle.softmax_logits_bwd(v["x"], v["dy"])
            y = oracle.softmax_fwd(v["x"])
            # c = sum dy y cancels: its rounding scales with sum |dy| y
            c_mag = np.sum(y * np.abs(v["dy"]), 1, keepdims=True)
            return {"dx": dx, "mag_dx": np.abs(y) * (np.abs(v["dy"]) + c_mag)}
        if self.op.startswith("quant"):
            fmt = "int8" if self.op == "quant_int8" else "fp8"
            codes, scale = oracle.quantize_rows(v["x"].astype(np.float32), fmt)
            return {"codes": codes, "scale": scale}
        x = v["x"]
        if self.op == "lnq":
            gm, bt = self.gamma.astype(np.float64), self.beta.astype(np.float64)
            y, mu, rs = oracle.layernorm_fwd(x, gm, bt, EPS)
            return {"y": y, "mag_y": np.abs(x) * rs[:, None] * gm + np.abs(bt), "mean": mu, "rstd": rs}
        if self.op == "pearson":
            with np.errstate(divide="ignore", invalid="ignore"):  # N = 1: r undefined
                return self._pearson_reference(x, v["y"], g)
        w = v["w"]
        gx, gw = oracle.wvar_bwd(x, w, self.g)
        W = w.sum(1, keepdims=True)
        mu = (w * x).sum(1, keepdims=True) / W
        var = (w * (x - mu) ** 2).sum(1, keepdims=True) / W
        ad = np.abs(x) + np.abs(mu)
        return {"dx": gx, "dw": gw, "mag_dx": 2 * np.abs(g) / W * np.abs(w) * ad,
                "mag_dw": np.abs(g) / W * (ad * ad + var)}

    def _pearson_reference(self, x, y, g):
        gx, gy = oracle.pearson_bwd(x, y, self.g)
        mx, my = x.mean(1, keepdims=True), y.mean(1, keepdims=True)
        sxx = ((x - mx) ** 2).sum(1, keepdims=True)
        syy = ((y - my) ** 2).sum(1, keepdims=True)
        ax, ay = np.abs(x) + np.abs(mx), np.abs(y) + np.abs(my)
        a = np.abs(g) / np.sqrt(sxx * syy)
        # r = Sxy / sqrt(Sxx Syy) cancels: its rounding scales with
        # sum |xc yc| / sqrt(Sxx Syy) <= 1, so |r| is bounded by 1 here
        return {"dx": gx, "dy": gy, "mag_dx": a * ay + np.abs(g) / sxx * ax,
                "mag_dy": a * ax + np.abs(g) / syy * ay}

    def run(self, h, plan, ld_pad=0, offset=0):
        dt = self.dtype
        ld = self.N + ld_pad
        dev = {k: to_device(r, dt, ld, offset) for k, (r, s) in self.raw.items()}
        sc = {k: scale_dev(s) for k, (r, s) in self.raw.items()}
        out = {}
        if self.op == "smxl":
            dx, dxs = C.softmax_logits_bwd(dev["x"], dev["dy"], sc["x"], sc["dy"], p=plan, h=h)
            out = {"dx": from_device(dx, dt, dxs), "dx_scale": dxs}
        elif self.op == "lnq":
            q, qs, mu, rs = C.layernorm_fwd_fp8_out(dev["x"], torch.from_numpy(self.gamma).cuda(),
                                                    torch.from_numpy(self.beta).cuda(), EPS, p=plan, h=h)
            out = {"y": oracle.decode(q.cpu().numpy(), "fp8", qs.cpu().numpy()), "y_scale": qs,
                   "mean": mu.double().cpu().numpy(), "rstd": rs.double().cpu().numpy()}
        elif self.op.startswith("quant"):
            fmt = "int8" if self.op == "quant_int8" else "fp8"
            qbuf = torch.zeros(self.M * ld + offset + 64, dtype=torch.int8 if fmt == "int8" else torch.uint8,
                               device="cuda")
            qv = qbuf[offset:offset + self.M * ld].view(self.M, ld)[:, :self.N]
            q, qs = C.quantize_rows(dev["x"], fmt, p=plan, out=qv, h=h)
            out = {"codes": q.cpu().numpy(), "scale": qs.cpu().numpy()}
        else:
            g = torch.from_numpy(self.g).cuda()
            if self.op == "pearson":
                gx, gy = C.pearson_bwd(dev["x"], dev["y"], g, p=plan, h=h)
                out = {"dx": from_device(gx, dt), "dy": from_device(gy, dt)}
            else:
                gx, gw = C.wvar_bwd(dev["x"], dev["w"], g, p=plan, h=h)
                out = {"dx": from_device(gx, dt), "dw": from_device(gw, dt)}
        torch.cuda.synchronize()
        assert h.check_errors() == C.OK
        return out


def check(case, got, ref):
    if case.op == "lnq":
        check_tensor("y", "layernorm_fwd", "fp8", got["y"], ref["y"], ref["mag_y"], got["y_scale"])
        assert np.max(np.abs(got["rstd"] - ref["rstd"])) <= 1e-6 * np.max(ref["rstd"])
        assert np.max(np.abs(got["mean"] - ref["mean"])) <= 1e-5 * max(1.0, np.max(np.abs(ref["mean"])))
        return
    if case.op.startswith("quant"):
        assert np.array_equal(got["scale"].view(np.uint32), ref["scale"].view(np.uint32)), "scale"
        bad = np.flatnonzero(got["codes"].ravel().view(np.uint8) != ref["codes"].ravel().view(np.uint8))
        assert bad.size == 0, f"{bad.size} codes differ, first at {bad[0]}"
        return
    for name in [k for k in ref if not k.startswith("mag")]:
        g, r, m = got[name], ref[name], ref["mag_" + name]
        fin = np.isfinite(r)
        # rows where the statistic is undefined (Pearson with N = 1: Sxx = 0)
        # are non-finite on both sides
        assert np.array_equal(np.isfinite(g), fin), f"{name}: finiteness differs"
        if not fin.all():
            g, r, m = g[fin], r[fin], m[fin]
        if case.dtype == "f32":
            ratio = np.abs(g - r) / (1e-5 * m + 1e-30)
            assert float(ratio.max(initial=0.0)) <= 1.0, f"{name}: {float(ratio.max()):.3f} of the FP32 bound"
        elif case.dtype == "bf16":
            allow = ulp_bf16(np.maximum(np.abs(r), m / 256.0))
            worst = float((np.abs(g - r) / allow).max(initial=0.0))
            assert worst <= 1.0, f"{name}: {worst:.3f} bf16 ulp"
        else:  # fp8 (softmax from logits)
            check_tensor(name, "softmax_bwd", "fp8", g, r, m, got.get("dx_scale"))


def legal_plans(h, op, dtype, M, N):
    o, d, _ = OPS[op]
    out = []
    for v, k in ALL_PLANS:
        p = C.plan(v, k)
        if h.plan_legal(o, d, DTN[dtype], M, N, p):
            out.append(p)
    return out


@pytest.mark.parametrize("M,N", SHAPES)
@pytest.mark.parametrize("op,dtype", [(o, d) for o, (_, _, dts) in OPS.items() for d in dts])
def test_workload_parity_all_plans(gpu_handle, op, dtype, M, N):
    case = WCase(op, dtype, M, N, seed=M * 1000 + N)
    ref = case.reference()
    plans = legal_plans(gpu_handle, op, dtype, M, N)
    assert any(p.variant == C.TWO_PASS for p in plans)
    for p in plans:
        print(f"[workload] {op} {dtype} M={M} N={N} {p}", flush=True)
        check(case, case.run(gpu_handle, p), ref)


@pytest.mark.parametrize("op", list(OPS))
def test_workload_strided_misaligned(gpu_handle, op):
    # padded leading dimensions and a start offset of one element: the
    # under-aligned 128-bit path and the element-wise tail
    dtype = "bf16" if op != "smxl" else "fp8"
    M, N = 6, 3001
    case = WCase(op, dtype, M, N, seed=17)
    ref = case.reference()
    for p in legal_plans(gpu_handle, op, dtype, M, N):
        print(f"[workload-strided] {op} {dtype} {p}", flush=True)
        check(case, case.run(gpu_handle, p, ld_pad=13, offset=1), ref)


@pytest.mark.parametrize("op", list(OPS))
def test_workload_split_deterministic(gpu_handle, op):
    M, N = 64, 50000
    case = WCase(op, "f32", M, N, seed=5)
    p = C.plan("split", 8)
    a = case.run(gpu_handle, p)
    b = case.run(gpu_handle, p)
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("op", list(OPS))
def test_workload_zero_rows_and_illegal_args(gpu_handle, op):
    o, d, dts = OPS[op]
    h = gpu_handle
    x = torch.empty((0, 10), dtype=torch.float32, device="cuda")
    if op == "smxl":
        dx, _ = C.softmax_logits_bwd(x, x, h=h, p=C.plan("two_pass"))
        assert dx.shape == (0, 10)
        z = torch.zeros((4, 10), device="cuda")
        st = C.lib().credit_softmax_logits_bwd(h.ptr, 4, 20, C.F32, z.data_ptr(), 10, None, z.data_ptr(), 10, None,
                                               z.data_ptr(), 10, None, None, None, 0, None)
        assert st == C.ERR_INVALID_ARG  # ld < N
    elif op.startswith("quant"):
        q, s = C.quantize_rows(x, "int8" if op == "quant_int8" else "fp8", p=C.plan("two_pass"), h=h)
        assert q.shape == (0, 10)
        # FP8 input is not a quantisation source
        z = torch.zeros((4, 16), dtype=torch.uint8, device="cuda")
        with pytest.raises(C.CreditError):
            C.quantize_rows(z, "int8", p=C.plan("two_pass"), h=h)
    elif op == "lnq":
        gm = torch.ones(10, device="cuda")
        q, qs, _, _ = C.layernorm_fwd_fp8_out(x, gm, gm, EPS, p=C.plan("two_pass"), h=h)
        assert q.shape == (0, 10)
        z = torch.zeros((4, 16), dtype=torch.uint8, device="cuda")
        with pytest.raises(C.CreditError):  # the input is FP32 or BF16
            C.layernorm_fwd_fp8_out(z, torch.ones(16, device="cuda"), torch.ones(16, device="cuda"), EPS,
                                    p=C.plan("two_pass"), h=h)
    else:
        g = torch.zeros(0, device="cuda")
        fn = C.pearson_bwd if op == "pearson" else C.wvar_bwd
        a, b = fn(x, x, g, p=C.plan("two_pass"), h=h)
        assert a.shape == (0, 10) and b.shape == (0, 10)
        z = torch.zeros((4, 16), dtype=torch.uint8, device="cuda")
        with pytest.raises(C.CreditError):  # no FP8 form
            fn(z, z, torch.zeros(4, device="cuda"), p=C.plan("two_pass"), h=h)
    # a pair that does not exist
    assert C.lib().credit_plan_legal(None, o, 1 - d, C.F32, 4, 16, C.plan("two_pass")) == C.ERR_INVALID_ARG


FULL_N = [16384, 65536]


def upload_full(op, M, N, seed, block=256):
    """Device inputs of the full matrix, generated and uploaded row block by
    row block; returns (case over all rows without host values, device dict)."""
    dev = None
    for r0 in range(0, M, block):
        rows = np.arange(r0, min(M, r0 + block))
        part = WCase(op, "f32", M, N, seed=seed, rows=rows)
        if dev is None:
            dev = {k: torch.empty((M, N), dtype=torch.float32, device="cuda") for k in part.raw}
        for k, (r, _) in part.raw.items():
            dev[k][r0:r0 + len(rows)].copy_(torch.from_numpy(r).cuda())
    return dev


@pytest.mark.parametrize("N", FULL_N)
@pytest.mark.parametrize("op", list(OPS))
def test_workload_full_size_sampled_rows(gpu_handle, op, N):
    # the evaluation suite's sizes (FP32, M = 4096): every legal plan on the
    # full matrix, the oracle on a seeded sample of rows
    M = 4096
    h = gpu_handle
    dev = upload_full(op, M, N, seed=3)
    rng = np.random.default_rng(N)
    rows = np.unique(np.concatenate([[0, M - 1], rng.choice(M, 6, replace=False)]))
    sub = WCase(op, "f32", M, N, seed=3, rows=rows)
    ref = sub.reference()
    g = torch.from_numpy(I.row_vector(M, 3)).cuda()
    ri = torch.from_numpy(rows).cuda()
    for p in legal_plans(h, op, "f32", M, N):
        print(f"[workload-full] {op} N={N} {p}", flush=True)
        if op == "smxl":
            dx, _ = C.softmax_logits_bwd(dev["x"], dev["dy"], p=p, h=h)
            got = {"dx": dx[ri].double().cpu().numpy()}
        elif op.startswith("quant"):
            q, qs = C.quantize_rows(dev["x"], "int8" if op == "quant_int8" else "fp8", p=p, h=h)
            got = {"codes": q[ri].cpu().numpy(), "scale": qs[ri].cpu().numpy()}
        elif op == "lnq":
            q, qs, mu, rs = C.layernorm_fwd_fp8_out(dev["x"], torch.from_numpy(sub.gamma).cuda(),
                                                    torch.from_numpy(sub.beta).cuda(), EPS, p=p, h=h)
            got = {"y": oracle.decode(q[ri].cpu().numpy(), "fp8", qs[ri].cpu().numpy()), "y_scale": qs[ri],
                   "mean": mu[ri].double().cpu().numpy(), "rstd": rs[ri].double().cpu().numpy()}
        elif op == "pearson":
            a, b = C.pearson_bwd(dev["x"], dev["y"], g, p=p, h=h)
            got = {"dx": a[ri].double().cpu().numpy(), "dy": b[ri].double().cpu().numpy()}
        else:
            a, b = C.wvar_bwd(dev["x"], dev["w"], g, p=p, h=h)
            got = {"dx": a[ri].double().cpu().numpy(), "dw": b[ri].double().cpu().numpy()}
        torch.cuda.synchronize()
        assert h.check_errors() == C.OK
        check(sub, got, ref)
