"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (the plans the installed selector ranks first, then every
other legal plan): inputs are generated row-block by
row-block from the per-row seeded generators and uploaded; the oracle then
regenerates only a seeded sample of rows and checks those rows exactly
(rows are independent).  dgamma / dbeta depend on every row and are checked
in full against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

from _cases import EPS, check_tensor, ulp_bf16

pytestmark = pytest.mark.gpu
TDT = {"f32": torch.float32, "bf16": torch.bfloat16, "fp8": torch.uint8}
NUM = {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}


def upload(M, N, dtype, gen_rows, block=256):
    """Device tensor (and FP8 row scales) filled block by block."""
    t = torch.empty((M, N), dtype=TDT[dtype], device="cuda")
    sc = torch.empty(M, dtype=torch.float32, device="cuda") if dtype == "fp8" else None
    for r0 in range(0, M, block):
        rows = np.arange(r0, min(M, r0 + block))
        raw, s = I.store(gen_rows(rows), dtype)
        host = torch.from_numpy(raw.view(np.int16)).view(torch.bfloat16) if dtype == "bf16" else torch.from_numpy(raw)
        t[r0:r0 + len(rows)].copy_(host.to("cuda"))
        if sc is not None:
            sc[r0:r0 + len(rows)].copy_(torch.from_numpy(s).cuda())
    return t, sc


def exact_rows(gen_rows, rows, dtype):
    """FP64 values the GPU consumed for the sampled rows."""
    raw, s = I.store(gen_rows(rows), dtype)
    return oracle.decode(raw, dtype, s)


def gpu_rows(t, rows, dtype, scale=None):
    sub = t[torch.from_numpy(rows).cuda()]
    if dtype == "f32":
        return sub.double().cpu().numpy()
    if dtype == "bf16":
        return oracle.decode_bf16(sub.view(torch.int16).cpu().numpy().view(np.uint16))
    return oracle.decode(sub.cpu().numpy(), "fp8", scale[torch.from_numpy(rows).cuda()].cpu().numpy())


def sample(M, n=8, seed=0):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([[0, M - 1], rng.choice(M, n, replace=False)]))


def plans_for(h, op, d, dt, M, N, all_plans):
    # the benchmark keeps the faster of the network's two best plans: test both
    f = C.features(op, d, NUM[dt], M, N)
    lg = h.mlp_predict(f[None, :])[0]
    legal = [c for c in range(C.NUM_PLANS) if h.plan_legal(op, d, NUM[dt], M, N, C.plan_of_class(c))]
    out = [C.plan_of_class(c) for c in sorted(legal, key=lambda c: -lg[c])[:2]]
    if all_plans:
        for c in range(C.NUM_PLANS):
            p = C.plan_of_class(c)
            if h.plan_legal(op, d, NUM[dt], M, N, p) and p.as_tuple() not in [q.as_tuple() for q in out]:
                out.append(p)
    return out


@pytest.fixture(scope="module")
def hsel(lib_built):
    h = C.Handle(0)  # with the installed selector model, as the benchmark runs
    assert h.model_loaded
    yield h
    h.close()


@pytest.mark.parametrize("N", [8192, 32768, 131072, 524288])
@pytest.mark.parametrize("op", ["layernorm_fwd", "rmsnorm_fwd"])
def test_bandwidth_config_full_size(hsel, op, N):
    # FP32 LayerNorm / RMSNorm forward, M = 1024, x ~ N(10, 1)
    M = 1024
    gen = lambda rows: I.norm_rows(M, N, seed=1, tensor=0, rows=rows)
    x, _ = upload(M, N, "f32", gen)
    g32, b32 = I.norm_params(N, seed=1)
    g, b = torch.from_numpy(g32).cuda(), torch.from_numpy(b32).cuda()
    rows = sample(M, seed=N)
    xr = exact_rows(gen, rows, "f32")
    if op == "layernorm_fwd":
        ref, _, _ = oracle.layernorm_fwd(xr, g32.astype(np.float64), b32.astype(np.float64), EPS)
    else:
        ref, _ = oracle.rmsnorm_fwd(xr, g32.astype(np.float64), EPS)
    o = C.LAYERNORM if op == "layernorm_fwd" else C.RMSNORM
    for p in plans_for(hsel, o, C.FWD, "f32", M, N, all_plans=True):
        print(f"[full] {op} N={N} {p}", flush=True)
        if op == "layernorm_fwd":
            y, _, _, _ = C.layernorm_fwd(x, g, b, EPS, p=p, h=hsel)
        else:
            y, _, _ = C.rmsnorm_fwd(x, g, EPS, p=p, h=hsel)
        torch.cuda.synchronize()
        check_tensor("y", op, "f32", gpu_rows(y, rows, "f32"), ref, np.abs(ref))
        del y
    assert hsel.check_errors() == C.OK


@pytest.mark.parametrize("N", [65536, 262144])
@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_precision_config_full_size(hsel, dtype, N):
    # softmax and LayerNorm forward, M = 4096, x = 3 N(0,1) with 1% outliers at +-40
    M = 4096
    gen = lambda rows: I.outlier_rows(M, N, seed=2, tensor=0, rows=rows)
    x, xs = upload(M, N, dtype, gen)
    g32, b32 = I.norm_params(N, seed=2)
    g, b = torch.from_numpy(g32).cuda(), torch.from_numpy(b32).cuda()
    rows = sample(M, seed=N + 1)
    xr = exact_rows(gen, rows, dtype)
    ys_ref = oracle.softmax_fwd(xr)
    yl_ref, mu, rs = oracle.layernorm_fwd(xr, g32.astype(np.float64), b32.astype(np.float64), EPS)
    mag_l = np.abs(xr) * rs[:, None] * g32 + np.abs(b32)
    for p in plans_for(hsel, C.SOFTMAX, C.FWD, dtype, M, N, all_plans=True):
        print(f"[full] softmax {dtype} N={N} {p}", flush=True)
        y, ysc = C.softmax_fwd(x, xs, p=p, h=hsel)
        torch.cuda.synchronize()
        check_tensor("y", "softmax_fwd", dtype, gpu_rows(y, rows, dtype, ysc), ys_ref, np.abs(ys_ref), ysc, rows=rows)
        del y
    for p in plans_for(hsel, C.LAYERNORM, C.FWD, dtype, M, N, all_plans=True):
        print(f"[full] layernorm {dtype} N={N} {p}", flush=True)
        y, ysc, _, _ = C.layernorm_fwd(x, g, b, EPS, xs, p=p, h=hsel)
        torch.cuda.synchronize()
        check_tensor("y", "layernorm_fwd", dtype, gpu_rows(y, rows, dtype, ysc), yl_ref, mag_l, ysc, rows=rows)
        del y
    assert hsel.check_errors() == C.OK


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_backward_config_full_size(hsel, dtype):
    # softmax backward and LayerNorm backward, M = 2048, N = 131072, dy ~ N(0,1)
    M, N = 2048, 131072
    # softmax backward: y = (rounded) softmax of 4 N(0, 1) rows, computed by the oracle
    gen_y = lambda rows: oracle.softmax_fwd(I.softmax_rows(M, N, seed=3, tensor=0, rows=rows))
    gen_dy = lambda rows: I.normal_rows(M, N, seed=3, tensor=1, rows=rows)
    y, _ = upload(M, N, dtype, gen_y)
    dy, _ = upload(M, N, dtype, gen_dy)
    rows = sample(M, seed=11)
    yr, dyr = exact_rows(gen_y, rows, dtype), exact_rows(gen_dy, rows, dtype)
    ref = oracle.softmax_bwd(yr, dyr)
    mag = np.abs(yr) * (np.abs(dyr) + np.abs(np.sum(yr * dyr, 1, keepdims=True)))
    for p in plans_for(hsel, C.SOFTMAX, C.BWD, dtype, M, N, all_plans=True):
        print(f"[full] softmax bwd {dtype} {p}", flush=True)
        dx, _ = C.softmax_bwd(y, dy, p=p, h=hsel)
        torch.cuda.synchronize()
        check_tensor("dx", "softmax_bwd", dtype, gpu_rows(dx, rows, dtype), ref, mag)
        del dx
    del y
    # LayerNorm backward with saved statistics; dgamma / dbeta over all rows
    gen_x = lambda rows: I.norm_rows(M, N, seed=3, tensor=2, rows=rows)
    x, _ = upload(M, N, dtype, gen_x)
    xall = np.empty((M, N))
    dyall = np.empty((M, N))
    for r0 in range(0, M, 256):
        rr = np.arange(r0, r0 + 256)
        xall[rr] = exact_rows(gen_x, rr, dtype)
        dyall[rr] = exact_rows(gen_dy, rr, dtype)
    g32, _ = I.norm_params(N, seed=3)
    g64 = g32.astype(np.float64)
    _, mu, rs = oracle.layernorm_fwd(xall, g64, np.zeros(N), EPS)
    dxr, dgr, dbr = oracle.layernorm_bwd(xall, dyall, g64, EPS)
    mean_t = torch.from_numpy(mu.astype(np.float32)).cuda()
    rstd_t = torch.from_numpy(rs.astype(np.float32)).cuda()
    g = torch.from_numpy(g32).cuda()
    xh = (xall[rows] - mu[rows, None]) * rs[rows, None]
    gg = dyall[rows] * g64
    c1 = gg.mean(1, keepdims=True)
    c2 = (gg * xh).mean(1, keepdims=True)
    magd = rs[rows, None] * (np.abs(gg) + np.abs(c1) + np.abs(xall[rows]) * rs[rows, None] * np.abs(c2))
    # column tolerances: 1e-5 of the summed magnitude (FP32 accumulation over M rows)
    dg_tol = 1e-5 * np.abs(dyall * (xall - mu[:, None]) * rs[:, None]).sum(0) + 1e-6
    db_tol = 1e-5 * np.abs(dyall).sum(0) + 1e-6
    del xall
    for p in plans_for(hsel, C.LAYERNORM, C.BWD, dtype, M, N, all_plans=True):
        print(f"[full] layernorm bwd {dtype} {p}", flush=True)
        dx, _, dg, db = C.layernorm_bwd(x, dy, g, mean_t, rstd_t, EPS, p=p, h=hsel)
        torch.cuda.synchronize()
        check_tensor("dx", "layernorm_bwd", dtype, gpu_rows(dx, rows, dtype), dxr[rows], magd)
        assert np.all(np.abs(dg.double().cpu().numpy() - dgr) <= dg_tol), "dgamma"
        assert np.all(np.abs(db.double().cpu().numpy() - dbr) <= db_tol), "dbeta"
        del dx
    assert hsel.check_errors() == C.OK
