#!/usr/bin/env python3
"""Benchmark of the reduction-reuse row kernels on one MI355X.

Workload (one "step"): FP32 LayerNorm and RMSNorm forward, eps = 1e-5, M = 1024
rows, N in {8192, 32768, 131072, 524288}; x ~ N(10, 1), gamma ~ U(0.5, 1.5),
beta ~ N(0, 0.1).  Every (op, N) call runs the plan the library's selector
picks for the shape (learned model if one is installed, else the profile-guided
analytic model); each call reads its own input buffers, so no input is served
from a cache warmed by the previous call.

Prints one JSON line: aggregate algorithmic GB/s over the timed steps, the
roofline of the dominant kernel (HIP events on the launch stream), the CPU
oracle timed on a bounded sample, and per-shape plan regret against
exhaustive timing.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M_ROWS = 1024
WIDTHS = (8192, 32768, 131072, 524288)
EPS = 1e-5
PEAK_GBPS = 8000.0
OPS = ("layernorm_fwd", "rmsnorm_fwd")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the kernel sources and of the build script (its compiler flags
    and per-file schedules shape the kernels as much as the sources do)."""
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_2609_01864_amd")
    csrc = os.path.join(pkg, "csrc")
    for path in [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))] + [os.path.join(pkg, "build.py")]:
        with open(path, "rb") as fh:
            h.update(os.path.basename(path).encode() + fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(op: str, M: int, N: int) -> int:
    # x read + y written once, gamma (and beta) once, mean/rstd per row
    vec = 2 if op == "layernorm_fwd" else 1
    return M * N * 4 * 2 + vec * N * 4 + vec * M * 4


def cpu_baseline(target_s: float = 10.0, single_s: float = 4.0):
    """The FP64 oracle (as it stands, built -O3 -march=native on this host) on
    the whole workload -- every (op, N), all 1024 rows -- repeated until about
    `target_s` seconds of oracle time on all host threads, then on one thread
    for about `single_s` seconds.  Input generation is outside the timed
    calls."""
    import numpy as np

    import oracle
    from paper_2609_01864_amd import inputs as I

    oracle.use_native()

    def run(limit_s, rows):
        total_bytes, total_s, passes = 0, 0.0, 0
        sel = np.arange(rows)
        while total_s < limit_s and passes < 60:
            for N in WIDTHS:
                x = I.norm_rows(M_ROWS, N, seed=1, tensor=0, rows=sel).astype(np.float32).astype(np.float64)
                g, b = I.norm_params(N, seed=1)
                g = g.astype(np.float64)
                b = b.astype(np.float64)
                t0 = time.perf_counter()
                oracle.layernorm_fwd(x, g, b, EPS)
                oracle.rmsnorm_fwd(x, g, EPS)
                total_s += time.perf_counter() - t0
                total_bytes += algorithmic_bytes("layernorm_fwd", rows, N) + algorithmic_bytes("rmsnorm_fwd", rows, N)
                del x
            passes += 1
        return total_bytes / total_s / 1e9, passes, total_s

    cores = oracle.num_threads()
    gb_all, passes, secs = run(target_s, M_ROWS)
    oracle.set_num_threads(1)
    gb_one, passes1, secs1 = run(single_s, 32)
    oracle.set_num_threads(cores)
    return {"value": round(gb_all, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "single_core_value": round(gb_one, 3),
            "sample": f"the whole workload (LayerNorm + RMSNorm forward, all 1024 rows of each N) x {passes} "
                      f"passes on {cores} threads ({secs:.1f} s of oracle time); on 1 thread the first 32 rows "
                      f"of each N x {passes1} passes ({secs1:.1f} s); FP64 C oracle, gcc -O3 -march=native "
                      f"-fopenmp"}


def device_identity(torch):
    """The GPU the numbers come from: name, architecture, CUs, PCI location
    and UUID, as the runtime reports them."""
    pr = torch.cuda.get_device_properties(0)
    return {"name": pr.name, "arch": pr.gcnArchName, "cus": pr.multi_processor_count,
            "pci": f"{pr.pci_domain_id:04x}:{pr.pci_bus_id:02x}:{pr.pci_device_id:02x}", "uuid": str(pr.uuid),
            "total_memory_gib": round(pr.total_memory / 2 ** 30, 1)}


def kernel_symbol(C, h, op_num, dt_num, M, N, p):
    """Demangled name prefix and grid (work-items) of the launch of plan p."""
    g = h.geometry(op_num, C.FWD if op_num < 3 else C.BWD, dt_num, M, N, p)
    kop = op_num
    if p.variant == C.TWO_PASS:
        return f"void credit::k_twopass<{kop}, {dt_num}, {g['block']}, 4>", g["grid"] * g["block"]
    if g["rows"] > 1:  # the multi-row norm forward
        return f"void credit::k_multirow<{kop}, {dt_num}, {g['vpt']}, {g['rows']}>", g["grid"] * g["block"]
    reg = min(g["vpt"], 32)  # slices past 32 vectors per thread keep the rest in LDS
    return f"void credit::k_resident<{kop}, {dt_num}, {reg}, {g['vpt'] - reg}>", g["grid"] * g["block"]


def precision_inputs(M, N, seed, dev):
    """The precision workload's rows on the GPU: x = 3 N(0,1) with exactly
    round(0.01 N) positions per row set to +-40 (random sign); FP32, BF16 and
    FP8-e4m3 copies (FP8: per-row scale amax / 448)."""
    import torch

    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    x = 3.0 * torch.randn((M, N), generator=g, device=dev)
    k = int(round(0.01 * N))
    pos = torch.rand((M, N), generator=g, device=dev).topk(k, dim=1).indices
    sign = torch.where(torch.rand((M, k), generator=g, device=dev) < 0.5, -40.0, 40.0)
    x.scatter_(1, pos, sign)
    del pos, sign
    xs = x.abs().amax(dim=1) / 448.0
    codes = (x / xs[:, None]).clamp(-448.0, 448.0).to(torch.float8_e4m3fn).view(torch.uint8)
    return {"f32": (x, None), "bf16": (x.to(torch.bfloat16), None), "fp8": (codes, xs.contiguous())}


def time_cold(fn, flush, reps=15, warm=3):
    """Median of `reps` runs of fn() between HIP events on torch's current
    stream (the stream the binding launches on), each after writing a 512 MiB
    buffer so the inputs come from HBM."""
    import torch

    st = torch.cuda.current_stream()
    t = []
    for r in range(warm + reps):
        flush.fill_(r)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn()
        e1.record(st)
        e1.synchronize()
        if r >= warm:
            t.append(e0.elapsed_time(e1) * 1e3)
    t.sort()
    return t[len(t) // 2] if len(t) % 2 else 0.5 * (t[len(t) // 2 - 1] + t[len(t) // 2])


def forms(C, h):
    """The precision workload (softmax and LayerNorm forward, M = 4096, N in
    {65536, 262144}, BF16 and FP8 I/O next to FP32, each against the FP32
    two-pass kernel) timed on its own rows (3 N(0,1) with 1% at +-40), cold
    cache, median of 15; GB/s on algorithmic bytes (rows in and out, FP8 row
    scales in and out, gamma / beta once, mean / rstd out).  Then the
    backward workload (softmax and LayerNorm backward, M = 2048,
    N = 131072, FP32 and BF16) and the LayerNorm -> e4m3 fusion, with the
    selector's plans."""
    import torch

    dev = torch.device("cuda:0")
    out = {"precision": [], "backward": []}
    e = {C.F32: 4, C.BF16: 2, C.FP8: 1}
    dnum = {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}
    flush = torch.empty(512 << 20, dtype=torch.uint8, device=dev)
    for N in (65536, 262144):
        M = 4096
        data = precision_inputs(M, N, seed=2 + N, dev=dev)
        g = torch.rand(N, device=dev) + 0.5
        b = 0.1 * torch.randn(N, device=dev)
        for op, name in ((C.SOFTMAX, "softmax_fwd"), (C.LAYERNORM, "layernorm_fwd")):
            def runner(dn, p):
                x, xs = data[dn]
                y = torch.empty_like(x)
                ys = torch.empty(M, device=dev) if dn == "fp8" else None
                if op == C.SOFTMAX:
                    return lambda: C.softmax_fwd(x, xs, p=p, out=y, out_scale=ys, h=h)
                return lambda: C.layernorm_fwd(x, g, b, EPS, xs, p=p, out=y, h=h)

            def alg(dn):
                nb = M * N * e[dnum[dn]] * 2 + (M * 8 if dn == "fp8" else 0)
                return nb + (N * 8 + M * 8 if op == C.LAYERNORM else 0)

            t2 = time_cold(runner("f32", C.plan("two_pass")), flush)
            row = {"op": name, "M": M, "N": N, "fp32_two_pass_us": round(t2, 1)}
            for dn in ("f32", "bf16", "fp8"):
                p, _ = h.select(op, C.FWD, dnum[dn], M, N)
                t = time_cold(runner(dn, p), flush)
                row[dn] = {"plan": list(p.as_tuple()), "us": round(t, 1), "gbps": round(alg(dn) / (t * 1e3), 1),
                           "speedup_vs_fp32_two_pass": round(t2 / t, 3)}
            out["precision"].append(row)
            log(f"precision {name} N={N}: {row}")
        del data
    del flush
    for op, name in ((C.SOFTMAX, "softmax_bwd"), (C.LAYERNORM, "layernorm_bwd")):
        M, N = 2048, 131072
        for dt, dn in ((C.F32, "f32"), (C.BF16, "bf16")):
            p, _ = h.select(op, C.BWD, dt, M, N)
            t = h.time_plan(op, C.BWD, dt, M, N, p, 15, True)
            t2 = h.time_plan(op, C.BWD, dt, M, N, C.plan("two_pass"), 15, True)
            out["backward"].append({"op": name, "dtype": dn, "M": M, "N": N, "plan": list(p.as_tuple()),
                                    "us": round(t, 1), "gbps": round(M * N * e[dt] * 3 / (t * 1e3), 1),
                                    "two_pass_us": round(t2, 1)})
            log(f"backward {name} {dn}: {out['backward'][-1]}")
    # LayerNorm -> e4m3 fusion: the fused operator against LayerNorm (FP32
    # out) followed by the row quantisation op, FP32 input, M = 4096
    out["fusion"] = []
    for N in (65536, 262144):
        M = 4096
        pf, _ = h.select(C.LAYERNORM_FP8_OUT, C.FWD, C.F32, M, N)
        tf = h.time_plan(C.LAYERNORM_FP8_OUT, C.FWD, C.F32, M, N, pf, 15, True)
        pl, _ = h.select(C.LAYERNORM, C.FWD, C.F32, M, N)
        tl = h.time_plan(C.LAYERNORM, C.FWD, C.F32, M, N, pl, 15, True)
        pq, _ = h.select(C.QUANT_FP8, C.FWD, C.F32, M, N)
        tq = h.time_plan(C.QUANT_FP8, C.FWD, C.F32, M, N, pq, 15, True)
        out["fusion"].append({"M": M, "N": N, "fused_plan": list(pf.as_tuple()), "fused_us": round(tf, 1),
                              "fused_gbps": round(M * N * 5 / (tf * 1e3), 1),
                              "unfused_us": round(tl + tq, 1), "speedup": round((tl + tq) / tf, 3)})
        log(f"fusion N={N}: {out['fusion'][-1]}")
    return out


def single(C, h, args):
    """One forward workload alone (rows as the precision workload draws them:
    3 N(0,1) with 1% at +-40), `warmup` untimed and `steps` timed launches
    between HIP events on the launch stream, one 1 GiB copy launch first (the
    traffic counters' calibration).  Returns the JSON the counter summaries
    read: the launch's kernel, grid, average duration and algorithmic bytes."""
    import torch

    op_name, dn, M, N = args.single.split(":")
    M, N = int(M), int(N)
    op = {"softmax_fwd": C.SOFTMAX, "layernorm_fwd": C.LAYERNORM, "rmsnorm_fwd": C.RMSNORM}[op_name]
    dnum = {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}[dn]
    dev = torch.device("cuda:0")
    x, xs = precision_inputs(M, N, seed=2 + N, dev=dev)[dn]
    g = torch.rand(N, device=dev) + 0.5
    b = 0.1 * torch.randn(N, device=dev)
    y = torch.empty_like(x)
    ys = torch.empty(M, device=dev) if dn == "fp8" else None
    if args.plan:
        var, k = args.plan.split(":")
        p = C.plan(var, int(k))
    else:
        p, _ = h.select(op, C.FWD, dnum, M, N)

    def call():
        if op == C.SOFTMAX:
            C.softmax_fwd(x, xs, p=p, out=y, out_scale=ys, h=h)
        elif op == C.LAYERNORM:
            C.layernorm_fwd(x, g, b, EPS, xs, p=p, out=y, h=h)
        else:
            C.rmsnorm_fwd(x, g, EPS, xs, p=p, out=y, h=h)

    h.copy_bandwidth(1 << 30, 1)
    for _ in range(max(args.warmup, 1)):
        call()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream(dev)
    ev = []
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        call()
        e1.record(st)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    assert h.check_errors() == C.OK
    us = 1e3 * sum(a.elapsed_time(c) for a, c in ev) / len(ev)
    e = {C.F32: 4, C.BF16: 2, C.FP8: 1}[dnum]
    # rows in and out, FP8 row scales in and out, gamma / beta once, statistics out
    nb = M * N * e * 2 + (M * 8 if dn == "fp8" else 0)
    nb += {C.SOFTMAX: 0, C.LAYERNORM: N * 8 + M * 8, C.RMSNORM: N * 4 + M * 4}[op]
    sym, grid = kernel_symbol(C, h, op, dnum, M, N, p)
    key = f"{op_name}:{dn}:M={M}:N={N}:plan={int(p.variant)},{int(p.k)}"
    return {"metric": "single-workload launch sequence", "value": round(nb / (us * 1e3), 1), "unit": "GB/s",
            "steps": args.steps, "warmup": args.warmup, "data": "synthetic", "dtype": dn,
            "config": {"workload": key}, "source_hash": source_hash(), "copy_kernel_bytes": 1 << 30,
            "roofline": {"bound": "hbm", "kernel": key, "kernel_symbol": sym, "grid_threads": grid,
                         "avg_launch_us": round(us, 2), "algorithmic_bytes_per_launch": nb,
                         "elements_per_launch": M * N, "achieved": round(nb / (us * 1e3), 1),
                         "peak": PEAK_GBPS, "unit": "GB/s", "frac": round(nb / (us * 1e3) / PEAK_GBPS, 4)}}


SUITE = (("layernorm_bwd", "LAYERNORM", "BWD", 2048), ("wvar_bwd", "WVAR", "BWD", 4096),
         ("pearson_bwd", "PEARSON", "BWD", 4096), ("softmax_logits_bwd", "SOFTMAX_LOGITS", "BWD", 4096),
         ("quant_int8", "QUANT_INT8", "FWD", 4096))
SUITE_N = (4096, 8192, 16384, 32768, 65536)


TRAFFIC_REPS = 3
TRAFFIC_CALIB_BYTES = 1 << 30


def _legal_splits(C, h, op, d, M, N):
    """Every legal split-row plan, so that the launch sequence (and the
    block each counter reading belongs to) is the same in every profiled
    run: timing under the profiler would not pick the same plan twice."""
    return tuple(("split", k) for k in (2, 4, 8, 16, 32)
                 if h.plan_legal(op, d, C.F32, M, N, C.plan("split", k)))


def _traffic_blocks(C, h, items, mode):
    """Launches each (workload, op, direction, M, N, plans) item's plans
    3 + TRAFFIC_REPS times with a cache flush before each launch, every plan
    behind a marker (a small copy-kernel launch whose size names the block),
    after a 1 GiB copy that calibrates the counters.  Meant to run under
    `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE); the JSON it returns tells
    the summary which block is which."""
    h.copy_bandwidth(TRAFFIC_CALIB_BYTES, 1)
    blocks = []
    for name, op, d, M, N, plans in items:
        w = C.workload_info(op, d, C.F32)
        for variant, k in plans:
            marker = 4096 * (1 + len(blocks))
            h.copy_bandwidth(marker, 1)
            h.time_plan(op, d, C.F32, M, N, C.plan(variant, k), TRAFFIC_REPS, True)
            blocks.append({"workload": name, "M": M, "N": N, "variant": variant, "k": k,
                           "marker_threads": marker // 16, "launches": 3 + TRAFFIC_REPS,
                           "algorithmic_bytes": M * N * (w.b_base if variant == "two_pass" else w.b_staged)})
    return {"mode": mode, "source_hash": source_hash(), "copy_kernel_bytes": TRAFFIC_CALIB_BYTES,
            "copy_threads": TRAFFIC_CALIB_BYTES // 16, "blocks": blocks}


def traffic_suite(C, h):
    """Launch sequence for the traffic validation of Sec. IV-E (the paper's
    DRAM-traffic figure at N = 65536): for every suite workload, the two-pass
    baseline and every legal split-row plan."""
    N = max(SUITE_N)
    items = []
    for name, opn, dirn, M in SUITE:
        op, d = getattr(C, opn), getattr(C, dirn)
        items.append((name, op, d, M, N, (("two_pass", 1),) + _legal_splits(C, h, op, d, M, N)))
    return _traffic_blocks(C, h, items, "traffic_suite")


def traffic_plans(C, h):
    """Launch sequence for the traffic of every variant on the bandwidth
    workload (FP32 LayerNorm / RMSNorm forward, M = 1024 rows, each width):
    the two-pass baseline, the row-resident kernel where the row fits one
    workgroup, and every legal split-row plan, so the counters show where
    the reread of the two-pass kernel reaches HBM and where a cache serves
    it."""
    items = []
    for name in OPS:
        op = C.LAYERNORM if name == "layernorm_fwd" else C.RMSNORM
        for N in WIDTHS:
            plans = (("two_pass", 1),)
            if h.plan_legal(op, C.FWD, C.F32, M_ROWS, N, C.plan("resident")):
                plans += (("resident", 1),)
            items.append((name, op, C.FWD, M_ROWS, N, plans + _legal_splits(C, h, op, C.FWD, M_ROWS, N)))
    return _traffic_blocks(C, h, items, "traffic_plans")


def suite(C, h, copy_gbps):
    """The paper's evaluation suite on this GPU (Sec. IV-A: FP32 input, M =
    2048 for LayerNorm and 4096 otherwise, N in 4K..64K; LayerNorm backward
    with saved statistics here): cold-cache times of every legal plan, the
    speedup of the best split-row plan over the best single-workgroup
    baseline, and the profitability question of the model validation
    (Sec. IV-D, Table V): is the split-row plan faster than the baseline the
    model is given (row-resident if the row fits one workgroup, else
    two-pass)?  Answered by Eq. (9) with the measured baseline time (Eq. (7))
    and, as the ablation, with the baseline priced at copy bandwidth plus a
    serialized deposit."""
    rows, acc, acc_peak, acc_res, n = [], 0, 0, 0, 0
    for name, opn, dirn, M in SUITE:
        op, d = getattr(C, opn), getattr(C, dirn)
        w = C.workload_info(op, d, C.F32)
        for N in SUITE_N:
            t = {}
            for c in range(C.NUM_PLANS):
                p = C.plan_of_class(c)
                if h.plan_legal(op, d, C.F32, M, N, p):
                    t[p.as_tuple()] = h.time_plan(op, d, C.F32, M, N, p, 15, True)
            base = (C.ROW_RESIDENT, 1) if (C.ROW_RESIDENT, 1) in t else (C.TWO_PASS, 1)
            single = min(v for k, v in t.items() if k[0] != C.SPLIT_ROW)
            splits = {k: v for k, v in t.items() if k[0] == C.SPLIT_ROW}
            ks = [2, 4, 8, 16, 32]
            c1 = h.time_control(op, d, C.F32, M, N, 1, 7)
            ctrl = [max(0.0, h.time_control(op, d, C.F32, M, N, k, 7) - c1) if (C.SPLIT_ROW, k) in splits else 0.0
                    for k in ks]
            delta = C.model_delta(h, op, d, C.F32, M, N, t[base], ctrl)
            tb_peak = M * N * w.b_base / (copy_gbps * 1e3)
            dep = M * N * w.b_keep / (copy_gbps * 1e3)
            delta_peak = [x - dep for x in C.model_delta(h, op, d, C.F32, M, N, tb_peak, ctrl)]
            row = {"workload": name, "M": M, "N": N,
                   "plans_us": {f"{v},{k}": round(x, 2) for (v, k), x in t.items()},
                   "baseline_plan": list(base), "baseline_us": round(t[base], 2), "best_single_us": round(single, 2)}
            if splits:
                kb, tbest = min(splits.items(), key=lambda kv: kv[1])
                meas = bool(tbest < t[base])
                pred = bool(max(delta) > 0)
                pred_peak = bool(max(delta_peak) > 0)
                # the other reading of b_reread: a row-resident baseline rereads
                # nothing from HBM, so T_save = 0 and Eq. (9) never favours a split
                pred_res = pred if base[0] == C.TWO_PASS else False
                n += 1
                acc += pred == meas
                acc_peak += pred_peak == meas
                acc_res += pred_res == meas
                row.update(best_split=list(kb), best_split_us=round(tbest, 2),
                           speedup_vs_best_single=round(single / tbest, 3),
                           gbps_best=round(M * N * w.b_staged / (min(tbest, single) * 1e3), 1),
                           measured_profitable=meas, predicted_profitable=pred, predicted_profitable_peak=pred_peak,
                           predicted_profitable_resident_no_reread=pred_res)
            rows.append(row)
            log(f"suite {name} N={N}: {row}")
    # crossover width N*: the narrowest swept width from which the split-row
    # plan stays ahead of the baseline (measured, and as the model predicts)
    cross = {}
    for name, _, _, _ in SUITE:
        rs = [r for r in rows if r["workload"] == name and "measured_profitable" in r]

        def nstar(key):
            ok = [r["N"] for i, r in enumerate(rs) if all(x[key] for x in rs[i:])]
            return min(ok) if ok else None

        cross[name] = {"measured": nstar("measured_profitable"), "model": nstar("predicted_profitable"),
                       "peak_model": nstar("predicted_profitable_peak")}
    # the headline of Sec. IV-B: geometric-mean speedup of the best split-row
    # plan over the best single-workgroup plan at the widest swept N
    nmax = max(SUITE_N)
    sp = [r["speedup_vs_best_single"] for r in rows if r["N"] == nmax and "speedup_vs_best_single" in r]
    gm = round(math.exp(sum(math.log(x) for x in sp) / len(sp)), 3) if sp else None
    return {"rows": rows, "profitability_pairs": n, "model_correct": acc, "peak_model_correct": acc_peak,
            "resident_no_reread_model_correct": acc_res,
            "crossover_N": cross, "geomean_speedup_at_widest_N": {"N": nmax, "workloads": len(sp), "speedup": gm}}


def traffic_for(kernel_key: str):
    """Counter-measured HBM bytes per launch for the dominant kernel, if the
    committed profile was taken from the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
        ent = d.get("kernels", {}).get(kernel_key)
        if ent and ent.get("source_hash") == source_hash():
            return ent.get("bytes_per_launch")
    except Exception:
        return None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-regret", action="store_true", help="skip exhaustive timing of all plans")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision / backward workloads")
    ap.add_argument("--no-suite", action="store_true", help="skip the evaluation-suite workloads")
    ap.add_argument("--selector", default="auto", choices=["auto", "learned", "learned_timed", "analytic", "fixed", "exhaustive"])
    ap.add_argument("--traffic-suite", action="store_true",
                    help="only the launch sequence of the suite traffic validation (run under rocprofv3 --pmc)")
    ap.add_argument("--traffic-plans", action="store_true",
                    help="only the launch sequence of every variant's traffic on the bandwidth workload "
                         "(run under rocprofv3 --pmc)")
    ap.add_argument("--single", default=None, metavar="OP:DTYPE:M:N",
                    help="only one forward workload (softmax_fwd | layernorm_fwd | rmsnorm_fwd, f32 | bf16 | fp8) "
                         "with the precision workload's rows, timed alone: the launch sequence a counter "
                         "profile of that kernel runs under")
    ap.add_argument("--plan", default=None, help="--single: plan as variant:k (default: the selector's)")
    ap.add_argument("--dominant", default=None, metavar="OP:N",
                    help="report the roofline for this shape (e.g. layernorm_fwd:524288) instead of the longest "
                         "launch, so that counter runs of two launches of nearly equal length name the same kernel")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the row kernels shard over rows with no communication, "
              "so a multi-GPU figure is not measured here", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_01864_amd import credit as C
    from paper_2609_01864_amd import tune as T

    dev = torch.device("cuda:0")
    h = C.Handle(0)
    sel_name = args.selector
    if sel_name == "auto":
        sel_name = "learned_timed" if h.model_loaded else "analytic"
    sel = {"learned": C.SEL_LEARNED, "learned_timed": C.SEL_LEARNED_TIMED, "analytic": C.SEL_ANALYTIC,
           "fixed": C.SEL_FIXED, "exhaustive": C.SEL_EXHAUSTIVE}[sel_name]
    h.set_selector(sel)
    log(f"selector={sel_name} model_loaded={h.model_loaded}")
    if args.traffic_suite:
        print(json.dumps(traffic_suite(C, h)), flush=True)
        return
    if args.traffic_plans:
        print(json.dumps(traffic_plans(C, h)), flush=True)
        return
    if args.single:
        print(json.dumps(single(C, h, args)), flush=True)
        return

    # ---------------------------------------------------------------- inputs
    gen = torch.Generator(device=dev)
    gen.manual_seed(1)
    bufs = {}
    for op in OPS:
        for N in WIDTHS:
            x = torch.randn((M_ROWS, N), generator=gen, device=dev, dtype=torch.float32) + 10.0
            gamma = torch.rand((N,), generator=gen, device=dev) + 0.5
            beta = 0.1 * torch.randn((N,), generator=gen, device=dev)
            y = torch.empty_like(x)
            mean = torch.empty(M_ROWS, device=dev)
            rstd = torch.empty(M_ROWS, device=dev)
            bufs[(op, N)] = (x, gamma, beta, y, mean, rstd)
    torch.cuda.synchronize()
    log("inputs ready")

    # ------------------------------------------------------ plan selection
    opnum = {"layernorm_fwd": C.LAYERNORM, "rmsnorm_fwd": C.RMSNORM}
    picks = {}
    t0 = time.time()
    for op in OPS:
        for N in WIDTHS:
            p, pred = h.select(opnum[op], C.FWD, C.F32, M_ROWS, N)
            picks[(op, N)] = (p, pred)
            log(f"pick {op} N={N}: {p} (predicted {pred:.1f} us)")
    sel_s = time.time() - t0

    stream = torch.cuda.current_stream(dev)

    def call(op, N):
        x, g, b, y, mean, rstd = bufs[(op, N)]
        p = picks[(op, N)][0]
        if op == "layernorm_fwd":
            C.layernorm_fwd(x, g, b, EPS, p=p, out=y, h=h)
        else:
            C.rmsnorm_fwd(x, g, EPS, p=p, out=y, h=h)

    # workspaces are sized on first use, outside the timed region
    for op in OPS:
        for N in WIDTHS:
            call(op, N)
    torch.cuda.synchronize()
    assert h.check_errors() == C.OK

    for _ in range(args.warmup):
        for op in OPS:
            for N in WIDTHS:
                call(op, N)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # ------------------------------------------------------------ timed
    events = {(op, N): [] for op in OPS for N in WIDTHS}
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        for op in OPS:
            for N in WIDTHS:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                call(op, N)
                e1.record(stream)
                events[(op, N)].append((e0, e1))
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    assert h.check_errors() == C.OK
    wall_ms = (t_end - t_start) * 1e3
    ms_per_step = wall_ms / args.steps
    step_bytes = sum(algorithmic_bytes(op, M_ROWS, N) for op in OPS for N in WIDTHS)
    value = step_bytes / (ms_per_step * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, {value:.1f} GB/s")

    per_shape = []
    for op in OPS:
        for N in WIDTHS:
            us = 1e3 * sum(a.elapsed_time(b) for a, b in events[(op, N)]) / len(events[(op, N)])
            gb = algorithmic_bytes(op, M_ROWS, N) / (us * 1e-6) / 1e9
            p = picks[(op, N)][0]
            g = h.geometry(opnum[op], C.FWD, C.F32, M_ROWS, N, p)
            per_shape.append({"op": op, "N": N, "plan": [int(p.variant), int(p.k)], "us": round(us, 2),
                              "gbps": round(gb, 1), "frac": round(gb / PEAK_GBPS, 4),
                              # launch shape: workgroups, co-resident workgroups per CU
                              # (runtime occupancy) and 16-byte vectors per thread
                              "geometry": {"grid": g["grid"], "per_cu": g["per_cu"], "vpt": g["vpt"],
                                           "rows": g["rows"]}})
    dom = max(per_shape, key=lambda r: r["us"])
    if args.dominant:
        dop, dn = args.dominant.split(":")
        dom = next(r for r in per_shape if r["op"] == dop and r["N"] == int(dn))
    dom_key = f"{dom['op']}:N={dom['N']}:plan={dom['plan'][0]},{dom['plan'][1]}"
    sym, grid_threads = kernel_symbol(C, h, opnum[dom["op"]], C.F32, M_ROWS, dom["N"], picks[(dom["op"], dom["N"])][0])
    roofline = {"bound": "hbm", "achieved": dom["gbps"], "peak": PEAK_GBPS, "unit": "GB/s",
                "frac": round(dom["gbps"] / PEAK_GBPS, 4), "traffic": traffic_for(dom_key),
                "kernel": dom_key, "kernel_symbol": sym, "grid_threads": grid_threads,
                "avg_launch_us": dom["us"],
                "algorithmic_bytes_per_launch": algorithmic_bytes(dom["op"], M_ROWS, dom["N"])}

    # --------------------------------------------- regret vs exhaustive
    regrets, regrets_na = [], []
    if not args.no_regret:
        for r in per_shape:
            o = opnum[r["op"]]
            best = None
            times, rec = {}, {"times": {}, "spread": {}}
            for c in range(C.NUM_PLANS):
                p = C.plan_of_class(c)
                if not h.plan_legal(o, C.FWD, C.F32, M_ROWS, r["N"], p):
                    continue
                st = h.time_plan_stats(o, C.FWD, C.F32, M_ROWS, r["N"], p, reps=15, flush=True)
                t = st["median_us"]
                times[f"{p.variant},{p.k}"] = round(t, 2)
                rec["times"][str(c)] = t
                rec["spread"][str(c)] = {"mad": st["mad_us"], "min": st["min_us"], "p90": st["p90_us"]}
                if best is None or t < best[1]:
                    best = (p, t)
            pk = picks[(r["op"], r["N"])][0]
            tp = times[f"{pk.variant},{pk.k}"]
            cls = {C.plan_of_class(c).as_tuple(): c for c in range(C.NUM_PLANS)}
            ra = T.regret_stats([rec], [cls[pk.as_tuple()]])
            r["plan_times_us"] = times
            r["plan_mad_us"] = {f"{C.plan_of_class(int(c)).variant},{C.plan_of_class(int(c)).k}": round(v["mad"], 2)
                                for c, v in rec["spread"].items()}
            r["best_plan"] = [int(best[0].variant), int(best[0].k)]
            jb = C.plan_of_class(T.judge_best(rec))
            r["judge_plan"] = [int(jb.variant), int(jb.k)]
            r["regret"] = round(tp / best[1] - 1.0, 4)
            r["regret_noise_aware"] = round(ra["noise_aware_geomean"] - 1.0, 4)
            regrets.append(tp / best[1])
            regrets_na.append(ra["noise_aware_geomean"])
            if h.model_loaded:  # the network's own first choice, before any timing
                h.set_selector(C.SEL_LEARNED)
                pu = h.select(o, C.FWD, C.F32, M_ROWS, r["N"])[0]
                h.set_selector(sel)
                r["learned_untimed_plan"] = [int(pu.variant), int(pu.k)]
                r["learned_untimed_regret"] = round(times[f"{pu.variant},{pu.k}"] / best[1] - 1.0, 4)
                r["learned_untimed_regret_noise_aware"] = round(
                    T.regret_stats([rec], [cls[pu.as_tuple()]])["noise_aware_geomean"] - 1.0, 4)
            log(f"{r['op']} N={r['N']}: times {times} pick {r['plan']} regret {r['regret']:+.3f}")
    copy_gbps = h.copy_bandwidth(1 << 30, 15)
    log(f"copy kernel: {copy_gbps:.1f} GB/s")
    extra = None if args.no_forms else forms(C, h)
    suite_res = None if args.no_suite else suite(C, h, copy_gbps)
    prims = h.probe_primitives(15)
    log(f"primitives: {prims}")

    cpu = None
    if not args.no_cpu:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline()

    out = {
        "metric": "HBM GB/s and % of 8 TB/s peak per op/shape; cost-model pick regret vs best",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "FP32 LayerNorm + RMSNorm forward, eps 1e-5, M=1024, N in {8192, 32768, 131072, "
                               "524288}, x~N(10,1), gamma~U(0.5,1.5), beta~N(0,0.1)",
                   "M": M_ROWS, "N": list(WIDTHS), "selector": sel_name,
                   "selection_s": round(sel_s, 2)},
        "frac_of_peak": round(value / PEAK_GBPS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "regret_geomean": round(math.exp(sum(math.log(x) for x in regrets) / len(regrets)) - 1.0, 4)
        if regrets else None,
        "regret_geomean_noise_aware": round(math.exp(sum(math.log(x) for x in regrets_na) / len(regrets_na)) - 1.0,
                                            4) if regrets_na else None,
        "regret_geomean_learned_untimed_noise_aware": round(math.exp(sum(
            math.log(1.0 + r["learned_untimed_regret_noise_aware"]) for r in per_shape) / len(per_shape)) - 1.0, 4)
        if per_shape and all("learned_untimed_regret_noise_aware" in r for r in per_shape) else None,
        "regret_geomean_learned_untimed": round(math.exp(sum(math.log(1.0 + r["learned_untimed_regret"])
                                                             for r in per_shape) / len(per_shape)) - 1.0, 4)
        if per_shape and all("learned_untimed_regret" in r for r in per_shape) else None,
        "copy_kernel_gbps": round(copy_gbps, 1),
        "copy_kernel_bytes": 1 << 30,
        "per_shape": per_shape,
        "forms": extra,
        "paper_suite": suite_res,
        "primitives": prims,
        "source_hash": source_hash(),
        "device": device_identity(torch),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
