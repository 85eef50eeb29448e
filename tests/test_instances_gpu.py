"""Parity of every compiled kernel instance: each row-resident / split-row
instance (operator x I/O dtype x vectors per thread) in both of its row loops,
and each two-pass instance (operator x dtype x workgroup size), element-wise
against the FP64 oracle.

A row-resident / split-row instance is reached through the plan and width that
resolve to it (the library reports the vectors per thread of a plan): with a
split factor k and N = k * VPT * 256 * EPV every member holds exactly VPT full
vectors per thread and runs the unmasked loop; five elements fewer leave the
last member a ragged slice, which runs the masked loop.  k = 2 exercises the
exchange; k = 1 (row-resident) at the full width covers the path without it.
The set of instances covered must equal the set the library instantiates."""
import numpy as np
import pytest

from paper_2609_01864_amd import credit as C

from _cases import Case, check_case
from test_workloads_gpu import WCase, check as wcheck

pytestmark = pytest.mark.gpu

VPTS = (1, 2, 4, 8, 12, 16, 24, 32, 48, 68)
BYTES = {"f32": 4, "bf16": 2, "fp8": 1}
DTN = {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}
# name, (op, direction), I/O dtypes, case family
OPS = [("softmax_fwd", (C.SOFTMAX, C.FWD), ("f32", "bf16", "fp8"), "core"),
       ("layernorm_fwd", (C.LAYERNORM, C.FWD), ("f32", "bf16", "fp8"), "core"),
       ("rmsnorm_fwd", (C.RMSNORM, C.FWD), ("f32", "bf16", "fp8"), "core"),
       ("softmax_bwd", (C.SOFTMAX, C.BWD), ("f32", "bf16", "fp8"), "core"),
       ("layernorm_bwd", (C.LAYERNORM, C.BWD), ("f32", "bf16", "fp8"), "core"),
       ("rmsnorm_bwd", (C.RMSNORM, C.BWD), ("f32", "bf16", "fp8"), "core"),
       ("smxl", (C.SOFTMAX_LOGITS, C.BWD), ("f32", "bf16", "fp8"), "work"),
       ("quant_int8", (C.QUANT_INT8, C.FWD), ("f32", "bf16"), "work"),
       ("quant_fp8", (C.QUANT_FP8, C.FWD), ("f32", "bf16"), "work"),
       ("pearson", (C.PEARSON, C.BWD), ("f32", "bf16"), "work"),
       ("wvar", (C.WVAR, C.BWD), ("f32", "bf16"), "work"),
       ("lnq", (C.LAYERNORM_FP8_OUT, C.FWD), ("f32", "bf16"), "work")]


def _run_and_check(h, name, fam, dtype, M, N, plan, seed):
    if fam == "core":
        case = Case(name, dtype, M, N, seed=seed)
        ref = case.reference()
        check_case(case, case.run(h, plan, ref=ref), ref)
    else:
        case = WCase(name, dtype, M, N, seed=seed)
        wcheck(case, case.run(h, plan), case.reference())


def _instances(h):
    out = set()
    for name, (o, d), dts, _ in OPS:
        for dt in dts:
            for v in VPTS:
                if C.instance_info(h, o, d, DTN[dt], v) is not None:
                    out.add((name, dt, v))
    return out


@pytest.mark.parametrize("name,opdir,dtypes,fam", OPS, ids=[o[0] for o in OPS])
def test_every_resident_instance_both_row_loops(gpu_handle, name, opdir, dtypes, fam):
    h = gpu_handle
    o, d = opdir
    compiled = {i for i in _instances(h) if i[0] == name}
    covered = set()
    M = 3
    for dt in dtypes:
        epv = 16 // BYTES[dt]
        for v in VPTS:
            info = C.instance_info(h, o, d, DTN[dt], v)
            if info is None:
                continue
            runs = [("resident", 1, v * 256 * epv)]
            if info["coresident_per_cu"] != 0:  # split plans exist for it
                runs += [("split", 2, 2 * v * 256 * epv), ("split", 2, 2 * v * 256 * epv - 5)]
            for var, k, N in runs:
                p = C.plan(var, k)
                geo = C.plan_geometry(h, o, d, DTN[dt], M, N, p)
                assert geo is not None and geo["vpt"] == v, (name, dt, v, var, k, N, geo)
                print(f"[instance] {name} {dt} vpt={v} {var} k={k} N={N} info={info}", flush=True)
                _run_and_check(h, name, fam, dt, M, N, p, seed=v * 7 + k)
            covered.add((name, dt, v))
    assert covered == compiled and covered
    assert h.check_errors() == C.OK


@pytest.mark.parametrize("name,opdir,dtypes,fam", OPS, ids=[o[0] for o in OPS])
def test_every_two_pass_instance(gpu_handle, name, opdir, dtypes, fam):
    # the two-pass kernel runs 256-thread workgroups for rows of fewer than
    # 4096 vectors and 1024-thread workgroups from there
    h = gpu_handle
    o, d = opdir
    p = C.plan("two_pass")
    for dt in dtypes:
        epv = 16 // BYTES[dt]
        for N, block in ((1000, 256), (4096 * epv - 16 * epv, 256), (4096 * epv, 1024), (4096 * epv + 3, 1024)):
            geo = C.plan_geometry(h, o, d, DTN[dt], 3, N, p)
            assert geo is not None and geo["block"] == block, (name, dt, N, geo)
            print(f"[instance] {name} {dt} two-pass block={block} N={N}", flush=True)
            _run_and_check(h, name, fam, dt, 3, N, p, seed=N)
    assert h.check_errors() == C.OK


def test_private_memory_instances_are_probed(gpu_handle):
    # every instance whose code uses private memory carries a co-residency
    # verdict from the handle's creation, and its split plans never run more
    # workgroups per CU than verified
    h = gpu_handle
    probed = 0
    for name, (o, d), dts, _ in OPS:
        for dt in dts:
            epv = 16 // BYTES[dt]
            for v in VPTS:
                info = C.instance_info(h, o, d, DTN[dt], v)
                if info is None:
                    continue
                assert info["per_cu"] >= 1
                if info["private_bytes"] == 0:
                    assert info["coresident_per_cu"] == -1
                    continue
                probed += 1
                print(f"[probe] {name} {dt} vpt={v} {info}", flush=True)
                assert 0 <= info["coresident_per_cu"] <= info["per_cu"]
                for k in (2, 4, 8, 16, 32):
                    N = k * v * 256 * epv
                    geo = C.plan_geometry(h, o, d, DTN[dt], 100000, N, C.plan("split", k))
                    if geo is None or geo["vpt"] != v:
                        continue
                    assert geo["per_cu"] <= info["coresident_per_cu"]
    assert probed > 0
