"""Split-row exchange protocol: bounded waits end in CREDIT_ERR_TIMEOUT when a
member never publishes (forced from the host: a test-only flag plus a tiny
spin limit, so every kernel still exits normally), epoch wrap-around, a
workspace poisoned with stale epochs, and run-to-run determinism."""
import numpy as np
import pytest
import torch

from paper_2609_01864_amd import credit as C

from _cases import Case, check_case

pytestmark = pytest.mark.gpu


def _ln_case():
    case = Case("layernorm_fwd", "f32", 40, 30000, seed=21)
    return case, case.reference()


def test_missing_partial_times_out_and_is_reported(gpu_handle):
    case, ref = _ln_case()
    h = gpu_handle
    assert h.check_errors() == C.OK
    h.set_option(C.OPT_SPIN_LIMIT, 64)
    h.set_option(C.OPT_TEST_DROP_PUBLISH, 1)
    try:
        print("[protocol] forced timeout", flush=True)
        x = torch.from_numpy(case.raw["x"][0]).cuda()
        g = torch.from_numpy(case.gamma).cuda()
        b = torch.from_numpy(case.beta).cuda()
        C.layernorm_fwd(x, g, b, 1e-5, p=C.plan("split", 4), h=h)
        torch.cuda.synchronize()
        assert h.check_errors() == C.ERR_TIMEOUT
        assert h.check_errors() == C.OK  # the flag is cleared once reported
    finally:
        h.set_option(C.OPT_TEST_DROP_PUBLISH, 0)
        h.set_option(C.OPT_SPIN_LIMIT, 1 << 22)
    # the library is usable again afterwards
    check_case(case, case.run(h, C.plan("split", 4), ref=ref), ref)


def test_epoch_wraparound(gpu_handle):
    case, ref = _ln_case()
    C.set_epoch(0xFFFFFFFE)
    for _ in range(4):  # epochs 0xFFFFFFFE, 0xFFFFFFFF, (0 skipped) 1, 2
        print("[protocol] epoch wrap", flush=True)
        check_case(case, case.run(gpu_handle, C.plan("split", 8), ref=ref), ref)


def test_poisoned_workspace(gpu_handle):
    # stale slot words from earlier launches (random epochs and values) must not
    # be taken for the current launch's partials
    case, ref = _ln_case()
    h = gpu_handle
    p = C.plan("split", 8)
    n = h.workspace_size(C.LAYERNORM, C.FWD, C.F32, case.M, case.N, p)
    ws = h.workspace(n, h._stream())
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    ws.copy_(torch.randint(0, 256, ws.shape, generator=gen, dtype=torch.uint8, device="cuda"))
    C.set_epoch(0x7FFFFFF0)
    print("[protocol] poisoned workspace", flush=True)
    check_case(case, case.run(h, p, ref=ref), ref)


def test_determinism_across_runs_and_plans_agree(gpu_handle):
    case = Case("softmax_fwd", "bf16", 16, 65536, seed=8)
    outs = {}
    for v, k in [("split", 2), ("split", 4), ("split", 8), ("split", 16)]:
        runs = [case.run(gpu_handle, C.plan(v, k))["y"] for _ in range(3)]
        assert all(np.array_equal(runs[0], r) for r in runs[1:]), (v, k)
        outs[k] = runs[0]
    # different split factors combine in different orders: equal to 1 BF16 ulp
    ref = case.reference()
    for k, y in outs.items():
        check_case(case, {"y": y}, ref)


def test_primitive_probes(gpu_handle):
    # the primitive table: every bounded wait completed, latencies ordered as
    # the memory hierarchy (LDS < L2 hit < a handoff through device memory),
    # exchange rounds grow with the row group, rates are positive
    p = gpu_handle.probe_primitives(reps=5)
    print(p, flush=True)
    assert p["errors"] == 0
    assert 0 < p["lds_load_ns"] < p["l2_load_ns"] < p["handoff_cross_xcd_ns"]
    assert 0 < p["handoff_same_xcd_ns"] and 0 < p["barrier_ns"]
    ex = p["exchange_ns"]
    assert 0 < ex["k2"] <= ex["k32"]
    assert min(p["lds_read_bpc"], p["lds_write_bpc"], p["l2_read_bpc"], p["global_write_bpc"]) > 0
    assert p["clock_mhz"] > 50
    assert gpu_handle.check_errors() == C.OK


@pytest.mark.parametrize("op,dtype", [("layernorm_fwd", "f32"), ("softmax_fwd", "bf16"), ("layernorm_bwd", "f32"),
                                      ("rmsnorm_fwd", "fp8")])
def test_exchange_under_member_skew(gpu_handle, op, dtype):
    # test-only skew: before each exchange, member c of row r waits
    # (7 c + r) % 13 microseconds, so members publish out of step and some
    # reach their wait long before the others publish (Sec. III-C: the
    # exchange must not depend on arrival order).  Every split factor: the
    # skewed run matches the oracle and is bitwise equal to the unskewed run.
    # Waits stay bounded (the default spin limit), so every kernel exits.
    h = gpu_handle
    case = Case(op, dtype, 48, 65536, seed=77)
    ref = case.reference()
    main = "y" if op.endswith("fwd") else "dx"
    for k in (2, 4, 8, 16, 32):
        p = C.plan("split", k)
        if not h.plan_legal(*{"layernorm_fwd": (C.LAYERNORM, C.FWD), "softmax_fwd": (C.SOFTMAX, C.FWD),
                              "layernorm_bwd": (C.LAYERNORM, C.BWD), "rmsnorm_fwd": (C.RMSNORM, C.FWD)}[op],
                            {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}[dtype], case.M, case.N, p):
            continue
        plain = case.run(h, p, ref=ref)
        h.set_option(C.OPT_TEST_SKEW, 1)
        try:
            print(f"[protocol] skew {op} {dtype} k={k}", flush=True)
            skewed = case.run(h, p, ref=ref)
        finally:
            h.set_option(C.OPT_TEST_SKEW, 0)
        assert h.check_errors() == C.OK
        check_case(case, skewed, ref)
        assert np.array_equal(plain[main], skewed[main]), f"k={k}: skew changed the result"
        if op == "layernorm_bwd":
            assert np.array_equal(plain["dgamma"], skewed["dgamma"]) and np.array_equal(plain["dbeta"],
                                                                                     skewed["dbeta"])
