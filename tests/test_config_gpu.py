"""Environment configuration read when a handle is created:
CREDIT_FORCE_PLAN, CREDIT_SELECTOR, CREDIT_SPIN_LIMIT, CREDIT_CHECKED and
CREDIT_LOG."""
import json

import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

pytestmark = pytest.mark.gpu


def test_forced_plan_used_where_legal(lib_built, monkeypatch):
    monkeypatch.setenv("CREDIT_FORCE_PLAN", "split:4")
    monkeypatch.setenv("CREDIT_SELECTOR", "fixed")
    h = C.Handle(0, load_default_model=False)
    try:
        p, pred = h.select(C.LAYERNORM, C.FWD, C.F32, 64, 20000)
        assert p.as_tuple() == (C.SPLIT_ROW, 4) and pred == -1.0
        # too wide for k = 4 slices: the selector decides instead
        p2, _ = h.select(C.LAYERNORM, C.FWD, C.F32, 8, 400000)
        assert p2.as_tuple() != (C.SPLIT_ROW, 4)
        assert h.plan_legal(C.LAYERNORM, C.FWD, C.F32, 8, 400000, p2)
        # an operator call without a plan runs the forced plan, correctly
        M, N = 37, 20000
        x64 = I.norm_rows(M, N, seed=9)
        g32, b32 = I.norm_params(N, seed=9)
        x = torch.from_numpy(x64.astype(np.float32)).cuda()
        y, _, _, _ = C.layernorm_fwd(x, torch.from_numpy(g32).cuda(), torch.from_numpy(b32).cuda(), 1e-5, h=h)
        ref, _, _ = oracle.layernorm_fwd(x64.astype(np.float32).astype(np.float64), g32.astype(np.float64),
                                         b32.astype(np.float64), 1e-5)
        assert np.max(np.abs(y.double().cpu().numpy() - ref)) <= 1e-5
        assert h.check_errors() == C.OK
    finally:
        h.close()


def test_unrecognised_values_are_ignored(lib_built, monkeypatch):
    monkeypatch.setenv("CREDIT_FORCE_PLAN", "split:3")
    monkeypatch.setenv("CREDIT_SELECTOR", "bogus")
    monkeypatch.setenv("CREDIT_SPIN_LIMIT", "-5")
    h = C.Handle(0, load_default_model=False)
    try:
        p, _ = h.select(C.SOFTMAX, C.FWD, C.F32, 16, 4096)
        # default without a model: the fixed rule (row-resident where the row fits)
        assert p.as_tuple() == (C.ROW_RESIDENT, 1)
    finally:
        h.close()


def test_spin_limit_from_environment(lib_built, monkeypatch):
    # a tiny bound with one member that never publishes (test option): the
    # wait gives up at once and the timeout is reported
    monkeypatch.setenv("CREDIT_SPIN_LIMIT", "64")
    h = C.Handle(0, load_default_model=False)
    try:
        h.set_option(C.OPT_TEST_DROP_PUBLISH, 1)
        x = torch.randn(8, 4096, device="cuda")
        print("[config] forced timeout through CREDIT_SPIN_LIMIT", flush=True)
        C.softmax_fwd(x, p=C.plan("split", 2), h=h)
        assert h.check_errors() == C.ERR_TIMEOUT
        h.set_option(C.OPT_TEST_DROP_PUBLISH, 0)
        h.set_option(C.OPT_SPIN_LIMIT, 1 << 22)  # a 64-poll bound is too tight for normal arrival skew
        C.softmax_fwd(x, p=C.plan("split", 2), h=h)
        assert h.check_errors() == C.OK
    finally:
        h.close()


def test_checked_mode_reports_the_timeout_from_the_call(lib_built, monkeypatch):
    # CREDIT_CHECKED=1: the call itself waits and returns CREDIT_ERR_TIMEOUT
    # (raised by the binding) when an exchange wait expired; the flag is then
    # clear, and a normal call afterwards succeeds
    monkeypatch.setenv("CREDIT_CHECKED", "1")
    h = C.Handle(0, load_default_model=False)
    try:
        x = torch.randn(8, 4096, device="cuda")
        C.softmax_fwd(x, p=C.plan("split", 2), h=h)
        h.set_option(C.OPT_SPIN_LIMIT, 64)
        h.set_option(C.OPT_TEST_DROP_PUBLISH, 1)
        print("[config] forced timeout in checked mode", flush=True)
        with pytest.raises(C.CreditError) as e:
            C.softmax_fwd(x, p=C.plan("split", 2), h=h)
        assert e.value.status == C.ERR_TIMEOUT
        assert h.check_errors() == C.OK
        h.set_option(C.OPT_TEST_DROP_PUBLISH, 0)
        h.set_option(C.OPT_SPIN_LIMIT, 1 << 22)
        y, _ = C.softmax_fwd(x, p=C.plan("split", 2), h=h)
        ref = torch.softmax(x.double().cpu(), dim=1)
        assert torch.max(torch.abs(y.double().cpu() - ref)).item() < 1e-6
    finally:
        h.close()


def test_checked_mode_records_into_a_graph(lib_built, monkeypatch):
    # a capturing stream is not waited on: the call records normally, and
    # every replay is checked through credit_check_errors
    monkeypatch.setenv("CREDIT_CHECKED", "1")
    h = C.Handle(0, load_default_model=False)
    side = torch.cuda.Stream()
    try:
        x = torch.randn(24, 30000, device="cuda")
        with torch.cuda.stream(side):
            C.softmax_fwd(x, p=C.plan("split", 4), h=h)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            y, _ = C.softmax_fwd(x, p=C.plan("split", 4), h=h)
        for rep in range(3):
            x.copy_(torch.randn(24, 30000, device="cuda") * (1 + rep))
            print(f"[config] checked-mode replay {rep}", flush=True)
            graph.replay()
            torch.cuda.synchronize()
            assert h.check_errors() == C.OK
            ref = torch.softmax(x.double().cpu(), dim=1)
            assert torch.max(torch.abs(y.double().cpu() - ref)).item() < 1e-6
    finally:
        h.close()


def test_call_log_has_one_record_per_call(lib_built, monkeypatch, tmp_path):
    path = tmp_path / "calls.jsonl"
    monkeypatch.setenv("CREDIT_LOG", str(path))
    monkeypatch.setenv("CREDIT_SELECTOR", "fixed")
    h = C.Handle(0, load_default_model=False)
    try:
        x = torch.randn(64, 20000, device="cuda")
        g = torch.rand(20000, device="cuda") + 0.5
        C.rmsnorm_fwd(x, g, 1e-5, p=C.plan("split", 4), h=h)
        C.rmsnorm_fwd(x, g, 1e-5, h=h)
        fixed, _ = h.select(C.RMSNORM, C.FWD, C.F32, 64, 20000)
        torch.cuda.synchronize()
    finally:
        h.close()
    recs = [json.loads(line) for line in path.read_text().splitlines()]
    assert len(recs) == 2  # operator calls only (not select)
    a, b = recs
    assert (a["op"], a["dtype"], a["M"], a["N"]) == ("rmsnorm_fwd", "f32", 64, 20000)
    assert a["plan"] == [C.SPLIT_ROW, 4] and a["plan_given"] and not a["forced"]
    assert a["status"] == "CREDIT_OK" and a["checked"] is False
    assert a["grid"] > 0 and a["grid"] % 4 == 0 and a["vpt"] >= 1 and a["per_cu"] >= 1
    assert not b["plan_given"] and b["selector"] == "fixed" and b["status"] == "CREDIT_OK"
    assert b["plan"] == list(fixed.as_tuple())


def test_register_model_is_a_lower_bound_of_runtime_occupancy(lib_built):
    # The host's register model (used without a handle) sets each instance's
    # minimum waves per SIMD; the compiled kernel may use fewer registers and
    # fit more.  Co-residency uses the runtime figure, which must never be
    # below the model's, for every instantiated (operator, dtype, vectors).
    import torch  # noqa: F401  (torch's HIP runtime first)

    h = C.Handle(0, load_default_model=False)
    try:
        pairs = [(C.SOFTMAX, C.FWD), (C.LAYERNORM, C.FWD), (C.RMSNORM, C.FWD), (C.SOFTMAX, C.BWD),
                 (C.LAYERNORM, C.BWD), (C.RMSNORM, C.BWD), (C.SOFTMAX_LOGITS, C.BWD), (C.QUANT_INT8, C.FWD),
                 (C.QUANT_FP8, C.FWD), (C.PEARSON, C.BWD), (C.WVAR, C.BWD), (C.LAYERNORM_FP8_OUT, C.FWD)]
        epv = {C.F32: 4, C.BF16: 8, C.FP8: 16}
        seen = 0
        for op, d in pairs:
            for dt in (C.F32, C.BF16, C.FP8):
                for vpt in (1, 2, 4, 8, 12, 16, 24, 32):
                    N = 2 * vpt * 256 * epv[dt]
                    p = C.plan("split", 2)
                    try:
                        g1 = h.geometry(op, d, dt, 4096, N, p)
                    except C.CreditError:
                        continue  # (operator, dtype) pair that does not exist
                    if g1 is None or g1["vpt"] != vpt:
                        continue
                    g0 = C.plan_geometry(None, op, d, dt, 4096, N, p)
                    assert g0 is not None and g1["per_cu"] >= g0["per_cu"] >= 1, (op, d, dt, vpt, g0, g1)
                    seen += 1
        assert seen >= 150
    finally:
        h.close()
