"""Environment configuration read when a handle is created:
CREDIT_FORCE_PLAN, CREDIT_SELECTOR, CREDIT_SPIN_LIMIT."""
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
