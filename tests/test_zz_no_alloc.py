"""The allocation-free LayerNorm forward (credit_layernorm_fwd_noalloc)
against the workspace entry point it shares its kernels with: the same plan
gives bitwise the same output, mean and rstd, and both match the FP64
oracle; two calls in a row, the second with a smaller input (the scratch
keeps the first call's contents).  A plan whose slots exceed the scratch is
refused with CREDIT_ERR_WORKSPACE, and the calls leave the device's free
memory unchanged."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

pytestmark = pytest.mark.gpu
EPS = 1e-5


def _ln_both(h, M, N, plan, seed):
    x64 = I.norm_rows(M, N, seed=seed)
    g32, b32 = I.norm_params(N, seed=seed)
    x = torch.from_numpy(x64.astype(np.float32)).cuda()
    g, b = torch.from_numpy(g32).cuda(), torch.from_numpy(b32).cuda()
    outs = []
    for noalloc in (False, True):
        y = torch.full((M, N), float("nan"), device="cuda")
        mean = torch.full((M,), float("nan"), device="cuda")
        rstd = torch.full((M,), float("nan"), device="cuda")
        s = torch.cuda.current_stream().cuda_stream
        pp = ctypes.byref(plan)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        if noalloc:
            st = C.lib().credit_layernorm_fwd_noalloc(h.ptr, M, N, C.F32, x.data_ptr(), N, None, g.data_ptr(),
                                                      b.data_ptr(), EPS, y.data_ptr(), N, None, mean.data_ptr(),
                                                      rstd.data_ptr(), pp, s)
        else:
            n = h.workspace_size(C.LAYERNORM, C.FWD, C.F32, M, N, plan)
            ws = torch.zeros(n, dtype=torch.uint8, device="cuda")
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            st = C.lib().credit_layernorm_fwd(h.ptr, M, N, C.F32, x.data_ptr(), N, None, g.data_ptr(), b.data_ptr(),
                                              EPS, y.data_ptr(), N, None, mean.data_ptr(), rstd.data_ptr(), pp,
                                              ws.data_ptr(), n, s)
        assert st == C.OK, C.status_string(st)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        outs.append((y.cpu().numpy(), mean.cpu().numpy(), rstd.cpu().numpy()))
    ref, mu, rs = oracle.layernorm_fwd(x64.astype(np.float32).astype(np.float64), g32.astype(np.float64),
                                       b32.astype(np.float64), EPS)
    return outs, (ref, mu, rs)


def test_noalloc_layernorm_matches_the_workspace_entry_point(gpu_handle):
    h = gpu_handle
    assert C.lib().credit_noalloc_scratch_bytes() == 16 << 20
    for (M, N, plan) in ((512, 131072, C.plan("split", 8)), (37, 20011, C.plan("split", 4)),
                         (300, 65536, C.plan("split", 16)), (5, 3001, C.plan("resident"))):
        print(f"[noalloc] M={M} N={N} {plan}", flush=True)
        (ws_out, na_out), (ref, mu, rs) = _ln_both(h, M, N, plan, seed=M + N)
        for a, b in zip(ws_out, na_out):
            assert np.array_equal(a, b)
        assert np.max(np.abs(na_out[0].astype(np.float64) - ref)) <= 1e-5
        assert np.max(np.abs(na_out[2] - rs)) <= 1e-6 * np.max(rs)
        assert np.max(np.abs(na_out[1] - mu)) <= 1e-5 * max(1.0, np.max(np.abs(mu)))
    assert h.check_errors() == C.OK


def test_noalloc_two_row_workgroups(gpu_handle):
    # shapes where the library holds two rows per workgroup: a row-resident
    # plan with more than twice as many rows as row-group slots, and a split
    # plan at k = 16 with two rows per workgroup forced
    h = gpu_handle
    cases = [(8192, 1024, C.plan("resident"), 0), (300, 65536, C.plan("split", 16), 2)]
    try:
        for M, N, plan, rows in cases:
            h.set_option(C.OPT_ROWS, rows)
            assert h.geometry(C.LAYERNORM, C.FWD, C.F32, M, N, plan)["rows"] == 2
            print(f"[noalloc] two rows M={M} N={N} {plan}", flush=True)
            (ws_out, na_out), (ref, mu, rs) = _ln_both(h, M, N, plan, seed=M + 7)
            for a, b in zip(ws_out, na_out):
                assert np.array_equal(a, b)
            assert np.max(np.abs(na_out[0].astype(np.float64) - ref)) <= 1e-5
            assert np.max(np.abs(na_out[2] - rs)) <= 1e-6 * np.max(rs)
    finally:
        h.set_option(C.OPT_ROWS, 0)
    assert h.check_errors() == C.OK


def test_noalloc_refuses_plans_beyond_its_scratch(gpu_handle):
    h = gpu_handle
    M, N = 12000, 4096  # split k = 32 needs M * 3 * 32 * 2 * 8 + 256 bytes > 16 MiB
    x = torch.zeros((M, N), device="cuda")
    g = torch.ones(N, device="cuda")
    y = torch.empty_like(x)
    s = torch.cuda.current_stream().cuda_stream
    p = C.plan("split", 32)
    assert h.workspace_size(C.LAYERNORM, C.FWD, C.F32, M, N, p) > C.lib().credit_noalloc_scratch_bytes()
    st = C.lib().credit_layernorm_fwd_noalloc(h.ptr, M, N, C.F32, x.data_ptr(), N, None, g.data_ptr(), g.data_ptr(),
                                              EPS, y.data_ptr(), N, None, None, None, ctypes.byref(p), s)
    assert st == C.ERR_WORKSPACE
    # plan == NULL on a fresh shape: the fixed rule, no device work besides the operator
    x2 = torch.from_numpy(I.norm_rows(64, 8192, seed=3).astype(np.float32)).cuda()
    g2 = torch.ones(8192, device="cuda")
    y2 = torch.empty_like(x2)
    st = C.lib().credit_layernorm_fwd_noalloc(h.ptr, 64, 8192, C.F32, x2.data_ptr(), 8192, None, g2.data_ptr(),
                                              g2.data_ptr(), EPS, y2.data_ptr(), 8192, None, None, None, None, s)
    assert st == C.OK
    torch.cuda.synchronize()
    ref, _, _ = oracle.layernorm_fwd(x2.double().cpu().numpy(), np.ones(8192), np.ones(8192), EPS)
    assert np.max(np.abs(y2.double().cpu().numpy() - ref)) <= 1e-5
    assert h.check_errors() == C.OK
