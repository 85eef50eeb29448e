"""Operators recorded into a HIP graph (torch.cuda.graph) and replayed with new
inputs: every replay must match the oracle.  Split-row launches take their
exchange epoch from device memory when recorded, so a replay never accepts the
previous replay's partials.  Eager work and synchronisations run between the
replays."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import inputs as I

pytestmark = pytest.mark.gpu
EPS = 1e-5


def test_graph_replay_with_new_inputs(lib_built):
    h = C.Handle(0, load_default_model=False)
    M, N = 48, 30000
    g32, b32 = I.norm_params(N, seed=31)
    gamma, beta = torch.from_numpy(g32).cuda(), torch.from_numpy(b32).cuda()
    static_x = torch.empty((M, N), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    try:
        # warm up on the capture stream: workspace and plans exist before capture
        static_x.copy_(torch.from_numpy(I.norm_rows(M, N, seed=30).astype(np.float32)))
        with torch.cuda.stream(side):
            C.softmax_fwd(static_x, p=C.plan("split", 4), h=h)
            C.layernorm_fwd(static_x, gamma, beta, EPS, p=C.plan("split", 8), h=h)
            C.rmsnorm_fwd(static_x, gamma, EPS, p=C.plan("resident"), h=h)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            ys, _ = C.softmax_fwd(static_x, p=C.plan("split", 4), h=h)
            yl, _, mu, rs = C.layernorm_fwd(static_x, gamma, beta, EPS, p=C.plan("split", 8), h=h)
            yr, _, _ = C.rmsnorm_fwd(static_x, gamma, EPS, p=C.plan("resident"), h=h)
        for rep in range(4):
            x64 = I.norm_rows(M, N, seed=100 + rep) * (1.0 + 0.5 * rep)
            x32 = x64.astype(np.float32)
            static_x.copy_(torch.from_numpy(x32))
            print(f"[graph] replay {rep}", flush=True)
            graph.replay()
            torch.cuda.synchronize()
            xr = x32.astype(np.float64)
            assert np.max(np.abs(ys.double().cpu().numpy() - oracle.softmax_fwd(xr))) <= 2e-6
            ref, _, _ = oracle.layernorm_fwd(xr, g32.astype(np.float64), b32.astype(np.float64), EPS)
            assert np.max(np.abs(yl.double().cpu().numpy() - ref)) <= 1e-5
            ref2, _ = oracle.rmsnorm_fwd(xr, g32.astype(np.float64), EPS)
            assert np.max(np.abs(yr.double().cpu().numpy() - ref2)) <= 1e-5
            # eager split-row work on the same handle between replays
            z = torch.randn(16, 20000, device="cuda")
            zz, _ = C.softmax_fwd(z, p=C.plan("split", 2), h=h)
            torch.cuda.synchronize()
            assert np.max(np.abs(zz.double().cpu().numpy() - oracle.softmax_fwd(z.double().cpu().numpy()))) <= 2e-6
        assert h.check_errors() == C.OK
    finally:
        h.close()


def test_graph_replay_backward_with_column_reduction(lib_built):
    # LayerNorm backward recorded with its dgamma / dbeta reduction kernels
    h = C.Handle(0, load_default_model=False)
    M, N = 600, 4096
    g32, _ = I.norm_params(N, seed=41)
    gamma = torch.from_numpy(g32).cuda()
    sx = torch.empty((M, N), dtype=torch.float32, device="cuda")
    sdy = torch.empty((M, N), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    try:
        sx.copy_(torch.from_numpy(I.norm_rows(M, N, seed=40).astype(np.float32)))
        sdy.normal_()
        with torch.cuda.stream(side):
            C.layernorm_bwd(sx, sdy, gamma, None, None, EPS, p=C.plan("split", 4), h=h)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            dx, _, dg, db = C.layernorm_bwd(sx, sdy, gamma, None, None, EPS, p=C.plan("split", 4), h=h)
        for rep in range(3):
            x32 = I.norm_rows(M, N, seed=200 + rep).astype(np.float32)
            dy32 = I.normal_rows(M, N, seed=200 + rep, tensor=1).astype(np.float32)
            sx.copy_(torch.from_numpy(x32))
            sdy.copy_(torch.from_numpy(dy32))
            print(f"[graph] backward replay {rep}", flush=True)
            graph.replay()
            torch.cuda.synchronize()
            x64, dy64 = x32.astype(np.float64), dy32.astype(np.float64)
            dxr, dgr, dbr = oracle.layernorm_bwd(x64, dy64, g32.astype(np.float64), EPS)
            assert np.max(np.abs(dx.double().cpu().numpy() - dxr)) <= 1e-5 * max(1.0, np.abs(dxr).max())
            _, mu, rs = oracle.layernorm_fwd(x64, g32.astype(np.float64), np.zeros(N), EPS)
            xh = (x64 - mu[:, None]) * rs[:, None]
            assert np.all(np.abs(dg.double().cpu().numpy() - dgr) <= 1e-5 * np.abs(dy64 * xh).sum(0) + 1e-6)
            assert np.all(np.abs(db.double().cpu().numpy() - dbr) <= 1e-5 * np.abs(dy64).sum(0) + 1e-6)
        assert h.check_errors() == C.OK
    finally:
        h.close()


def test_graph_replay_after_the_stream_workspace_grew(lib_built):
    # a graph captured with the stream's small workspace, then an eager call
    # with a larger shape on the same stream (the handle replaces the
    # workspace) and fresh allocations that may reuse freed memory: the replay
    # must still write its exchange slots and partials into memory it owns
    h = C.Handle(0, load_default_model=False)
    M, N = 64, 8192
    g32, _ = I.norm_params(N, seed=51)
    gamma = torch.from_numpy(g32).cuda()
    sx = torch.empty((M, N), dtype=torch.float32, device="cuda")
    sdy = torch.empty((M, N), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    try:
        sx.copy_(torch.from_numpy(I.norm_rows(M, N, seed=50).astype(np.float32)))
        sdy.normal_()
        with torch.cuda.stream(side):
            C.layernorm_bwd(sx, sdy, gamma, None, None, EPS, p=C.plan("split", 2), h=h)
        torch.cuda.synchronize()
        ws_small = h._ws[side.cuda_stream].data_ptr()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            dx, _, dg, db = C.layernorm_bwd(sx, sdy, gamma, None, None, EPS, p=C.plan("split", 2), h=h)
        # a much larger call on the capture stream replaces its workspace
        big_x = torch.randn(2048, 65536, device="cuda") + 10
        big_dy = torch.randn(2048, 65536, device="cuda")
        big_g = torch.ones(65536, device="cuda")
        with torch.cuda.stream(side):
            C.layernorm_bwd(big_x, big_dy, big_g, None, None, EPS, p=C.plan("split", 8), h=h)
        torch.cuda.synchronize()
        assert h._ws[side.cuda_stream].data_ptr() != ws_small
        del big_x, big_dy
        # fill whatever the allocator hands out now with garbage
        junk = [torch.full((1 << 22,), -1, dtype=torch.int32, device="cuda") for _ in range(16)]
        torch.cuda.synchronize()
        for rep in range(3):
            x32 = I.norm_rows(M, N, seed=300 + rep).astype(np.float32)
            dy32 = I.normal_rows(M, N, seed=300 + rep, tensor=1).astype(np.float32)
            sx.copy_(torch.from_numpy(x32))
            sdy.copy_(torch.from_numpy(dy32))
            print(f"[graph] replay after workspace growth {rep}", flush=True)
            graph.replay()
            torch.cuda.synchronize()
            assert all(int((j != -1).sum()) == 0 for j in junk), "the replay wrote into reallocated memory"
            x64, dy64 = x32.astype(np.float64), dy32.astype(np.float64)
            dxr, dgr, dbr = oracle.layernorm_bwd(x64, dy64, g32.astype(np.float64), EPS)
            assert np.max(np.abs(dx.double().cpu().numpy() - dxr)) <= 1e-5 * max(1.0, np.abs(dxr).max())
            assert np.all(np.abs(db.double().cpu().numpy() - dbr) <= 1e-5 * np.abs(dy64).sum(0) + 1e-6)
        assert h.check_errors() == C.OK
    finally:
        h.close()
