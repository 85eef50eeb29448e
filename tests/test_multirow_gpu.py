"""GPU parity of the multi-row LayerNorm / RMSNorm forward (a workgroup holds
the same slice of R rows at once): every compiled instance in both row loops,
small and ragged shapes with row counts that leave a partial last block,
padded and misaligned rows, few row groups, and exchange skew -- each against
the FP64 oracle.  (The one-row kernel visits a thread's slots in an order
rotated by its row group, so the two round their per-thread sums in different
orders and are not compared bitwise.)"""
import numpy as np
import pytest

from paper_2609_01864_amd import credit as C

from _cases import ALL_PLANS, OPNUM, Case, check_case

pytestmark = pytest.mark.gpu

OPS = ["layernorm_fwd", "rmsnorm_fwd"]
BYTES = {"f32": 4, "bf16": 2, "fp8": 1}
DTN = {"f32": C.F32, "bf16": C.BF16, "fp8": C.FP8}
MR_VPTS = (1, 2, 4, 8)
ROWS = (2, 4)


@pytest.fixture(scope="module")
def handles(lib_built):
    hs = {}
    for r in (1,) + ROWS:
        h = C.Handle(0, load_default_model=False)
        h.set_option(C.OPT_ROWS, r)
        hs[r] = h
    yield hs
    for h in hs.values():
        h.close()


def _plans(h, op, dtype, M, N):
    o, d = OPNUM[op]
    out = []
    for v, k in ALL_PLANS:
        p = C.plan(v, k)
        if v != "two_pass" and h.plan_legal(o, d, C.DTYPE_NAMES[dtype], M, N, p):
            out.append(p)
    return out


def _check_rows(hs, rows, op, dtype, M, N, seed, **kw):
    case = Case(op, dtype, M, N, seed=seed)
    ref = case.reference()
    o, d = OPNUM[op]
    plans = _plans(hs[rows], op, dtype, M, N)
    assert plans
    multi = 0
    for p in plans:
        geo = hs[rows].geometry(o, d, DTN[dtype], M, N, p)
        print(f"[multirow] {op} {dtype} M={M} N={N} {p} rows={geo['rows']} {kw}", flush=True)
        out = case.run(hs[rows], p, ref=ref, **kw)
        try:
            check_case(case, out, ref)
        except AssertionError as e:
            raise AssertionError(f"{p} rows={geo['rows']}: {e}") from None
        multi += geo["rows"] > 1
    return multi


@pytest.mark.parametrize("rows", ROWS)
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("M,N", [(1, 1), (3, 7), (5, 17), (2, 33), (37, 1000), (7, 4097), (3, 20011), (9, 65536)])
def test_multirow_parity(handles, rows, op, dtype, M, N):
    multi = _check_rows(handles, rows, op, dtype, M, N, seed=M * 1000 + N + rows)
    if M >= 2 and N >= 1000:
        assert multi > 0, "no plan ran the multi-row kernel"


@pytest.mark.parametrize("rows", ROWS)
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_multirow_strided_and_misaligned(handles, rows, op, dtype):
    for ld_pad, offset in ((4, 0), (1, 1), (3, 5)):
        _check_rows(handles, rows, op, dtype, 6, 1029, seed=11, ld_pad=ld_pad, offset=offset)


@pytest.mark.parametrize("op", OPS)
def test_multirow_every_instance_both_row_loops(handles, op):
    # N = k * VPT * 256 * EPV gives every member exactly VPT full vectors per
    # thread (unmasked loop); five elements fewer leave a ragged last slice;
    # M = 2R + 1 rows leave a partial last row block
    o, d = OPNUM[op]
    covered = set()
    for rows in ROWS:
        h = handles[rows]
        for dt in ("f32", "bf16", "fp8"):
            epv = 16 // BYTES[dt]
            for v in MR_VPTS:
                info = C.instance_info(h, o, d, DTN[dt], v, rows)
                if dt == "fp8" and v * rows > 8:  # FP8 holds at most 8 vectors per thread over its rows
                    assert info is None
                    continue
                assert info is not None and info["per_cu"] >= 1, (op, dt, v, rows)
                M = 2 * rows + 1
                for var, k, N in (("resident", 1, v * 256 * epv), ("split", 2, 2 * v * 256 * epv),
                                  ("split", 2, 2 * v * 256 * epv - 5)):
                    p = C.plan(var, k)
                    geo = h.geometry(o, d, DTN[dt], M, N, p)
                    assert geo is not None and geo["vpt"] == v and geo["rows"] == rows, (dt, v, rows, var, N, geo)
                    print(f"[multirow instance] {op} {dt} vpt={v} rows={rows} {var} k={k} N={N} {info}", flush=True)
                    case = Case(op, dt, M, N, seed=v * 7 + k + rows)
                    ref = case.reference()
                    check_case(case, case.run(h, p, ref=ref), ref)
                covered.add((dt, v, rows))
    assert len(covered) == 2 * len(MR_VPTS) * len(ROWS) + 5  # FP8: (1, 2, 4) x 2 rows, (1, 2) x 4 rows
    for rows in ROWS:
        assert C.instance_info(handles[rows], o, d, C.F32, 12, rows) is None  # beyond the multi-row slices
        assert handles[rows].check_errors() == C.OK


@pytest.mark.parametrize("op", OPS)
def test_multirow_more_blocks_than_row_groups(handles, op):
    M, N = 203, 777
    for rows in ROWS:
        h = handles[rows]
        h.set_option(C.OPT_MAX_GROUPS, 3)
        try:
            _check_rows(handles, rows, op, "f32", M, N, seed=3)
        finally:
            h.set_option(C.OPT_MAX_GROUPS, 0)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("dtype", ["f32", "fp8"])
def test_multirow_exchange_under_member_skew(handles, op, dtype):
    # members of a row group publish out of step; results must not change
    M, N = 11, 16384
    for rows in ROWS:
        h = handles[rows]
        case = Case(op, dtype, M, N, seed=21)
        ref = case.reference()
        for k in (2, 4, 8):
            p = C.plan("split", k)
            plain = case.run(h, p, ref=ref)
            h.set_option(C.OPT_TEST_SKEW, 1)
            try:
                print(f"[multirow] skew {op} {dtype} rows={rows} k={k}", flush=True)
                skewed = case.run(h, p, ref=ref)
            finally:
                h.set_option(C.OPT_TEST_SKEW, 0)
            check_case(case, skewed, ref)
            assert np.array_equal(plain["y"], skewed["y"])


def test_rows_option_is_validated(handles):
    h = handles[1]
    with pytest.raises(C.CreditError):
        h.set_option(C.OPT_ROWS, 3)
    with pytest.raises(C.CreditError):
        h.set_option(C.OPT_ROWS, -1)
    # the backward and softmax plans never take the multi-row kernel
    h2 = handles[4]
    for op, d in ((C.SOFTMAX, C.FWD), (C.LAYERNORM, C.BWD)):
        assert h2.geometry(op, d, C.F32, 64, 8192, C.plan("resident"))["rows"] == 1
    assert h2.geometry(C.LAYERNORM, C.FWD, C.F32, 64, 8192, C.plan("resident"))["rows"] == 4
    assert h2.geometry(C.LAYERNORM, C.FWD, C.F32, 1, 8192, C.plan("resident"))["rows"] == 1


def test_multirow_graph_replay_with_new_inputs(lib_built):
    # two-row split launches recorded into a HIP graph: every replay takes a
    # new device-side epoch, so no row block accepts a previous replay's slots
    import torch

    import oracle
    from paper_2609_01864_amd import inputs as I

    h = C.Handle(0, load_default_model=False)
    h.set_option(C.OPT_ROWS, 2)
    M, N, eps = 37, 30000, 1e-5
    g32, b32 = I.norm_params(N, seed=61)
    gamma, beta = torch.from_numpy(g32).cuda(), torch.from_numpy(b32).cuda()
    sx = torch.empty((M, N), dtype=torch.float32, device="cuda")
    side = torch.cuda.Stream()
    p = C.plan("split", 4)
    try:
        for o in (C.LAYERNORM, C.RMSNORM):
            assert h.geometry(o, C.FWD, C.F32, M, N, p)["rows"] == 2
        sx.copy_(torch.from_numpy(I.norm_rows(M, N, seed=60).astype(np.float32)))
        with torch.cuda.stream(side):
            C.layernorm_fwd(sx, gamma, beta, eps, p=p, h=h)
            C.rmsnorm_fwd(sx, gamma, eps, p=p, h=h)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            yl, _, _, _ = C.layernorm_fwd(sx, gamma, beta, eps, p=p, h=h)
            yr, _, _ = C.rmsnorm_fwd(sx, gamma, eps, p=p, h=h)
        for rep in range(3):
            x32 = I.norm_rows(M, N, seed=400 + rep).astype(np.float32)
            sx.copy_(torch.from_numpy(x32))
            print(f"[multirow graph] replay {rep}", flush=True)
            graph.replay()
            torch.cuda.synchronize()
            xr = x32.astype(np.float64)
            ref, _, _ = oracle.layernorm_fwd(xr, g32.astype(np.float64), b32.astype(np.float64), eps)
            assert np.max(np.abs(yl.double().cpu().numpy() - ref)) <= 1e-5
            ref2, _ = oracle.rmsnorm_fwd(xr, g32.astype(np.float64), eps)
            assert np.max(np.abs(yr.double().cpu().numpy() - ref2)) <= 1e-5
            # eager two-row work on the same handle between replays
            z = torch.randn(9, 30000, device="cuda") + 3.0
            zz, _, _ = C.rmsnorm_fwd(z, gamma, eps, p=p, h=h)
            torch.cuda.synchronize()
            zr, _ = oracle.rmsnorm_fwd(z.double().cpu().numpy(), g32.astype(np.float64), eps)
            assert np.max(np.abs(zz.double().cpu().numpy() - zr)) <= 1e-5
        assert h.check_errors() == C.OK
    finally:
        h.close()
