"""GPU parity at the largest rows each resident form accepts: a row exactly at
a split plan's capacity (32 workgroups x 256 threads x the largest vectors
per thread of the operator and dtype -- registers, plus LDS for the FP32 /
BF16 softmax, LayerNorm and RMSNorm forward) runs every legal plan and
matches the FP64 oracle; one element more makes every split plan illegal and
the two-pass kernel takes it, also to the oracle's tolerance."""
import pytest

from paper_2609_01864_amd import credit as C

from _cases import ALL_PLANS, OPNUM, Case, check_case

pytestmark = pytest.mark.gpu

# (operator, dtype, elements per 16-byte vector, largest vectors per thread)
LIMITS = [("layernorm_fwd", "f32", 4, 68), ("softmax_fwd", "bf16", 8, 68), ("rmsnorm_fwd", "f32", 4, 68),
          ("rmsnorm_fwd", "fp8", 16, 16), ("softmax_bwd", "f32", 4, 16), ("layernorm_bwd", "bf16", 8, 4)]


@pytest.mark.parametrize("op,dtype,epv,vmax", LIMITS)
def test_split_capacity_limit_and_one_past_it(gpu_handle, op, dtype, epv, vmax):
    h = gpu_handle
    o, d = OPNUM[op]
    dt = C.DTYPE_NAMES[dtype]
    n_max = 32 * 256 * vmax * epv
    for N, split_legal in ((n_max, True), (n_max + 1, False)):
        print(f"[max] {op} {dtype} N={N}", flush=True)
        assert h.plan_legal(o, d, dt, 3, N, C.plan("split", 32)) == split_legal
        case = Case(op, dtype, 3, N, seed=N % 9973)
        ref = case.reference()
        plans = [C.plan(v, k) for v, k in ALL_PLANS if h.plan_legal(o, d, dt, 3, N, C.plan(v, k))]
        assert any(p.variant == C.TWO_PASS for p in plans)
        assert all(p.variant == C.TWO_PASS for p in plans) == (not split_legal)
        for p in plans:
            try:
                check_case(case, case.run(h, p, ref=ref), ref)
            except AssertionError as e:
                raise AssertionError(f"N={N} {p}: {e}") from None
