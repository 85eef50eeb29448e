"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, invariants, special cases that reduce to a textbook function or
an independent library routine, brute force on tiny inputs, and finite
differences.  Each test is chosen so that a plausible mistake (a dropped term,
a wrong sign, index or normalisation, eps in the wrong place, biased vs
unbiased variance) fails it.  CPU only."""
import math

import numpy as np
import pytest
import torch

import oracle

RNG = np.random.default_rng(1234)


# ------------------------------------------------------------------ softmax
def test_softmax_rows_sum_to_one_and_positive():
    x = 4.0 * RNG.standard_normal((7, 301))
    y = oracle.softmax_fwd(x)
    assert np.all(y > 0)
    assert np.max(np.abs(y.sum(1) - 1.0)) < 1e-13


def test_softmax_shift_invariance_and_large_offsets():
    x = 4.0 * RNG.standard_normal((5, 64))
    y = oracle.softmax_fwd(x)
    # a shift leaves y unchanged up to the rounding of x + c (|c| * 2^-53);
    # +800 would overflow exp without the max shift
    for c in (-512.0, 800.0):
        assert np.max(np.abs(oracle.softmax_fwd(x + c) - y)) < 1e-13


def test_softmax_ratio_is_exp_of_difference():
    # y_i / y_j = exp(x_i - x_j): pins the sign of the exponent and the indexing
    x = RNG.standard_normal((3, 10))
    y = oracle.softmax_fwd(x)
    for i, j in [(0, 1), (3, 7), (9, 2)]:
        r = y[:, i] / y[:, j]
        assert np.allclose(r, np.exp(x[:, i] - x[:, j]), rtol=1e-13, atol=0)


def test_softmax_special_cases():
    # constant row -> 1/N
    y = oracle.softmax_fwd(np.full((2, 37), 3.25))
    assert np.max(np.abs(y - 1.0 / 37)) < 1e-16
    # N = 2 -> logistic(x0 - x1) (textbook sigmoid, via math.exp)
    x = RNG.standard_normal((6, 2)) * 3
    y = oracle.softmax_fwd(x)
    sig = np.array([1.0 / (1.0 + math.exp(-(a - b))) for a, b in x])
    assert np.max(np.abs(y[:, 0] - sig)) < 1e-15
    # permutation equivariance
    x = RNG.standard_normal((4, 19))
    perm = RNG.permutation(19)
    assert np.max(np.abs(oracle.softmax_fwd(x[:, perm]) - oracle.softmax_fwd(x)[:, perm])) < 1e-16
    # N = 1 -> 1
    assert oracle.softmax_fwd(np.array([[123.0]]))[0, 0] == 1.0


def test_softmax_masked_entries_reduce_to_the_unmasked_subset():
    # an entry of -inf drops out: the row's softmax equals the softmax of its
    # finite entries alone, placed back, with 0 where masked; the from-logits
    # backward likewise gives 0 there and the subset's gradient elsewhere
    x = RNG.standard_normal((3, 40)) * 4
    mask = RNG.random((3, 40)) < 0.4
    mask[2, :39] = True  # a single finite entry: a one-hot row
    dy = RNG.standard_normal((3, 40))
    xm = np.where(mask, -np.inf, x)
    y = oracle.softmax_fwd(xm)
    dx = oracle.softmax_logits_bwd(xm, dy)
    for r in range(3):
        keep = ~mask[r]
        sub = x[r, keep][None, :]
        assert np.all(y[r, mask[r]] == 0.0) and np.all(dx[r, mask[r]] == 0.0)
        np.testing.assert_allclose(y[r, keep], oracle.softmax_fwd(sub)[0], rtol=1e-14, atol=0)
        np.testing.assert_allclose(dx[r, keep], oracle.softmax_logits_bwd(sub, dy[r, keep][None, :])[0],
                                   rtol=1e-12, atol=1e-15)
    assert y[2, 39] == 1.0 and dx[2, 39] == 0.0
    # no finite entry: 0/0
    with np.errstate(invalid="ignore"):
        assert np.all(np.isnan(oracle.softmax_fwd(np.full((1, 8), -np.inf))))


def test_softmax_matches_independent_library():
    x = 4.0 * RNG.standard_normal((4, 8))
    ref = torch.softmax(torch.from_numpy(x), dim=1).numpy()
    assert np.max(np.abs(oracle.softmax_fwd(x) - ref)) < 1e-15


def test_softmax_bwd_equals_jacobian_transpose_product():
    # brute force: J = diag(y) - y y^T, dx = J^T dy, built entry by entry
    y = oracle.softmax_fwd(RNG.standard_normal((4, 16)) * 2)
    dy = RNG.standard_normal((4, 16))
    dx = oracle.softmax_bwd(y, dy)
    for m in range(4):
        J = np.empty((16, 16))
        for i in range(16):
            for j in range(16):
                J[i, j] = (y[m, i] if i == j else 0.0) - y[m, i] * y[m, j]
        assert np.max(np.abs(J.T @ dy[m] - dx[m])) < 1e-15
    # sum of dx is c * (1 - sum y) = 0 up to rounding
    assert np.max(np.abs(dx.sum(1))) < 1e-15


def test_softmax_bwd_finite_differences():
    x = RNG.standard_normal((4, 16))
    dy = RNG.standard_normal((4, 16))
    dx = oracle.softmax_bwd(oracle.softmax_fwd(x), dy)
    h = 1e-6
    for m in range(4):
        for i in range(16):
            xp = x.copy(); xp[m, i] += h
            xm = x.copy(); xm[m, i] -= h
            fd = (np.sum(dy * oracle.softmax_fwd(xp)) - np.sum(dy * oracle.softmax_fwd(xm))) / (2 * h)
            assert abs(fd - dx[m, i]) <= 1e-8 * max(1.0, abs(dx[m, i]))


# --------------------------------------------------------------- LayerNorm
def test_layernorm_normalised_moments_closed_form():
    x = 10.0 + RNG.standard_normal((6, 513))
    one, zero = np.ones(513), np.zeros(513)
    eps = 1e-5
    y, mu, rs = oracle.layernorm_fwd(x, one, zero, eps)
    var = np.var(x, axis=1)  # numpy's biased variance, independent of the oracle
    assert np.max(np.abs(y.mean(1))) < 1e-12
    assert np.max(np.abs(np.mean(y * y, 1) - var / (var + eps))) < 1e-12
    assert np.max(np.abs(mu - x.mean(1))) < 1e-13
    assert np.max(np.abs(rs - 1.0 / np.sqrt(var + eps))) < 1e-12


def test_layernorm_special_cases():
    eps = 1e-5
    # N = 2: y0 = ((x0 - x1)/2) / sqrt((x0 - x1)^2/4 + eps)  (eps inside the root)
    x = RNG.standard_normal((5, 2)) * 0.01
    y, _, _ = oracle.layernorm_fwd(x, np.ones(2), np.zeros(2), eps)
    d = (x[:, 0] - x[:, 1]) / 2
    assert np.max(np.abs(y[:, 0] - d / np.sqrt(d * d + eps))) < 1e-13
    assert np.max(np.abs(y[:, 1] + d / np.sqrt(d * d + eps))) < 1e-13
    # constant row -> beta
    beta = RNG.standard_normal(31)
    y, _, _ = oracle.layernorm_fwd(np.full((2, 31), 7.5), RNG.uniform(0.5, 1.5, 31), beta, eps)
    assert np.max(np.abs(y - beta)) < 1e-12
    # affine input a*x + b: rstd = 1/sqrt(a^2 var + eps)
    x = RNG.standard_normal((3, 100))
    a, b = 3.0, -40.0
    _, _, rs = oracle.layernorm_fwd(a * x + b, np.ones(100), np.zeros(100), eps)
    assert np.max(np.abs(rs - 1.0 / np.sqrt(a * a * np.var(x, 1) + eps))) < 1e-12


def test_layernorm_matches_independent_library():
    x = 10.0 + RNG.standard_normal((4, 8))
    g = RNG.uniform(0.5, 1.5, 8)
    b = 0.1 * RNG.standard_normal(8)
    ref = torch.nn.functional.layer_norm(torch.from_numpy(x), (8,), torch.from_numpy(g), torch.from_numpy(b), 1e-5)
    y, _, _ = oracle.layernorm_fwd(x, g, b, 1e-5)
    assert np.max(np.abs(y - ref.numpy())) < 1e-13


def _ln_loss(x, g, b, dy):
    return np.sum(dy * oracle.layernorm_fwd(x, g, b, 1e-5)[0])


def test_layernorm_bwd_finite_differences():
    x = 10.0 + RNG.standard_normal((4, 16))
    g = RNG.uniform(0.5, 1.5, 16)
    b = 0.1 * RNG.standard_normal(16)
    dy = RNG.standard_normal((4, 16))
    dx, dg, db = oracle.layernorm_bwd(x, dy, g, 1e-5)
    h = 1e-6
    for m in range(4):
        for i in range(16):
            xp = x.copy(); xp[m, i] += h
            xm = x.copy(); xm[m, i] -= h
            fd = (_ln_loss(xp, g, b, dy) - _ln_loss(xm, g, b, dy)) / (2 * h)
            assert abs(fd - dx[m, i]) <= 1e-7 * max(1.0, abs(dx[m, i]))
    for j in range(16):
        gp = g.copy(); gp[j] += h
        gm = g.copy(); gm[j] -= h
        assert abs((_ln_loss(x, gp, b, dy) - _ln_loss(x, gm, b, dy)) / (2 * h) - dg[j]) < 1e-7
        bp = b.copy(); bp[j] += h
        bm = b.copy(); bm[j] -= h
        assert abs((_ln_loss(x, g, bp, dy) - _ln_loss(x, g, bm, dy)) / (2 * h) - db[j]) < 1e-7


def test_layernorm_bwd_invariants_and_column_sums():
    x = 10.0 + RNG.standard_normal((9, 40))
    g = RNG.uniform(0.5, 1.5, 40)
    dy = RNG.standard_normal((9, 40))
    eps = 1e-5
    dx, dg, db = oracle.layernorm_bwd(x, dy, g, eps)
    assert np.max(np.abs(dx.sum(1))) < 1e-12  # sum dx = 0
    # sum dx * xhat = rstd * sum(g xhat) * (1 - var/(var+eps))
    mu = x.mean(1, keepdims=True)
    var = np.var(x, 1, keepdims=True)
    rs = 1.0 / np.sqrt(var + eps)
    xh = (x - mu) * rs
    lhs = np.sum(dx * xh, 1)
    rhs = rs[:, 0] * np.sum(dy * g * xh, 1) * (1.0 - var[:, 0] / (var[:, 0] + eps))
    assert np.max(np.abs(lhs - rhs)) < 1e-11
    # dbeta is the plain column sum of dy (correctly rounded by math.fsum)
    assert all(abs(db[j] - math.fsum(dy[:, j])) < 1e-14 for j in range(40))
    ref_dg = [math.fsum(dy[:, j] * xh[:, j]) for j in range(40)]
    assert np.max(np.abs(dg - ref_dg)) < 1e-12


def test_layernorm_bwd_matches_torch_autograd():
    x = torch.from_numpy(10.0 + RNG.standard_normal((4, 16))).requires_grad_(True)
    g = torch.from_numpy(RNG.uniform(0.5, 1.5, 16)).requires_grad_(True)
    b = torch.from_numpy(0.1 * RNG.standard_normal(16)).requires_grad_(True)
    dy = torch.from_numpy(RNG.standard_normal((4, 16)))
    torch.nn.functional.layer_norm(x, (16,), g, b, 1e-5).backward(dy)
    dx, dg, db = oracle.layernorm_bwd(x.detach().numpy(), dy.numpy(), g.detach().numpy(), 1e-5)
    assert np.max(np.abs(dx - x.grad.numpy())) < 1e-12
    assert np.max(np.abs(dg - g.grad.numpy())) < 1e-12
    assert np.max(np.abs(db - b.grad.numpy())) < 1e-12


# ----------------------------------------------------------------- RMSNorm
def test_rmsnorm_closed_forms():
    eps = 1e-5
    x = RNG.standard_normal((5, 77)) * 3
    y, rs = oracle.rmsnorm_fwd(x, np.ones(77), eps)
    ms = np.mean(x * x, 1)
    assert np.max(np.abs(np.mean(y * y, 1) - ms / (ms + eps))) < 1e-12
    assert np.max(np.abs(rs - 1.0 / np.sqrt(ms + eps))) < 1e-12
    # constant row c, gamma = 1 -> c / sqrt(c^2 + eps)
    y, _ = oracle.rmsnorm_fwd(np.full((1, 9), 0.02), np.ones(9), eps)
    assert np.max(np.abs(y - 0.02 / math.sqrt(0.02 ** 2 + eps))) < 1e-15
    # scale invariance up to eps: y(a x) = y(x) when eps -> 0
    y1, _ = oracle.rmsnorm_fwd(x, np.ones(77), 0.0)
    y2, _ = oracle.rmsnorm_fwd(5.0 * x, np.ones(77), 0.0)
    assert np.max(np.abs(y1 - y2)) < 1e-13


def test_rmsnorm_matches_torch():
    x = torch.from_numpy(RNG.standard_normal((4, 8)) + 1).requires_grad_(True)
    g = torch.from_numpy(RNG.uniform(0.5, 1.5, 8)).requires_grad_(True)
    dy = torch.from_numpy(RNG.standard_normal((4, 8)))
    out = torch.nn.functional.rms_norm(x, (8,), g, 1e-5)
    out.backward(dy)
    y, _ = oracle.rmsnorm_fwd(x.detach().numpy(), g.detach().numpy(), 1e-5)
    assert np.max(np.abs(y - out.detach().numpy())) < 1e-13
    dx, dg = oracle.rmsnorm_bwd(x.detach().numpy(), dy.numpy(), g.detach().numpy(), 1e-5)
    assert np.max(np.abs(dx - x.grad.numpy())) < 1e-12
    assert np.max(np.abs(dg - g.grad.numpy())) < 1e-12


def test_rmsnorm_bwd_finite_differences():
    x = RNG.standard_normal((4, 16)) + 0.5
    g = RNG.uniform(0.5, 1.5, 16)
    dy = RNG.standard_normal((4, 16))
    dx, dg = oracle.rmsnorm_bwd(x, dy, g, 1e-5)
    h = 1e-6

    def loss(xx, gg):
        return np.sum(dy * oracle.rmsnorm_fwd(xx, gg, 1e-5)[0])

    for m in range(4):
        for i in range(16):
            xp = x.copy(); xp[m, i] += h
            xm = x.copy(); xm[m, i] -= h
            assert abs((loss(xp, g) - loss(xm, g)) / (2 * h) - dx[m, i]) <= 1e-7 * max(1, abs(dx[m, i]))
    for j in range(16):
        gp = g.copy(); gp[j] += h
        gm = g.copy(); gm[j] -= h
        assert abs((loss(x, gp) - loss(x, gm)) / (2 * h) - dg[j]) < 1e-7


# ------------------------------------------------------------------ codecs
def test_e4m3_decode_all_codes_match_torch():
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.decode_e4m3(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert nan.sum() == 2  # S.1111.111 only
    assert np.array_equal(ours[~nan], ref[~nan])
    assert ours[0x7E] == 448.0 and ours[1] == 2.0 ** -9


def test_e4m3_encode_roundtrip_and_torch_in_range():
    finite = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], dtype=np.uint8)
    vals = oracle.decode_e4m3(finite)
    back = oracle.encode_e4m3(vals)
    # +0 and -0 both exist; compare values
    assert np.array_equal(oracle.decode_e4m3(back), vals)
    x = np.concatenate([RNG.standard_normal(200000) * 50, RNG.uniform(-460, 460, 100000),
                        RNG.standard_normal(50000) * 1e-3]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    ours = oracle.encode_e4m3(x.astype(np.float64))
    # torch is RNE inside the finite range (|x| < 464)
    assert np.array_equal(oracle.decode_e4m3(ours), oracle.decode_e4m3(ref))


def test_e4m3_ties_and_saturation():
    enc = lambda v: oracle.decode_e4m3(oracle.encode_e4m3(np.array([v])))[0]
    assert enc(2.0 ** -10) == 0.0            # half of the smallest subnormal: tie to even (0)
    assert enc(1.5 * 2.0 ** -10) == 2.0 ** -9
    assert enc(1.0 + 1.0 / 16) == 1.0        # tie between 1 and 1.125 -> even (1)
    assert enc(1.0 + 3.0 / 16) == 1.25       # tie between 1.125 and 1.25 -> even (1.25)
    assert enc(460.0) == 448.0
    assert enc(1e9) == 448.0 and enc(-1e9) == -448.0
    assert oracle.encode_e4m3(np.array([np.nan]))[0] == 0x7F
    assert oracle.e4m3_step(1.0) == 0.125 and oracle.e4m3_step(300.0) == 32.0
    assert oracle.e4m3_step(2.0 ** -8) == 2.0 ** -9


def test_bf16_decode_and_encode_against_torch():
    bits = np.arange(65536, dtype=np.uint32).astype(np.uint16)
    ours = oracle.decode_bf16(bits)
    ref = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])
    # FP32 inputs: torch's FP32 -> BF16 conversion is round-to-nearest-even
    x = np.concatenate([RNG.standard_normal(300000) * 10.0 ** RNG.integers(-30, 30, 300000)]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(oracle.encode_bf16(x.astype(np.float64)), ref)


def test_bf16_encode_from_double_has_no_double_rounding():
    # 1 + 2^-8 + 2^-30 is just above the tie between 1 and 1 + 2^-7: RNE gives
    # 1 + 2^-7 (a conversion through FP32 would first drop 2^-30 and tie to 1)
    v = 1.0 + 2.0 ** -8 + 2.0 ** -30
    assert oracle.decode_bf16(oracle.encode_bf16(np.array([v])))[0] == 1.0 + 2.0 ** -7
    assert oracle.decode_bf16(oracle.encode_bf16(np.array([1.0 + 2.0 ** -8])))[0] == 1.0
    assert oracle.decode_bf16(oracle.encode_bf16(np.array([1.0 + 3 * 2.0 ** -8])))[0] == 1.0 + 2.0 ** -6


def test_fsum_is_compensated():
    v = np.array([1e16, 1.0, -1e16, 1.0] * 1000)
    assert oracle.fsum(v) == math.fsum(v) == 2000.0


# -------------------------------------------------------- selector network
def _mlp_case(n=9, C=7, seed=0):
    from oracle import mlp

    rng = np.random.default_rng(seed)
    params = rng.standard_normal(mlp.num_params(C)) * 0.3
    feats = rng.standard_normal((n, 12)) * 2 + 1
    mu, sd = feats.mean(0), feats.std(0) + 0.5
    mask = rng.random((n, C)) < 0.7
    mask[:, 0] = True
    t = rng.random((n, C)) * mask
    t /= t.sum(1, keepdims=True)
    return params, mu, sd, feats, t, mask


def test_mlp_forward_closed_form():
    from oracle import mlp

    C = 3
    P = {"W1": np.zeros((64, 12)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((C, 64)), "b3": np.array([1.0, -2.0, 0.5])}
    P["W1"][0, 3] = 2.0   # h1_0 = ReLU(2 z_3)
    P["W2"][5, 0] = -1.0  # h2_5 = ReLU(-h1_0)
    P["W3"][1, 5] = 3.0
    P["W3"][2, 0] = 7.0   # h2_0 = 0 always
    f = np.zeros((2, 12)); f[0, 3] = 1.5; f[1, 3] = -1.5
    logits, _ = mlp.forward(mlp.pack(P, C), np.zeros(12), np.ones(12), f, C)
    assert np.allclose(logits[0], [1.0, -2.0, 0.5])          # h1_0 = 3 -> h2_5 = 0
    assert np.allclose(logits[1], [1.0, -2.0, 0.5])          # h1_0 = 0
    # uniform logits over the legal set, one-hot target -> loss = log(#legal)
    P["b3"][:] = 0.0
    mask = np.array([[True, True, False], [True, True, True]])
    tgt = np.array([[1.0, 0, 0], [0, 0, 1.0]])
    loss, _ = mlp.loss_and_grad(mlp.pack(P, C), np.zeros(12), np.ones(12), np.zeros((2, 12)), tgt, mask, C)
    assert abs(loss - (math.log(2) + math.log(3)) / 2) < 1e-15


def test_mlp_gradient_finite_differences():
    from oracle import mlp

    params, mu, sd, feats, t, mask = _mlp_case()
    loss, g = mlp.loss_and_grad(params, mu, sd, feats, t, mask, 7)
    rng = np.random.default_rng(1)
    idx = rng.choice(params.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        pp = params.copy(); pp[i] += h
        pm = params.copy(); pm[i] -= h
        fd = (mlp.loss_and_grad(pp, mu, sd, feats, t, mask, 7)[0] - mlp.loss_and_grad(pm, mu, sd, feats, t, mask, 7)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9


def test_mlp_adam_first_step_is_signed_lr():
    from oracle import mlp

    # with bias correction the first Adam step moves each weight by ~lr * sign(g)
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    new, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(new, p - 0.01 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8), rtol=1e-12)
