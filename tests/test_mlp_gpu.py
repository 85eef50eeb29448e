"""The learned selector's HIP kernels (forward, masked soft-target loss and
gradient, Adam) against the FP64 CPU network from identical parameters, model
file round trip and rejection, and learnability of a known rule."""
import os

import numpy as np
import pytest

from oracle import mlp as ref
from paper_2609_01864_amd import credit as C

pytestmark = pytest.mark.gpu
NC = C.NUM_PLANS


def _case(n=257, seed=0):
    rng = np.random.default_rng(seed)
    params = (rng.standard_normal(ref.num_params(NC)) * 0.2).astype(np.float32)
    feats = (rng.standard_normal((n, 12)) * 3 + 2).astype(np.float32)
    mu = feats.mean(0).astype(np.float32)
    sd = (feats.std(0) + 0.5).astype(np.float32)
    mask = (rng.random((n, NC)) < 0.6).astype(np.uint8)
    mask[:, 0] = 1
    t = rng.random((n, NC)) * mask
    t = (t / t.sum(1, keepdims=True)).astype(np.float32)
    return params, mu, sd, feats, t, mask


def test_param_count_matches_reference(lib_built):
    assert C.lib().credit_mlp_num_params() == ref.num_params(NC) == 12 * 64 + 64 + 64 * 64 + 64 + NC * 64 + NC


def test_forward_and_gradient_match_fp64(gpu_handle):
    params, mu, sd, feats, t, mask = _case()
    gpu_handle.mlp_set(params, mu, sd)
    logits = gpu_handle.mlp_predict(feats)
    rl, _ = ref.forward(params, mu, sd, feats, NC)
    assert np.max(np.abs(logits - rl)) <= 1e-5 * max(1.0, np.abs(rl).max())
    loss, g = gpu_handle.mlp_grad(feats, t, mask)
    rloss, rg = ref.loss_and_grad(params, mu, sd, feats, t, mask.astype(bool), NC)
    assert abs(loss - rloss) <= 1e-5 * max(1.0, abs(rloss))
    assert np.max(np.abs(g - rg)) <= 1e-5 * max(1e-3, np.abs(rg).max())


def test_one_adam_step_matches_fp64(gpu_handle):
    params, mu, sd, feats, t, mask = _case(seed=1)
    gpu_handle.mlp_set(params, mu, sd)
    gpu_handle.mlp_train(feats, t, mask, epochs=1, lr=1e-3, seed=0)
    got, _, _ = gpu_handle.mlp_get()
    _, rg = ref.loss_and_grad(params, mu, sd, feats, t, mask.astype(bool), NC)
    want, _, _ = ref.adam_step(params.astype(np.float64), rg, np.zeros_like(rg), np.zeros_like(rg), 1, 1e-3)
    # the first step moves each weight by ~lr: compare the step itself
    step, rstep = got - params, want - params
    assert np.max(np.abs(step - rstep)) <= 1e-5 * 1e-3 + 2e-7


def test_training_learns_a_rule_and_reduces_loss(gpu_handle):
    rng = np.random.default_rng(3)
    n = 600
    feats = rng.standard_normal((n, 12)).astype(np.float32) * 2
    cls = np.where(feats[:, 8] > 0.5, 4, np.where(feats[:, 7] < -1, 0, 1))
    mask = np.ones((n, NC), np.uint8)
    t = np.full((n, NC), 1e-3, np.float32)
    t[np.arange(n), cls] = 1.0
    t /= t.sum(1, keepdims=True)
    l0 = gpu_handle.mlp_train(feats, t, mask, epochs=1, lr=3e-3, seed=7)
    l1 = gpu_handle.mlp_train(feats, t, mask, epochs=1500, lr=3e-3, seed=7)
    assert l1 < 0.5 * l0
    acc = np.mean(gpu_handle.mlp_predict(feats).argmax(1) == cls)
    assert acc >= 0.95, acc


def test_model_file_round_trip_and_rejection(gpu_handle, tmp_path):
    params, mu, sd, feats, t, mask = _case(seed=2)
    gpu_handle.mlp_set(params, mu, sd)
    path = str(tmp_path / "m.txt")
    gpu_handle.save_model(path)
    before = gpu_handle.mlp_predict(feats)
    assert gpu_handle.load_model(path) == C.OK
    assert np.array_equal(gpu_handle.mlp_predict(feats), before)
    txt = open(path).read()
    bad = str(tmp_path / "bad.txt")
    open(bad, "w").write(txt.replace("arch gfx950", "arch gfx942"))
    assert gpu_handle.load_model(bad) == C.ERR_MODEL
    open(bad, "w").write(txt[: len(txt) // 2])
    assert gpu_handle.load_model(bad) == C.ERR_MODEL
    assert gpu_handle.load_model(str(tmp_path / "missing.txt")) == C.ERR_MODEL
    # without a model the default selection falls back to the fixed rule


def test_training_resumes_from_a_saved_checkpoint(lib_built, tmp_path):
    # 24 epochs in one call, and 12 + save / load (parameters, standardization,
    # Adam moments and step count in the file) + 12 on a fresh handle, take
    # the same steps: bit-identical networks
    _, _, _, feats, t, mask = _case(n=300, seed=5)
    path = str(tmp_path / "ckpt.txt")
    ha, hb, hc = (C.Handle(0, load_default_model=False) for _ in range(3))
    try:
        ha.mlp_train(feats, t, mask, epochs=24, lr=3e-3, seed=11)
        hb.mlp_train(feats, t, mask, epochs=12, lr=3e-3, seed=11)
        hb.save_model(path)
        assert hc.load_model(path) == C.OK
        hc.mlp_train(feats, t, mask, epochs=12, lr=3e-3, seed=0)
        for a, c in zip(ha.mlp_get(), hc.mlp_get()):
            assert np.array_equal(a, c)
        # without the moments (a format-1 file) the continuation differs
        txt = open(path).read()
        head, _, _ = txt.partition("adam ")
        v1 = head.replace("CREDIT-MLP 2", "CREDIT-MLP 1", 1)
        v1 = v1[:v1.index("library ")] + v1[v1.index("mu "):] + "end\n"
        open(path, "w").write(v1)
        assert hc.load_model(path) == C.OK
        hc.mlp_train(feats, t, mask, epochs=12, lr=3e-3, seed=0)
        assert not np.array_equal(ha.mlp_get()[0], hc.mlp_get()[0])
        # a file whose plan classes differ from the library's is refused
        bad = txt.replace("classes 0:1 1:1 2:2", "classes 0:1 1:1 2:4", 1)
        assert bad != txt
        open(path, "w").write(bad)
        assert hc.load_model(path) == C.ERR_MODEL
    finally:
        for h in (ha, hb, hc):
            h.close()


def test_timed_learned_selector_keeps_the_faster_of_the_two_best(gpu_handle):
    # the untimed pick is the tie rule's (among legal plans within 0.5 of the
    # best logit, the one moving the fewest bytes); the timed selector times
    # the shipped model's two highest-scoring legal plans once and keeps one
    # of them, the faster by the library's own timing
    from paper_2609_01864_amd import tune as T

    h = C.Handle(0)
    try:
        assert h.model_loaded
        M, N = 1024, 524288
        op = C.LAYERNORM
        f = C.features(op, C.FWD, C.F32, M, N)
        lg = h.mlp_predict(f[None, :])[0]
        legal = [c for c in range(NC) if h.plan_legal(op, C.FWD, C.F32, M, N, C.plan_of_class(c))]
        top2 = sorted(legal, key=lambda c: -lg[c])[:2]
        best = max(lg[c] for c in legal)
        untimed = min((c for c in legal if best - lg[c] <= T.TIE_LOGIT), key=T.bytes_rank)
        h.set_selector(C.SEL_LEARNED)
        assert h.select(op, C.FWD, C.F32, M, N)[0].as_tuple() == C.plan_of_class(untimed).as_tuple()
        h.set_selector(C.SEL_LEARNED_TIMED)
        p, pred = h.select(op, C.FWD, C.F32, M, N)
        assert p.as_tuple() in [C.plan_of_class(c).as_tuple() for c in top2]
        assert pred > 0
        # other operators fall back to the analytic model, which also predicts a time
        q, _ = h.select(C.QUANT_INT8, C.FWD, C.F32, 4096, 65536)
        assert h.plan_legal(C.QUANT_INT8, C.FWD, C.F32, 4096, 65536, q)
    finally:
        h.close()
