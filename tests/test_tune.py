"""Selector dataset plumbing on the CPU: the shape sampler (stratification,
the aligned set, resumable prefixes), feature recomputation on load, soft
targets and the stratified split."""
import json
import math

import numpy as np

from paper_2609_01864_amd import credit as C
from paper_2609_01864_amd import tune as T


def test_sampler_is_stratified_bounded_and_resumable(lib_built):
    a = T.sample_shapes(360)
    assert a[:180] == T.sample_shapes(180)  # a longer run extends a shorter one
    combos = {(s["op"], s["dir"], s["dt"]) for s in a}
    assert len(combos) == 18
    for s in a:
        assert 1 <= s["M"] <= 16384 and 1024 <= s["N"] <= 4194304
        assert T.io_bytes(s["op"], s["dir"], s["dt"], s["M"], s["N"]) <= T.MAX_IO_BYTES
    al = T.sample_shapes(180, seed=5, align=64)
    assert all(s["N"] % 64 == 0 and s["N"] >= 1024 for s in al)
    assert {T.key_of(s) for s in al}.isdisjoint({T.key_of(s) for s in a})


def test_load_recomputes_features_and_targets(lib_built, tmp_path):
    rec = {"op": C.LAYERNORM, "dir": C.FWD, "dt": C.F32, "M": 1024, "N": 8192, "legal": [0, 1, 2],
           "times": {"0": 20.0, "1": 15.0, "2": 21.0}, "ctrl": {"1": 5.0}, "feats": [0.0] * 12}
    path = tmp_path / "t.jsonl"
    path.write_text(json.dumps(rec) + "\n")
    r = T.load(str(path))[0]
    assert np.allclose(r["feats"], C.features(C.LAYERNORM, C.FWD, C.F32, 1024, 8192))
    assert r["feats"][6] == 1.0  # whole aligned vectors
    t, m = T.soft_targets(r)
    assert list(m[:3]) == [1, 1, 1] and m[3:].sum() == 0
    assert math.isclose(t.sum(), 1.0) and t.argmax() == 1
    # tau = 0.02: a plan 5% slower than the best weighs exp(-2.5) of it
    assert math.isclose(t[0] / t[1], math.exp(-(20.0 / 15.0 - 1.0) / T.TAU))


def test_split_is_stratified_and_deterministic(lib_built):
    recs = [dict(s, times={"0": 1.0}) for s in T.sample_shapes(360)]
    tr, te = T.split(recs)
    tr2, te2 = T.split(list(reversed(recs)))
    assert [T.key_of(r) for r in te] == [T.key_of(r) for r in te2]
    assert len(tr) + len(te) == len(recs) and len(te) == 18 * 4


def test_noise_aware_regret_and_judge_tie_break():
    # plan 2 (split k=2) is 0.5% slower than the two-pass plan: within the 1%
    # noise floor, so the judge takes the plan moving fewer bytes (split k=2
    # before two-pass); plan 3 is 3% slower but with MADs of 1%, 2 MAD covers it
    rec = {"times": {"0": 100.0, "2": 100.5, "3": 103.0, "4": 110.0},
           "spread": {"0": {"mad": 1.0}, "2": {"mad": 0.1}, "3": {"mad": 1.6}, "4": {"mad": 0.5}}}
    assert T.judge_best(rec) == 2
    st = T.regret_stats([rec] * 4, [0, 2, 3, 4])
    assert math.isclose(st["geomean"], (1.0 * 1.005 * 1.03 * 1.10) ** 0.25)
    assert math.isclose(st["noise_aware_geomean"], 1.10 ** 0.25)
    assert st["share_within_noise"] == 0.75 and st["share_judge_pick"] == 0.25
    # without spread (older records) only the 1% floor applies
    bare = {"times": {"0": 100.0, "2": 100.5, "3": 103.0}}
    assert T.judge_best(bare) == 2
    assert T.regret_stats([bare], [3])["noise_aware_geomean"] == 1.03
    # ranking by bytes: resident, split by increasing k, two-pass last
    assert sorted(range(C.NUM_PLANS), key=T.bytes_rank) == [1, 2, 3, 4, 5, 6, 0]


def test_learned_pick_breaks_near_ties_by_bytes():
    # the untimed pick: the largest logit among legal plans, or within 0.5 of
    # it (a predicted 1% under tau = 0.02) the plan moving the fewest bytes
    class Net:
        def mlp_predict(self, X):
            return np.tile(np.array([[2.0, 1.0, 1.3, 1.6, 0.0, 0.0, 0.0]], np.float32), (len(X), 1))

    recs = [{"feats": [0.0] * 12, "times": {"0": 1.0, "1": 1.0, "2": 1.0, "3": 1.0}},  # 0 best, 3 within
            {"feats": [0.0] * 12, "times": {"1": 1.0, "2": 1.0, "3": 1.0}},  # 3 best; 2 within, 1 not
            {"feats": [0.0] * 12, "times": {"1": 1.0, "3": 1.0}}]  # 3 best; 1 is 0.6 below
    assert T.pick_learned(Net(), recs) == [3, 2, 3]


def test_fresh_shapes_are_drawn_by_no_training_round(lib_built):
    # the fresh check judges the model on shapes it never saw: the shipped
    # model's collection (two rounds of 6000 ragged, 3000 aligned and 1000
    # power-of-two shapes, seeds 4-9, and 6000 dense shapes, seeds 30 and 31)
    # re-derived here, against the fresh draw
    reg = dict(m_range=(256, 16384), n_range=(8192, 1048576))
    train = set()
    for r in range(2):
        train |= {T.key_of(s) for s in T.sample_shapes(6000, seed=4 + 3 * r) +
                  T.sample_shapes(3000, seed=5 + 3 * r, align=64) + T.sample_shapes(1000, seed=6 + 3 * r, align=0)}
    train |= {T.key_of(s) for s in T.sample_shapes(3000, seed=30, **reg) +
              T.sample_shapes(3000, seed=31, align=64, **reg)}
    assert len(train) == 25924  # the distinct shapes of the shipped model's dataset
    fresh = T.fresh_shapes(1000)
    keys = {T.key_of(s) for s in fresh}
    assert len(fresh) >= 990 and len(keys) == len(fresh) and not keys & train
    assert sum(s["N"] % 64 == 0 for s in fresh) >= 495
