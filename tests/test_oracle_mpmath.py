"""The FP64 oracle against the plain definitions evaluated in 50-digit
arithmetic (mpmath) on tiny inputs (4 rows x 8 columns, including rows offset
by 10 and scaled by 1e3 / 1e-3): softmax forward and backward, LayerNorm and
RMSNorm forward and backward (dx, dgamma, dbeta).  Each 50-digit value is
computed from the definition written out independently here; the oracle
must agree to within a few FP64 rounding errors of the magnitudes involved."""
import mpmath as mp
import numpy as np
import pytest

import oracle

mp.mp.dps = 50
EPS = 1e-5
RNG = np.random.default_rng(20261203)


def _rows():
    x = RNG.standard_normal((4, 8))
    x[1] += 10.0          # offset rows stress x - mean
    x[2] *= 1e3
    x[3] = x[3] * 1e-3 + 0.5
    return x


def _mp_softmax(row):
    m = max(row)
    e = [mp.exp(mp.mpf(v) - m) for v in row]
    s = mp.fsum(e)
    return [v / s for v in e]


def _mp_ln(row, g, b):
    n = len(row)
    xs = [mp.mpf(v) for v in row]
    mu = mp.fsum(xs) / n
    var = mp.fsum([(v - mu) ** 2 for v in xs]) / n
    r = 1 / mp.sqrt(var + mp.mpf(EPS))
    return [(v - mu) * r * mp.mpf(gi) + mp.mpf(bi) for v, gi, bi in zip(xs, g, b)], mu, r


def _mp_rms(row, g):
    n = len(row)
    xs = [mp.mpf(v) for v in row]
    r = 1 / mp.sqrt(mp.fsum([v * v for v in xs]) / n + mp.mpf(EPS))
    return [v * r * mp.mpf(gi) for v, gi in zip(xs, g)], r


def _close(got, ref, mag, rel):
    ref = np.array([float(v) for v in ref])
    assert np.all(np.abs(got - ref) <= rel * mag), (got, ref)


def test_softmax_forward_and_backward_50_digits():
    x = _rows()
    dy = RNG.standard_normal((4, 8))
    y = oracle.softmax_fwd(x)
    dx = oracle.softmax_bwd(y, dy)
    for m in range(4):
        ys = _mp_softmax(x[m])
        # exp amplifies the rounding of x - max (one FP64 subtraction): a
        # relative error of |x - max| 2^-53 on top of a few roundings
        cond = 1.0 + np.abs(x[m] - x[m].max()) * 2.0 ** -53 / 4e-15
        _close(y[m], ys, np.abs(y[m]) * cond, 4e-15)
        # backward from the given y (its FP64 values), dx_i = y_i (dy_i - sum_j dy_j y_j)
        yy = [mp.mpf(v) for v in y[m]]
        c = mp.fsum([mp.mpf(d) * v for d, v in zip(dy[m], yy)])
        ref = [v * (mp.mpf(d) - c) for v, d in zip(yy, dy[m])]
        mag = np.abs(y[m]) * (np.abs(dy[m]) + np.sum(np.abs(dy[m] * y[m])))
        _close(dx[m], ref, mag, 4e-15)


def test_layernorm_forward_and_backward_50_digits():
    x = _rows()
    g = RNG.uniform(0.5, 1.5, 8)
    b = RNG.normal(0, 0.1, 8)
    dy = RNG.standard_normal((4, 8))
    y, mean, rstd = oracle.layernorm_fwd(x, g, b, EPS)
    dx, dg, db = oracle.layernorm_bwd(x, dy, g, EPS)
    ref_dg = [mp.mpf(0)] * 8
    ref_db = [mp.mpf(0)] * 8
    for m in range(4):
        ys, mu, r = _mp_ln(x[m], g, b)
        mag = np.abs(x[m] - mean[m]) * rstd[m] * g + np.abs(b) + np.abs(mean[m]) * rstd[m] * g
        _close(y[m], ys, mag, 1e-14)
        assert abs(mean[m] - float(mu)) <= 1e-15 * max(np.abs(x[m]))
        assert abs(rstd[m] - float(r)) <= 1e-14 * rstd[m]
        # backward: xhat, gg = dy gamma, dx = r (gg - mean gg - xhat mean(gg xhat))
        xh = [(mp.mpf(v) - mu) * r for v in x[m]]
        gg = [mp.mpf(d) * mp.mpf(gi) for d, gi in zip(dy[m], g)]
        c1 = mp.fsum(gg) / 8
        c2 = mp.fsum([a * b_ for a, b_ in zip(gg, xh)]) / 8
        ref = [r * (a - c1 - h * c2) for a, h in zip(gg, xh)]
        magd = rstd[m] * (np.abs(dy[m] * g) + np.abs(dy[m] * g).mean()
                          + np.abs(x[m]) * rstd[m] * np.abs(dy[m] * g).mean() * 10)
        _close(dx[m], ref, magd, 1e-13)
        for j in range(8):
            ref_dg[j] += mp.mpf(dy[m, j]) * xh[j]
            ref_db[j] += mp.mpf(dy[m, j])
    _close(dg, ref_dg, np.abs(dy).sum(0) * (np.abs(x) * rstd[:, None]).max(), 1e-13)
    _close(db, ref_db, np.abs(dy).sum(0), 1e-15)


def test_rmsnorm_forward_and_backward_50_digits():
    x = _rows()
    g = RNG.uniform(0.5, 1.5, 8)
    dy = RNG.standard_normal((4, 8))
    y, rstd = oracle.rmsnorm_fwd(x, g, EPS)
    dx, dg = oracle.rmsnorm_bwd(x, dy, g, EPS)
    ref_dg = [mp.mpf(0)] * 8
    for m in range(4):
        ys, r = _mp_rms(x[m], g)
        _close(y[m], ys, np.abs(x[m]) * rstd[m] * g, 4e-15)
        assert abs(rstd[m] - float(r)) <= 4e-15 * rstd[m]
        xh = [mp.mpf(v) * r for v in x[m]]
        gg = [mp.mpf(d) * mp.mpf(gi) for d, gi in zip(dy[m], g)]
        c = mp.fsum([a * b_ for a, b_ in zip(gg, xh)]) / 8
        ref = [r * (a - h * c) for a, h in zip(gg, xh)]
        magd = rstd[m] * (np.abs(dy[m] * g) + np.abs(x[m]) * rstd[m] * np.abs(dy[m] * g * x[m] * rstd[m]).mean())
        _close(dx[m], ref, magd, 1e-14)
        for j in range(8):
            ref_dg[j] += mp.mpf(dy[m, j]) * xh[j]
    _close(dg, ref_dg, (np.abs(dy) * np.abs(x) * rstd[:, None]).sum(0), 1e-14)


@pytest.mark.parametrize("mistake", ["unbiased", "eps_outside"])
def test_a_planted_mistake_is_caught_at_50_digits(mistake):
    # the comparison above distinguishes the definition from its usual slips
    x = _rows()
    g = np.ones(8)
    b = np.zeros(8)
    y, _, _ = oracle.layernorm_fwd(x, g, b, EPS)
    mu = x.mean(1, keepdims=True)
    if mistake == "unbiased":
        wrong = (x - mu) / np.sqrt(x.var(1, ddof=1, keepdims=True) + EPS)
    else:
        wrong = (x - mu) / (np.sqrt(x.var(1, keepdims=True)) + EPS)
    assert np.max(np.abs(wrong - y)) > 1e-6
