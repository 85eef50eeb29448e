"""Rows for the row-quantisation tests and the exact code by brute force.

The code of an element is defined as the grid point nearest to the real
number x * Q / amax, ties to the even code (Q = 127: the integers -127..127;
Q = 448: the finite e4m3 values).  ``exact_codes`` finds it by brute force
over the whole grid in rational arithmetic, independently of the oracle.

Two kinds of rows stress the decision:

* exact ties of x * Q / amax whose amax makes Q / amax inexact in FP32, so an
  FP32 evaluation of x * fl32(Q / amax) lands beside the midpoint instead of
  on it (``tie_rows``; every value has at most 8 significant bits, so BF16
  holds the rows exactly);
* FP32 values found by a seeded search next to a decision boundary where the
  FP32 product x * fl32(Q / amax) rounds to another code than x * Q / amax
  (``fp32_departure_rows``)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import torch

Q_OF = {"int8": 127, "fp8": 448}


def _e4m3_grid():
    codes = np.arange(256, dtype=np.uint8)
    vals = torch.from_numpy(codes).view(torch.float8_e4m3fn).double().numpy()
    keep = np.isfinite(vals)
    return codes[keep], [Fraction(float(v)) for v in vals[keep]]


_E4M3 = _e4m3_grid()


def exact_codes(x: np.ndarray, fmt: str) -> np.ndarray:
    """Codes of one row (uint8 storage: int8 two's complement or e4m3) by brute
    force over the grid with rational arithmetic."""
    x = np.asarray(x, dtype=np.float32)
    amax = Fraction(float(np.max(np.abs(x))))
    out = np.zeros(x.shape, dtype=np.uint8)
    if amax == 0:
        if fmt == "fp8":
            out[np.signbit(x)] = 0x80
        return out
    q = Q_OF[fmt]
    for i, xi in enumerate(x.tolist()):
        v = Fraction(xi) * q / amax
        if fmt == "int8":
            cands = range(-127, 128)
            d = [abs(Fraction(c) - v) for c in cands]
            best = min(d)
            ties = [c for c, dc in zip(cands, d) if dc == best]
            c = ties[0] if len(ties) == 1 else [t for t in ties if t % 2 == 0][0]
            out[i] = np.uint8(c & 0xFF)
        else:
            codes, vals = _E4M3
            d = [abs(g - v) for g in vals]
            best = min(d)
            ties = [(int(codes[j]), vals[j]) for j in range(len(vals)) if d[j] == best]
            # +0 and -0 are one value: take the sign of x
            if all(t[1] == 0 for t in ties):
                out[i] = 0x80 if np.signbit(np.float32(xi)) else 0x00
                continue
            mags = {t[0] for t in ties}
            pick = [c for c in sorted(mags) if c % 2 == 0] if len(mags) > 1 else sorted(mags)
            out[i] = np.uint8(pick[0])
    return out


def _exact_one(x: float, amax: float, fmt: str) -> int:
    """The code of one value x > 0 (search helper; the pins use exact_codes)."""
    v = Fraction(x) * Q_OF[fmt] / Fraction(amax)
    if fmt == "int8":
        f = v.numerator // v.denominator
        r = v - f
        c = f if r < Fraction(1, 2) else f + 1 if r > Fraction(1, 2) else (f if f % 2 == 0 else f + 1)
        return int(c) & 0xFF
    codes, vals = _E4M3
    order = sorted((g, int(c)) for g, c in zip(vals, codes) if g >= 0 and not (g == 0 and c != 0))
    lo = max(i for i, (g, _) in enumerate(order) if g <= v)
    if lo + 1 < len(order):
        g0, c0 = order[lo]
        g1, c1 = order[lo + 1]
        mid = (g0 + g1) / 2
        if v > mid or (v == mid and c0 % 2 == 1):
            return c1
    return order[lo][1]


def fp32_product_codes(x: np.ndarray, fmt: str) -> np.ndarray:
    """Codes of v = x * fl32(Q / amax) rounded to FP32, then to the grid (numpy
    FP32 arithmetic; torch's e4m3fn rounding)."""
    x = np.asarray(x, dtype=np.float32)
    amax = np.float32(np.max(np.abs(x)))
    inv = np.float32(Q_OF[fmt]) / amax if amax > 0 else np.float32(1.0)
    v = (x * inv).astype(np.float32)
    if fmt == "int8":
        return np.clip(np.rint(v), -127, 127).astype(np.int8).view(np.uint8)
    v = np.clip(v, -448.0, 448.0).astype(np.float32)
    return torch.from_numpy(v).to(torch.float8_e4m3fn).view(torch.uint8).numpy()


def _midpoints(fmt: str):
    if fmt == "int8":
        return [Fraction(2 * c + 1, 2) for c in range(0, 127)]
    _, vals = _E4M3
    pos = sorted({v for v in vals if v >= 0})
    return [(a + b) / 2 for a, b in zip(pos[:-1], pos[1:])]


def tie_rows(N: int, fmt: str, seed: int = 0) -> np.ndarray:
    """Rows whose amax has an odd part other than 1 (so Q / amax is inexact in
    FP32) and whose other values put x * Q / amax exactly on a midpoint.  All
    values have at most 8 significant bits.  int8: 127 is prime, so with such
    an amax the only tie is x = +-amax / 2 (63.5); e4m3: midpoints with a
    factor 7 in their numerator (21/16 2^e and 7/2 2^-9) and amax with at most
    six significant bits."""
    rng = np.random.default_rng([61, N, seed, fmt == "int8"])
    rows = []
    if fmt == "int8":
        for amax in (3.0, 5.0 * 2 ** -3, 11.0 * 2 ** 4, 255.0, 7.0 * 2 ** -20):
            r = np.zeros(N)
            pos = rng.permutation(N)
            r[pos[: N // 2]] = amax / 2 * np.where(rng.random(N // 2) < 0.5, -1, 1)
            r[pos[N // 2]] = amax
            rows.append(r)
    else:
        for amax in (5.0, 11.0 * 2 ** -2, 37.0 * 2 ** 3, 13.0, 45.0 * 2 ** -30):
            r = np.zeros(N)
            e = rng.integers(-6, 8, N)
            m = Fraction(21, 16)
            vals = np.array([float(m * Fraction(2) ** int(k) * Fraction(amax) / 448) for k in e])
            sub = rng.random(N) < 0.15
            vals[sub] = float(Fraction(7, 2) * Fraction(1, 512) * Fraction(amax) / 448)
            vals *= np.where(rng.random(N) < 0.5, -1, 1)
            r[:] = vals
            r[rng.integers(N)] = amax
            rows.append(r)
    x = np.array(rows, dtype=np.float64)
    assert np.array_equal(x.astype(np.float32).astype(np.float64), x)
    return x


def fp32_departure_rows(N: int, fmt: str, seed: int = 0, per_row: int = 24) -> np.ndarray:
    """FP32 rows holding values where the FP32 product and the definition give
    different codes (found next to the decision boundaries of a random amax);
    the rest of each row is random and below amax."""
    rng = np.random.default_rng([67, N, seed, fmt == "int8"])
    q = Q_OF[fmt]
    mids = _midpoints(fmt)
    rows = []
    while len(rows) < 4:
        amax = np.float32(rng.uniform(1.0, 100.0))
        found = []
        for _ in range(4000):
            b = mids[rng.integers(len(mids))]
            x0 = np.float32(float(b * Fraction(float(amax)) / q))
            for k in range(-3, 4):
                xv = np.float32(x0)
                step = np.float32(np.inf) if k > 0 else np.float32(-np.inf)
                for _ in range(abs(k)):
                    xv = np.nextafter(xv, step)
                if abs(xv) > amax:
                    continue
                pair = np.array([amax, xv], dtype=np.float32)
                if _exact_one(float(xv), float(amax), fmt) != fp32_product_codes(pair, fmt)[1]:
                    found.append(float(xv) * (1 if rng.random() < 0.5 else -1))
            if len(found) >= per_row:
                break
        if len(found) < per_row:
            continue
        r = rng.uniform(-1, 1, N) * float(amax) * 0.99
        pos = rng.permutation(N)
        r[pos[: len(found)]] = found
        r[pos[len(found)]] = float(amax)
        rows.append(r.astype(np.float32).astype(np.float64))
    return np.array(rows)
