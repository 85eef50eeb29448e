"""FP64 reference of the learned plan selector's network (TEST INFRASTRUCTURE
ONLY; see the package docstring).  Not part of the paper, whose model fits no
coefficient: this is the plain definition of the network the library trains.

Network: standardized features z = (f - mu) / sd; h1 = ReLU(W1 z + b1);
h2 = ReLU(W2 h1 + b2); logits = W3 h2 + b3.  Parameters are one flat vector in
the order W1 [64][12], b1 [64], W2 [64][64], b2 [64], W3 [C][64], b3 [C].
Loss: masked soft-target cross-entropy averaged over samples,
L = -(1/n) sum_s sum_{c legal} t_sc log softmax_legal(logits_s)_c.
Optimiser: Adam (beta1, beta2, eps) with bias correction.
"""
from __future__ import annotations

import numpy as np

F, H = 12, 64


def shapes(C: int):
    return [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (C, H)), ("b3", (C,))]


def num_params(C: int) -> int:
    return sum(int(np.prod(s)) for _, s in shapes(C))


def unpack(params, C: int):
    p = np.asarray(params, dtype=np.float64)
    out, off = {}, 0
    for name, s in shapes(C):
        n = int(np.prod(s))
        out[name] = p[off:off + n].reshape(s)
        off += n
    assert off == p.size
    return out


def pack(d, C: int) -> np.ndarray:
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in shapes(C)])


def forward(params, mu, sd, feats, C: int):
    """Returns (logits, cache)."""
    P = unpack(params, C)
    z = (np.asarray(feats, np.float64) - np.asarray(mu, np.float64)) / np.asarray(sd, np.float64)
    a1 = z @ P["W1"].T + P["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(a2, 0.0)
    logits = h2 @ P["W3"].T + P["b3"]
    return logits, (z, a1, h1, a2, h2)


def masked_log_softmax(logits, mask):
    m = np.asarray(mask, bool)
    lg = np.where(m, logits, -np.inf)
    mx = lg.max(axis=1, keepdims=True)
    lse = mx + np.log(np.sum(np.where(m, np.exp(lg - mx), 0.0), axis=1, keepdims=True))
    return np.where(m, logits - lse, 0.0)


def loss_and_grad(params, mu, sd, feats, targets, mask, C: int):
    logits, (z, a1, h1, a2, h2) = forward(params, mu, sd, feats, C)
    n = logits.shape[0]
    m = np.asarray(mask, bool)
    t = np.asarray(targets, np.float64)
    lp = masked_log_softmax(logits, m)
    loss = -np.sum(np.where(m, t * lp, 0.0)) / n
    p = np.where(m, np.exp(lp), 0.0)
    dl = np.where(m, (p - t) / n, 0.0)
    P = unpack(params, C)
    g = {}
    g["W3"] = dl.T @ h2
    g["b3"] = dl.sum(0)
    dh2 = (dl @ P["W3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ P["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ z
    g["b1"] = dh1.sum(0)
    return loss, pack(g, C)


def adam_step(params, grad, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
