"""TEST INFRASTRUCTURE ONLY: float64 reference of the learned proposal's
network training (forward, backward, Adam), written plainly in numpy.

The network (an addition to the paper's method, which has none) maps the 32
quantised features of an edge to one logit: 32 -> 64 -> 64 -> 1 with ReLU.
Weights of layer l lie on the grid k 2^-e_l (|k| <= 127), biases on the same
grid; hidden activations are scaled by 2^a_l and rounded to integers in
[0, 127].  Training keeps float master weights and passes gradients straight
through the roundings (zero where a value is clamped).  Loss: mean binary
cross-entropy of the logit against committed (1) / rejected (0).

Flat parameter layout (6337 values): W1 (64 x 32, row = unit) | b1 (64) |
W2 (64 x 64) | b2 (64) | W3 (64) | b3.
"""
from __future__ import annotations

import numpy as np

NPARAM = 6337
O_W1, O_B1, O_W2, O_B2, O_W3, O_B3 = 0, 2048, 2112, 6208, 6272, 6336
BIAS_MAX = 2 ** 22


def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    return (P[O_W1:O_B1].reshape(64, 32), P[O_B1:O_W2], P[O_W2:O_B2].reshape(64, 64), P[O_B2:O_W3],
            P[O_W3:O_B3], P[O_B3])


def quant_w(w, e, quantize=True):
    """(quantised weight, straight-through mask)."""
    if not quantize:
        return w, np.ones_like(w)
    s = np.ldexp(w, e)
    k = np.clip(np.rint(s), -127, 127)
    return np.ldexp(k, -e), (np.abs(s) <= 127).astype(np.float64)


def quant_b(b, e, quantize=True):
    if not quantize:
        return b, np.ones_like(b)
    s = np.ldexp(b, e)
    k = np.clip(np.rint(s), -BIAS_MAX, BIAS_MAX)
    return np.ldexp(k, -e), (np.abs(s) <= BIAS_MAX).astype(np.float64)


def act(z, a, quantize=True):
    """(activation, derivative of the activation with respect to z)."""
    if not quantize:
        h = np.maximum(z, 0.0) * 2.0 ** a
        return h, (z > 0).astype(np.float64) * 2.0 ** a
    s = np.ldexp(np.maximum(z, 0.0), a)
    h = np.minimum(np.rint(s), 127.0)
    return h, ((z > 0) & (s <= 127)).astype(np.float64) * 2.0 ** a


def forward(P, meta, X, quantize=True):
    W1, b1, W2, b2, W3, b3 = unpack(P)
    e1, e2, e3, a1, a2 = (meta[k] for k in ("e1", "e2", "e3", "a1", "a2"))
    W1q, _ = quant_w(W1, e1, quantize)
    b1q, _ = quant_b(b1, e1, quantize)
    W2q, _ = quant_w(W2, e2, quantize)
    b2q, _ = quant_b(b2, e2, quantize)
    W3q, _ = quant_w(W3, e3, quantize)
    b3q, _ = quant_b(np.array([b3]), e3, quantize)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1q.T + b1q
    h1, d1 = act(z1, a1, quantize)
    z2 = h1 @ W2q.T + b2q
    h2, d2 = act(z2, a2, quantize)
    z3 = h2 @ W3q + b3q[0]
    return z3, (X, z1, h1, d1, z2, h2, d2, W1q, W2q, W3q)


def loss_and_grad(P, meta, X, y, quantize=True):
    """Mean BCE-with-logits loss and its gradient (straight-through)."""
    W1, b1, W2, b2, W3, b3 = unpack(P)
    e1, e2, e3 = meta["e1"], meta["e2"], meta["e3"]
    z3, (X, z1, h1, d1, z2, h2, d2, W1q, W2q, W3q) = forward(P, meta, X, quantize)
    y = np.asarray(y, dtype=np.float64)
    B = len(y)
    loss = np.mean(np.maximum(z3, 0) - y * z3 + np.log1p(np.exp(-np.abs(z3))))
    g3 = (1.0 / (1.0 + np.exp(-z3)) - y) / B          # d loss / d z3
    gW3 = h2.T @ g3
    gb3 = g3.sum()
    gz2 = np.outer(g3, W3q) * d2
    gW2 = gz2.T @ h1
    gb2 = gz2.sum(0)
    gz1 = (gz2 @ W2q) * d1
    gW1 = gz1.T @ X
    gb1 = gz1.sum(0)
    _, m1 = quant_w(W1, e1, quantize)
    _, mb1 = quant_b(b1, e1, quantize)
    _, m2 = quant_w(W2, e2, quantize)
    _, mb2 = quant_b(b2, e2, quantize)
    _, m3 = quant_w(W3, e3, quantize)
    _, mb3 = quant_b(np.array([b3]), e3, quantize)
    g = np.concatenate([(gW1 * m1).ravel(), gb1 * mb1, (gW2 * m2).ravel(), gb2 * mb2, gW3 * m3, [gb3 * mb3[0]]])
    return loss, g


def adam(P, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t = 1 for the first); returns new (P, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v


def model_dict(P, meta, threshold):
    """The network as the simplifier takes it: quantised weights (float32)."""
    W1, b1, W2, b2, W3, b3 = unpack(P)
    e1, e2, e3 = meta["e1"], meta["e2"], meta["e3"]
    return {"w1": quant_w(W1, e1)[0].astype(np.float32), "b1": quant_b(b1, e1)[0].astype(np.float32),
            "w2": quant_w(W2, e2)[0].astype(np.float32), "b2": quant_b(b2, e2)[0].astype(np.float32),
            "w3": quant_w(W3, e3)[0].astype(np.float32),
            "b3": float(quant_b(np.array([b3]), e3)[0][0]),
            "e1": e1, "e2": e2, "e3": e3, "a1": meta["a1"], "a2": meta["a2"], "threshold": float(threshold)}
