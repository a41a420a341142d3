"""FP64 oracle of the BF16 warm-start network (test infrastructure only).

Mirrors the GPU computation step by step in float64, rounding to BF16
(round to nearest even, 8 significant bits) at exactly the points where the
GPU stores BF16: the network input, the weights, the hidden activations and
the per-layer gradient with respect to the pre-activation.  Matrix products
and sums are exact-ish float64 (the GPU accumulates in float32).

Shares no code with the GPU path.  Pinned in tests/test_mlp_oracle.py by
closed-form rounding cases, by agreement with a plain float64 matrix product
when every operand is BF16-representable, and by central finite differences
of the unrounded network.
"""
from __future__ import annotations

import numpy as np


def bf16(x, rounding=True):
    """Round float64 values to the nearest BF16 value (ties to even)."""
    x = np.asarray(x, dtype=np.float64)
    if not rounding:
        return x
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def forward(X, weights, rounding=True):
    """Network output (float64) and the BF16 activations [input, h1, ...]."""
    h = bf16(X, rounding)
    acts = [h]
    L = len(weights)
    for l, (W, b) in enumerate(weights):
        z = h @ bf16(W, rounding).T + b
        if l < L - 1:
            h = bf16(np.maximum(z, 0.0), rounding)
            acts.append(h)
        else:
            return z, acts


def backward(dOut, weights, acts, rounding=True):
    """(dW, db) for d loss / d out = dOut, following the GPU's order."""
    L = len(weights)
    dW, db = [None] * L, [None] * L
    g = np.asarray(dOut, dtype=np.float64)
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            g = g * (acts[l + 1] > 0)
        g16 = bf16(g, rounding)
        dW[l] = g16.T @ acts[l]
        db[l] = g16.sum(axis=0)
        if l > 0:
            g = g16 @ bf16(weights[l][0], rounding)
    return dW, db


def mse(y, t):
    d = np.asarray(y, np.float64) - np.asarray(t, np.float64)
    return float((d * d).mean()), 2.0 * d / d.size


def adam(w, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015, Algorithm 1) in float64."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
