"""Literal masking reference for tiny signals (test infrastructure only).

Builds the arrays of arXiv 2501.04194 Sec. IV exactly as described there and
reduces them with numpy, as an independent check of the loop oracle in
``stl_oracle.c``:

* Sec. IV-B Step 1: pad the end of the signal and repeat it column-wise into
  a (L+P) x L array S with S[j, t] = s_j (padded rows hold the pad value).
* Step 2: the subsignal mask removes entries with j < t; the time-interval
  mask removes entries with j - t outside [a, b]; the final mask is their sum.
* Step 3: masked entries are replaced by a large value of the right sign and
  each column is reduced with max (Eventually) or min (Always).
* Sec. IV-C: Until stacks, for every i in [a, b], the 2-D masks of
  Always_[0,i] phi and Always_[i,i] psi into 3-D arrays, then reduces with a
  min over the stacked pair (S1, S2) and a max over i (S3).

Smooth variants replace the reductions by logsumexp (Sec. III-C) with masked
entries excluded; the smooth time mask (Sec. VI) enters as log-weights, on
the window offset (Eventually / Always) or on the Until index i.
P (number of pad rows) is b: the largest offset a window can reach.  The
paper pads by K = b - a + 1 rows, which is enough only when a <= 1 (as in
its Example 1).
"""
from __future__ import annotations

import numpy as np

BIG = 1e5   # "large" fill value used for masked-out entries


def unroll(s, P, pad_value):
    """Step 1: (L+P) x L array with S[j, t] = s_j (rows >= L hold the pad)."""
    L = len(s)
    col = np.concatenate([np.asarray(s, dtype=np.float64), np.full(P, pad_value, dtype=np.float64)])
    return np.repeat(col[:, None], L, axis=1)


def masks(L, P, a, b):
    """Step 2: keep-mask (True = kept) = not subsignal-masked and inside [a, b]."""
    j = np.arange(L + P)[:, None]
    t = np.arange(L)[None, :]
    subsig = j >= t                                        # M_subsig keeps j >= t
    time = (j - t >= a) & (j - t <= (b if b is not None else L + P))
    return subsig & time


def window_op(s, a, b, kind="max", smooth=False, beta=10.0, pad="neutral", pad_value=0.0):
    """Eventually (kind='max') or Always (kind='min') robustness trace.

    pad: 'neutral' drops out-of-range rows (empty window -> -/+BIG),
    'last' pads with s[L-1], 'const' pads with pad_value.
    """
    s = np.asarray(s, dtype=np.float64)
    L = len(s)
    P = b if b is not None else 0
    fill = {"last": s[-1], "const": pad_value, "neutral": 0.0}[pad]
    S = unroll(s, P, fill)
    keep = masks(L, P, a, b)
    if pad == "neutral" or b is None:
        keep[L:, :] = False                                # padded rows do not take part
    sg = 1.0 if kind == "max" else -1.0
    V = sg * S
    if not smooth:
        R = np.where(keep, V, -BIG).max(axis=0)            # Step 3, M (.)- S then column max
    else:
        Z = np.where(keep, beta * V, -np.inf)
        m = Z.max(axis=0)
        m = np.where(np.isfinite(m), m, 0.0)
        with np.errstate(divide="ignore"):
            R = (m + np.log(np.exp(Z - m).sum(axis=0))) / beta
        R = np.where(keep.any(axis=0), R, -BIG)
    return sg * R


def _smooth_mask(k, a, b, c, eps):
    """Sec. VI smooth mask at offsets k (before the clamp at 0)."""
    sig = lambda z: 1.0 / (1.0 + np.exp(-z))
    return sig(c * (k - a)) - (0.0 if b is None else sig(c * (k - b))) - eps


def _mask_support_end(a, b, c, eps):
    """Largest offset with a positive weight (bounded masks)."""
    k, last = 0, -1
    while True:
        if _smooth_mask(float(k), a, b, c, eps) > 0:
            last = k
        elif k > b:
            return last
        k += 1


def smooth_mask_op(s, a, b, c, eps, kind="max", smooth=True, beta=10.0, pad="neutral", pad_value=0.0):
    """Eventually / Always with the smooth time mask of Sec. VI as weights.

    With pad 'last' / 'const' (bounded masks) the unrolled signal of Step 1
    gets as many pad rows as the mask support reaches, and every padded entry
    keeps the weight of its offset.
    """
    s = np.asarray(s, dtype=np.float64)
    L = len(s)
    padded = pad != "neutral" and b is not None
    P = max(0, _mask_support_end(a, b, c, eps)) if padded else 0
    fill = {"last": s[-1], "const": pad_value, "neutral": 0.0}[pad]
    j = np.arange(L + P)[:, None]
    t = np.arange(L)[None, :]
    k = (j - t).astype(np.float64)
    w = _smooth_mask(k, a, b, c, eps)
    w = np.where((j >= t) & (w > 0), w, 0.0)               # subsignal mask and clamp
    sg = 1.0 if kind == "max" else -1.0
    V = sg * unroll(s, P, fill)
    keep = w > 0
    if not smooth:
        R = np.where(keep, V, -BIG).max(axis=0)
    else:
        with np.errstate(divide="ignore"):
            Z = np.where(keep, beta * V + np.log(np.where(keep, w, 1.0)), -np.inf)
        m = np.where(keep, beta * V, -np.inf).max(axis=0)
        m = np.where(np.isfinite(m), m, 0.0)
        with np.errstate(divide="ignore"):
            R = (m + np.log(np.exp(Z - m).sum(axis=0))) / beta
        R = np.where(keep.any(axis=0), R, -BIG)
    return sg * R


def until_op(phi, psi, a, b, smooth=False, beta=10.0):
    """phi U_[a,b] psi by the 3-D unroll of Sec. IV-C (NEUTRAL end handling)."""
    phi = np.asarray(phi, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    L = len(phi)
    bb = (L - 1) if b is None else b
    P = bb
    Sphi = unroll(phi, P, BIG)                              # padded rows never win a min
    Spsi = unroll(psi, P, -BIG)                             # out-of-range psi excludes i
    I = list(range(a, bb + 1))
    K = len(I)
    if K == 0:
        return np.full(L, -BIG)
    S1 = np.empty((2, L, K))
    for n, i in enumerate(I):
        kphi = masks(L, P, 0, i)                            # Always_[0,i] phi
        kpsi = masks(L, P, i, i)                            # Always_[i,i] psi
        if not smooth:
            S1[0, :, n] = np.where(kphi, Sphi, BIG).min(axis=0)
            S1[1, :, n] = np.where(kpsi, Spsi, BIG).min(axis=0)
        else:
            S1[0, :, n] = _smin_cols(Sphi, kphi, beta)
            S1[1, :, n] = _smin_cols(Spsi, kpsi, beta)
    # an index i with t + i past the end takes no part
    valid = np.array([[t + i <= L - 1 for i in I] for t in range(L)])
    if not smooth:
        S2 = S1.min(axis=0)
        S2 = np.where(valid, S2, -BIG)
        return S2.max(axis=1)
    S2 = -_lse(-beta * S1, axis=0) / beta
    Z = np.where(valid, beta * S2, -np.inf)
    out = _lse(Z, axis=1) / beta
    return np.where(valid.any(axis=1), out, -BIG)


def smooth_mask_until_op(phi, psi, a, b, c, eps, smooth=True, beta=10.0):
    """phi U psi with the smooth time mask of Sec. VI on the Until index i:
    the 3-D unroll of Sec. IV-C over every i, the S3 reduction weighted by
    w_i (kept where w_i > 0)."""
    phi = np.asarray(phi, dtype=np.float64)
    psi = np.asarray(psi, dtype=np.float64)
    L = len(phi)
    P = L - 1
    Sphi = unroll(phi, P, BIG)
    Spsi = unroll(psi, P, -BIG)
    I = np.arange(L)
    S1 = np.empty((2, L, L))
    for i in I:
        kphi = masks(L, P, 0, i)
        kpsi = masks(L, P, i, i)
        if not smooth:
            S1[0, :, i] = np.where(kphi, Sphi, BIG).min(axis=0)
            S1[1, :, i] = np.where(kpsi, Spsi, BIG).min(axis=0)
        else:
            S1[0, :, i] = _smin_cols(Sphi, kphi, beta)
            S1[1, :, i] = _smin_cols(Spsi, kpsi, beta)
    w = _smooth_mask(I.astype(np.float64), a, b, c, eps)
    valid = np.array([[t + i <= L - 1 and w[i] > 0 for i in I] for t in range(L)])
    if not smooth:
        S2 = np.where(valid, S1.min(axis=0), -BIG)
        return S2.max(axis=1)
    S2 = -_lse(-beta * S1, axis=0) / beta
    with np.errstate(divide="ignore", invalid="ignore"):
        Z = np.where(valid, beta * S2 + np.log(np.where(w > 0, w, 1.0))[None, :], -np.inf)
    out = _lse(Z, axis=1) / beta
    return np.where(valid.any(axis=1), out, -BIG)


def _lse(Z, axis):
    m = np.max(Z, axis=axis, keepdims=True)
    m = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        return np.squeeze(m, axis=axis) + np.log(np.exp(Z - m).sum(axis=axis))


def _smin_cols(S, keep, beta):
    Z = np.where(keep, -beta * S, -np.inf)
    return -_lse(Z, axis=0) / beta
