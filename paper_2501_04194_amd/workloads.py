"""Seeded synthetic workloads: random-walk trajectories, upstream gradients and
formula descriptions as plain data.

This module holds no robustness arithmetic.  It is the only code shared by the
GPU path and the FP64 oracle: both receive the arrays and the formula
description produced here and evaluate them independently.

Formula description (plain, JSON-able dictionaries).  A number field may be a
literal or the name of an entry in the ``params`` dictionary that travels with
the formula; named entries are the learnable (or annealable) scalars.

  {"op": "true"}
  {"op": "linear", "w": [..D..], "c": c}                 -> w.x_t - c
  {"op": "norm", "A": [[..D..], ...], "p": [...], "r": r, "sign": s}
                                                         -> s*(||A x_t - p|| - r)
  {"op": "not", "child": f}
  {"op": "and" | "or", "children": [f, ...], "smooth": bool, "beta": num}
  {"op": "eventually" | "always", "child": f, "a": int, "b": int | None,
   "smooth": bool, "beta": num, "pad": "neutral" | "last" | "const",
   "pad_value": float}
  {"op": "eventually" | "always", "child": f, "mask": {"a": num, "b": num | None,
   "c": num, "eps": num}, "smooth": bool, "beta": num, "pad": ..., "pad_value": float}
  {"op": "until", "left": f, "right": f, "a": int, "b": int | None,
   "smooth": bool, "beta": num}
  {"op": "until", "left": f, "right": f, "mask": {...}, "smooth": bool, "beta": num}

A smooth mask replaces the integer interval; on Until it weights the Until
index (the right operand's offset).

``"smooth": "softmax"`` selects the softmax-weighted smooth max/min of
Sec. III-C (sum v exp(beta v) / sum exp(beta v)) on and/or and on unmasked
windows; ``True`` the logsumexp form.

``b: None`` means an unbounded interval.  Intervals are inclusive timestep
offsets.  The workloads mirror the shapes and value laws of the benchmark
configurations (random walks started uniformly in [-1, 1]^D with Gaussian
steps); inputs are drawn in float64 with numpy's PCG64 and cast to float32.
"""
from __future__ import annotations

import numpy as np

BETA = 10.0  # logsumexp temperature 0.1 expressed as the inverse temperature


def random_walks(seed: int, B: int, T: int, D: int, step_sigma: float) -> np.ndarray:
    """[B, T, D] float32 random walks: x_0 ~ U[-1,1]^D, x_{t+1} = x_t + N(0, s^2 I)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = rng.uniform(-1.0, 1.0, size=(B, 1, D))
    steps = rng.normal(0.0, step_sigma, size=(B, T - 1, D))
    x = np.concatenate([x0, steps], axis=1).cumsum(axis=1)
    return x.astype(np.float32)


def ragged_walks(seed: int, n: int, lmin: int, lmax: int, D: int, step_sigma: float):
    """Packed ragged random walks: ([N_total, D] float32, offsets int64[n+1])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lengths = rng.integers(lmin, lmax + 1, size=n)
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=offsets[1:])
    total = int(offsets[-1])
    x = np.empty((total, D), dtype=np.float32)
    chunk = 1 << 22
    # generate in chunks of whole trajectories to bound peak memory
    i = 0
    while i < n:
        j = i
        while j < n and offsets[j + 1] - offsets[i] <= chunk:
            j += 1
        j = max(j, i + 1)
        lo, hi = int(offsets[i]), int(offsets[j])
        steps = rng.normal(0.0, step_sigma, size=(hi - lo, D))
        starts = rng.uniform(-1.0, 1.0, size=(j - i, D))
        for k in range(i, j):
            a, b = int(offsets[k]) - lo, int(offsets[k + 1]) - lo
            steps[a] = starts[k - i]
            x[lo + a:lo + b] = np.cumsum(steps[a:b], axis=0)
        i = j
    return x, offsets


def upstream_grad(seed: int, shape) -> np.ndarray:
    """Upstream gradient G ~ N(0, 1) of the root robustness trace, float32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0.0, 1.0, size=shape).astype(np.float32)


# ---------------------------------------------------------------------------
# the five benchmark workloads
# ---------------------------------------------------------------------------

def lin(w, c=0.0):
    return {"op": "linear", "w": list(map(float, w)), "c": float(c)}


def cfg0_formula():
    """Always[0,99](||x|| >= 0.3) and Eventually[10,30](x in [0.5,1]^2); hard."""
    dist = {"op": "norm", "A": [[1.0, 0.0], [0.0, 1.0]], "p": [0.0, 0.0], "r": 0.3, "sign": 1.0}
    box = {"op": "and", "smooth": False, "children": [
        lin([1, 0], 0.5), lin([-1, 0], -1.0), lin([0, 1], 0.5), lin([0, -1], -1.0)]}
    return {"op": "and", "smooth": False, "children": [
        {"op": "always", "a": 0, "b": 99, "smooth": False, "child": dist},
        {"op": "eventually", "a": 10, "b": 30, "smooth": False, "child": box}]}


def cfg1_formula(D: int = 4, beta=BETA):
    """Always[0,inf)(Eventually[0,50](x0 > 0.2)) and (x1 < 0.5 Until[20,200] x2 + x3 > 0.1).

    With D = 3 (ragged workload) the index 3 wraps to 0.
    """
    w2 = [0.0] * D
    w2[2] += 1.0
    w2[3 % D] += 1.0
    e0 = [0.0] * D
    e0[0] = 1.0
    e1 = [0.0] * D
    e1[1] = -1.0
    inner = {"op": "eventually", "a": 0, "b": 50, "smooth": True, "beta": beta,
             "child": lin(e0, 0.2)}
    outer = {"op": "always", "a": 0, "b": None, "smooth": True, "beta": beta, "child": inner}
    until = {"op": "until", "a": 20, "b": 200, "smooth": True, "beta": beta,
             "left": lin(e1, -0.5), "right": lin(w2, 0.1)}
    return {"op": "and", "smooth": True, "beta": beta, "children": [outer, until]}


def cfg2_formula(beta=BETA):
    """Smooth-mask Eventually(x0 > 0) and smooth-mask Always(x1 < 0.5), learnable bounds."""
    ev = {"op": "eventually", "smooth": True, "beta": beta,
          "mask": {"a": "ev_a", "b": "ev_b", "c": "ev_c", "eps": "ev_eps"},
          "child": lin([1, 0], 0.0)}
    al = {"op": "always", "smooth": True, "beta": beta,
          "mask": {"a": "al_a", "b": "al_b", "c": "al_c", "eps": "al_eps"},
          "child": lin([0, -1], -0.5)}
    return {"op": "and", "smooth": True, "beta": beta, "children": [ev, al]}


def cfg2_params():
    return {"ev_a": 100.0, "ev_b": 400.0, "ev_c": 1.0, "ev_eps": 1e-6,
            "al_a": 100.0, "al_b": 400.0, "al_c": 1.0, "al_eps": 1e-6}


WORKLOADS = {
    0: dict(name="hard_B16_T100_D2", B=16, T=100, D=2, sigma=0.1, seed=0),
    1: dict(name="smooth_until_B1024_T1000_D4", B=1024, T=1000, D=4, sigma=0.05, seed=1),
    2: dict(name="smooth_mask_B4096_T2048_D2", B=4096, T=2048, D=2, sigma=0.05, seed=2),
    3: dict(name="ragged_N10000_L64-8192_D3", N=10000, lmin=64, lmax=8192, D=3,
            sigma=0.05, seed=3),
}


def workload(k: int, B: int | None = None, T: int | None = None):
    """(formula, params, x) for benchmark workload k (0, 1 or 2); B/T may shrink it."""
    c = WORKLOADS[k]
    B = c["B"] if B is None else B
    T = c["T"] if T is None else T
    x = random_walks(c["seed"], B, T, c["D"], c["sigma"])
    if k == 0:
        return cfg0_formula(), {}, x
    if k == 1:
        return cfg1_formula(c["D"]), {}, x
    if k == 2:
        return cfg2_formula(), cfg2_params(), x
    raise ValueError(k)


def ragged_workload(n: int | None = None, seed: int | None = None):
    """(formula, params, x_packed, offsets) for the ragged workload."""
    c = WORKLOADS[3]
    x, off = ragged_walks(c["seed"] if seed is None else seed, c["N"] if n is None else n,
                          c["lmin"], c["lmax"], c["D"], c["sigma"])
    return cfg1_formula(c["D"]), {}, x, off


# ---------------------------------------------------------------------------
# the formula suite of Table II (computational-properties study)
# ---------------------------------------------------------------------------

TABLE2_INTERVAL = (2, 20)      # the table leaves I open: a fixed bounded window


def _region(k: int):
    """phi_k and psi_k of region k on a 2-D state: x0 > c_k and x1 < d_k (linear
    predicates at distinct, fixed thresholds)."""
    return lin([1, 0], -0.9 + 0.17 * k), lin([0, -1], -(0.9 - 0.13 * k))


def _conj(children, smooth, beta):
    """n-ary And as a tree of at most four children per node (the plan's limit;
    min and logsumexp are associative, so the value is that of the flat And)."""
    while len(children) > 4:
        children = [{"op": "and", "smooth": smooth, "beta": beta, "children": children[i:i + 4]}
                    if len(children[i:i + 4]) > 1 else children[i]
                    for i in range(0, len(children), 4)]
    return {"op": "and", "smooth": smooth, "beta": beta, "children": children}


def table2_formulas(smooth: bool = True, beta: float = BETA, interval=TABLE2_INTERVAL) -> dict:
    """phi_1 .. phi_6 of Table II with synthetic linear predicates on D = 2
    (invariance, stabilization, strict ordering, sequenced visits, sequenced
    visit + stabilization, ten regions in any order)."""
    a, b = interval
    s = {"smooth": smooth, "beta": beta}

    def both(k):
        p, q = _region(k)
        return dict({"op": "and", "children": [p, q]}, **s)

    def ev(child, lo=a, hi=b):
        return dict({"op": "eventually", "a": lo, "b": hi, "child": child}, **s)

    def al(child, lo=a, hi=b):
        return dict({"op": "always", "a": lo, "b": hi, "child": child}, **s)

    p0, q0 = _region(0)
    phi4 = ev(both(0))
    for k in (1, 2, 3):
        phi4 = ev(dict({"op": "and", "children": [_region(k)[0], _region(k)[1], phi4]}, **s))
    return {
        "phi1": al(both(0), 0, None),
        "phi2": ev(al(both(0), 0, None), 0, None),
        "phi3": dict({"op": "until", "a": 0, "b": None, "left": p0, "right": q0}, **s),
        "phi4": phi4,
        "phi5": ev(dict({"op": "and", "children": [_region(2)[0], _region(2)[1], ev(al(both(0)))]}, **s)),
        "phi6": _conj([ev(both(k)) for k in range(10)], smooth, beta),
    }
