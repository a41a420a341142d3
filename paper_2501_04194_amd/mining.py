"""Parametric-STL mining with differentiable time intervals (Sec. VII-B, the
pSTL problem): find the largest [a, b] (fractions of the horizon) such that the
signals of a dataset satisfy Always_[aT, bT](s > 0), by gradient descent on

    L(a, b) = mean_s max(-rho(s, Always_[aT, bT](s > 0)), 0) + gamma (a - b)

through the smooth time mask, with a and b passed through a sigmoid and the
mask steepness and the logsumexp temperature annealed along a sigmoid
schedule.  Every robustness value and its d/da, d/db come from
``stl_interval_sweep`` on the GPU; the optimiser step is plain tensor
arithmetic.  A coarse sweep over a grid of intervals (one launch) can pick the
starting point, as the paper suggests (global search by sampling, then local
refinement by gradient descent).
"""
from __future__ import annotations

import time

import numpy as np

from . import stl


def make_dataset(n: int = 500, T: int = 20, a: float = 0.23, b: float = 0.59, jitter: float = 0.02,
                 noise: float = 0.05, seed: int = 0) -> np.ndarray:
    """[n, T, 1] float32 signals equal to 1 on [a_i T, b_i T] and 0 elsewhere,
    a_i = a + N(0, jitter^2), b_i = b + N(0, jitter^2), plus N(0, noise^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ai = a + rng.normal(0.0, jitter, size=(n, 1))
    bi = b + rng.normal(0.0, jitter, size=(n, 1))
    t = np.arange(T)[None, :]
    s = ((t >= ai * T) & (t <= bi * T)).astype(np.float64) + rng.normal(0.0, noise, size=(n, T))
    return s[:, :, None].astype(np.float32)


def schedule(k: int, steps: int, lo: float, hi: float) -> float:
    """Sigmoid annealing from lo to hi over the steps (the schedule of stl_pstl_descent)."""
    return lo + (hi - lo) / (1.0 + np.exp(-12.0 * (k / max(1, steps - 1) - 0.5)))


def coarse_start(x, n_grid: int = 40, gamma: float = 0.1, c: float = 20.0, beta: float = 20.0):
    """Loss of every (a, b) on an n_grid x n_grid grid of fractions (one
    interval-sweep launch over all signals); returns the best (a, b)."""
    import torch
    T = x.shape[1]
    g = torch.linspace(0.02, 0.98, n_grid, device=x.device)
    A, Bm = torch.meshgrid(g, g, indexing="ij")
    keep = (A < Bm).reshape(-1)
    a, b = A.reshape(-1)[keep].contiguous(), Bm.reshape(-1)[keep].contiguous()
    rho = stl.interval_sweep(x, a * T, b * T, [1.0], op="always", beta=beta, mask_c=c, grads=False)
    loss = torch.relu(-rho).mean(dim=0) + gamma * (a - b)
    i = int(torch.argmin(loss))
    return float(a[i]), float(b[i])


def mine(x, steps: int = 5000, lr: float = 1e-2, gamma: float = 0.1, c_range=(1.0, 20.0), beta_range=(1.0, 20.0),
         init=(0.1, 0.9), eps: float = 1e-6, want_loss: bool = False):
    """Gradient descent on the pSTL loss, the whole loop in one launch
    (``stl_pstl_descent``); returns (a, b, per-step seconds[, loss per step])."""
    import torch
    logit = lambda v: float(np.log(v / (1.0 - v)))
    p = torch.tensor([logit(init[0]), logit(init[1])], dtype=torch.float32, device=x.device)
    torch.cuda.synchronize(x.device)
    t0 = time.perf_counter()
    loss = stl.pstl_descent(x, p, steps, lr=lr, gamma=gamma, c_range=c_range, beta_range=beta_range,
                            mask_eps=eps, want_loss=want_loss)
    torch.cuda.synchronize(x.device)
    dt = (time.perf_counter() - t0) / max(1, steps)
    ab = torch.sigmoid(p).cpu().numpy()
    if want_loss:
        return float(ab[0]), float(ab[1]), dt, loss.cpu().numpy()
    return float(ab[0]), float(ab[1]), dt


def mine_stepwise(x, steps: int = 5000, lr: float = 1e-2, gamma: float = 0.1, c_range=(1.0, 20.0),
                  beta_range=(1.0, 20.0), init=(0.1, 0.9), eps: float = 1e-6):
    """The same descent with one interval-sweep launch per step and the update
    in tensor arithmetic (a cross-check of ``mine``); returns (a, b, per-step seconds)."""
    import torch
    dev = x.device
    T = x.shape[1]
    logit = lambda v: float(np.log(v / (1.0 - v)))
    p = torch.tensor([logit(init[0]), logit(init[1])], dtype=torch.float32, device=dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for k in range(steps):
        c = schedule(k, steps, *c_range)
        beta = schedule(k, steps, *beta_range)
        ab = torch.sigmoid(p)
        a_steps, b_steps = (ab[0:1] * T).contiguous(), (ab[1:2] * T).contiguous()
        rho, ga, gb = stl.interval_sweep(x, a_steps, b_steps, [1.0], op="always", beta=beta, mask_c=c,
                                         mask_eps=eps)
        active = (rho < 0).float()
        # d L / d a_frac = T * mean(-[rho < 0] d rho / d a_steps) + gamma; same for b with -gamma
        dl = torch.cat([T * (-(active * ga)).mean(0) + gamma, T * (-(active * gb)).mean(0) - gamma])
        p = p - lr * dl * ab * (1.0 - ab)
    torch.cuda.synchronize(dev)
    dt = (time.perf_counter() - t0) / max(1, steps)
    ab = torch.sigmoid(p).cpu().numpy()
    return float(ab[0]), float(ab[1]), dt
