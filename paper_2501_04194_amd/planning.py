"""Trajectory planning with a learnable time interval (Sec. VII-A): controls u
(single integrator, x_{t+1} = x_t + dt u_t) and the normalized interval (a, b)
of phi = Always_[aT, bT](inside Y) and Eventually(inside G) are optimised
together on

    gamma_1 ReLU(-rho(x, phi)) + gamma_2 exp(2 (I - b + a))
      + gamma_3 mean_t ReLU(||u_t|| - u_max) + gamma_4 mean_t ||u_t||^2

by gradient descent.  rho at t = 0 and its gradients with respect to the
trajectory and to the mask bounds come from the library (``stl.robustness``:
stl_forward_saving / stl_backward_saved on the generic executor); the dynamics
and the other cost terms are tensor arithmetic.  Several coefficient settings
(or random initialisations) run as one batch: each trajectory carries its own
controls, and the masks of the batch share (a, b) only when asked to, so by
default one plan per setting is used.

The paper gives the horizon, step, limits, coefficients and the initial
interval but not the region geometry: the regions here are axis-aligned boxes
(stated in ``REGIONS``): a corridor Y on the way from the start to G, so
that a longer visit costs little control effort and the interval can grow.
"""
from __future__ import annotations

import time

import numpy as np

from . import stl

T = 51
DT = 0.1
U_MAX = 2.0
I_NOM = 0.2
GAMMA = (1.1, 0.05, 2.0, 0.5)
START = (0.0, 0.0)
REGIONS = {"yellow": (0.3, 1.5, -0.4, 0.4), "green": (1.9, 2.5, -0.3, 0.3)}   # x_lo, x_hi, y_lo, y_hi


def inside(box, smooth=True, beta=10.0):
    """Smooth And of the four half-planes of an axis-aligned box (state (x, y))."""
    x0, x1, y0, y1 = box
    lin = lambda w, c: {"op": "linear", "w": list(map(float, w)), "c": float(c)}
    return {"op": "and", "smooth": smooth, "beta": beta,
            "children": [lin([1, 0], x0), lin([-1, 0], -x1), lin([0, 1], y0), lin([0, -1], -y1)]}


def formula(beta=10.0, mask_c=2.0):
    """Always over the smooth mask [a, b] (timesteps, learnable) of inside Y,
    and Eventually (unbounded) of inside G, smooth And at the root."""
    return {"op": "and", "smooth": True, "beta": beta, "children": [
        {"op": "always", "smooth": True, "beta": beta, "child": inside(REGIONS["yellow"], beta=beta),
         "mask": {"a": "a", "b": "b", "c": mask_c, "eps": 1e-6}},
        {"op": "eventually", "a": 0, "b": None, "smooth": True, "beta": beta,
         "child": inside(REGIONS["green"], beta=beta)}]}


def rollout(u, x0):
    """Single-integrator states x_0 .. x_{T-1} from controls u_0 .. u_{T-2} ([B, T-1, 2])."""
    import torch
    return torch.cat([x0[:, None, :], x0[:, None, :] + DT * torch.cumsum(u, dim=1)], dim=1)


class _Problem:
    """State of `batch` planning problems and one optimisation step."""

    def __init__(self, batch, seed, init_ab, gamma, lr, device, capturable):
        import torch
        dev = torch.device(device)
        self.dev, self.batch, self.gamma = dev, batch, gamma
        g = torch.Generator(device="cpu").manual_seed(seed)
        self.u = (0.5 * torch.randn(batch, T - 1, 2, generator=g)).to(dev).requires_grad_(True)
        logit = lambda v: float(np.log(v / (1.0 - v)))
        self.W = 0.5 * I_NOM
        q0 = (init_ab[1] - init_ab[0] - self.W) / (1.0 - init_ab[0] - self.W)
        self.pq = torch.tensor([[logit(init_ab[0] / (1.0 - self.W)), logit(q0)]] * batch,
                               device=dev).requires_grad_(True)
        self.x0 = torch.tensor([START] * batch, dtype=torch.float32, device=dev)
        spec = formula()
        self.plans = [stl.Plan(spec, 2, {"a": 0.0, "b": 1.0}) for _ in range(batch)]
        slots = self.plans[0].slots
        self.ia = [i for i, (nm, _) in enumerate(slots) if nm == "a"][0]
        self.ib = [i for i, (nm, _) in enumerate(slots) if nm == "b"][0]
        self.base = torch.from_numpy(self.plans[0].param_vector()).to(dev)
        self.sel = torch.tensor([self.ia, self.ib], device=dev)
        self.saved = [p.saved_buffer(torch.zeros(1, T, 2, device=dev)) for p in self.plans]
        self.G = torch.zeros(1, T, device=dev)       # upstream gradient: d rho(t=0)
        self.G[0, 0] = 1.0
        self.opt = torch.optim.Adam([self.u, self.pq], lr=lr, capturable=capturable)

    def interval(self):
        import torch
        a = (1.0 - self.W) * torch.sigmoid(self.pq[:, 0])
        return a, a + self.W + (1.0 - a - self.W) * torch.sigmoid(self.pq[:, 1])

    def rho_and_grads(self, x, a, b, k):
        """rho(t=0) of problem k and its gradients in x and (a, b) (normalized)."""
        import torch
        T_ = float(T)
        pv = self.base.index_put((self.sel,), torch.stack([a[k], b[k]]).detach() * T_)
        xk = x[k:k + 1].detach().contiguous()
        root = self.plans[k].forward(xk, pv, saved=self.saved[k])
        dx, gp = self.plans[k].backward(xk, self.G, pv, saved=self.saved[k])
        return root[0, 0], dx[0], gp[self.ia] * T_, gp[self.ib] * T_

    def step(self):
        import torch
        g1, g2, g3, g4 = self.gamma
        self.opt.zero_grad(set_to_none=False)
        a, b = self.interval()
        x = rollout(self.u, self.x0)
        nu = torch.linalg.norm(self.u, dim=2)
        J = (g2 * torch.exp(2.0 * (I_NOM - b + a)) + g3 * torch.relu(nu - U_MAX).mean(1)
             + g4 * (nu ** 2).mean(1)).sum()
        # the STL term through the library's hand-written backward:
        # d/d(.) gamma_1 ReLU(-rho) = -gamma_1 [rho < 0] d rho/d(.)
        gx = torch.zeros_like(x)
        ga = torch.zeros(self.batch, device=self.dev)
        gb = torch.zeros(self.batch, device=self.dev)
        for k in range(self.batch):
            r, dx, da, db = self.rho_and_grads(x, a, b, k)
            w = -g1 * (r < 0).float()
            gx[k] = w * dx
            ga[k] = w * da
            gb[k] = w * db
        (J + (x * gx).sum() + (a * ga).sum() + (b * gb).sum()).backward()
        self.opt.step()

    def result(self):
        import torch
        with torch.no_grad():
            a, b = self.interval()
            x = rollout(self.u, self.x0)
            rho = torch.stack([self.rho_and_grads(x, a, b, k)[0] for k in range(self.batch)])
        return self.u.detach(), a.cpu().numpy(), b.cpu().numpy(), rho.cpu().numpy()


def plan(steps=2000, lr=0.05, batch=1, seed=0, init_ab=(0.14, 0.82), gamma=GAMMA, device="cuda", graph=True):
    """Optimise `batch` independent problems (random initial controls, one plan
    each); returns (u, a, b, rho, seconds per step) with a, b the normalized
    interval.  The interval is parametrised as a = (1 - W) sig(p),
    b = a + W + (1 - a - W) sig(q) with W = I/2, so the Always keeps a window
    of at least half the nominal size: an empty or vanishing window would make
    it vacuously true, which the optimiser otherwise finds before it steers the
    trajectory into the region.  With ``graph`` one step (library calls, cost,
    backward and Adam) is captured once in a HIP graph and replayed."""
    import torch
    P = _Problem(batch, seed, init_ab, gamma, lr, device, capturable=graph)
    if graph:
        s = torch.cuda.Stream(P.dev)
        s.wait_stream(torch.cuda.current_stream(P.dev))
        with torch.cuda.stream(s):
            for _ in range(3):                  # warm-up on a side stream before capture
                P.step()
        torch.cuda.current_stream(P.dev).wait_stream(s)
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            P.step()
        torch.cuda.synchronize(P.dev)
        t0 = time.perf_counter()
        for _ in range(steps - 3):              # capturing records the step without running it
            gr.replay()
        torch.cuda.synchronize(P.dev)
        dt = (time.perf_counter() - t0) / max(1, steps - 3)
    else:
        torch.cuda.synchronize(P.dev)
        t0 = time.perf_counter()
        for _ in range(steps):
            P.step()
        torch.cuda.synchronize(P.dev)
        dt = (time.perf_counter() - t0) / max(1, steps)
    u, a, b, rho = P.result()
    return u, a, b, rho, dt
