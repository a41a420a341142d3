"""Learned warm start for STL trajectory optimisation on the GPU.

Problem family (seeded, synthetic): a 2-D workspace [-1, 1]^2 with three
circular obstacles (centres U[-0.6, 0.6]^2, radii U[0.1, 0.3], drawn once per
experiment), a start and a goal drawn uniformly outside the obstacles, and
200 waypoints x_0 .. x_199 with x_0 the start.  Specification (reach-avoid):

    Always_[0,inf) ( and_k ||x - o_k|| >= r_k )  and  Eventually_[50,150] ||x - g|| <= 0.1

Plain method: start from the straight line start -> goal and raise the smooth
robustness (beta = 10) at t = 0 by fixed-step gradient ascent on x_1..x_199
(gradients from stl_backward, the update by stl_ascent_update); every
`check` steps the hard robustness is evaluated on the GPU and a problem is
solved when it is > 0.  Learned method: an MLP 4 -> 256 -> 256 -> 400 (BF16
weights and activations, FP32 accumulation, trained with the library's own
kernels) maps (start, goal) to a residual added to the straight line; the
same ascent then starts from that proposal.  Robustness as a differentiable
planning objective follows arXiv 2501.04194 Sec. VII-A; the warm start
itself is not in the paper.
"""
from __future__ import annotations

import time

import numpy as np

from . import mlp as M
from . import stl

T = 200
D = 4                 # state seen by the formula: position (2) + goal (2)
BETA = 10.0


def obstacles(seed=0, n=3):
    rng = np.random.default_rng(np.random.PCG64(10_000 + seed))
    c = rng.uniform(-0.6, 0.6, size=(n, 2))
    r = rng.uniform(0.1, 0.3, size=n)
    return c, r


def problems(n, obst, seed, margin=0.05):
    """n (start, goal) pairs outside the obstacles (+ margin), float32 [n, 4]."""
    c, r = obst
    rng = np.random.default_rng(np.random.PCG64(seed))
    out = np.empty((0, 4))
    while len(out) < n:
        cand = rng.uniform(-1.0, 1.0, size=(2 * n, 4))
        ok = np.ones(len(cand), bool)
        for k in range(len(r)):
            for o in (0, 2):
                ok &= np.linalg.norm(cand[:, o:o + 2] - c[k], axis=1) > r[k] + margin
        ok &= np.linalg.norm(cand[:, 0:2] - cand[:, 2:4], axis=1) > 0.3
        out = np.concatenate([out, cand[ok]])
    return out[:n].astype(np.float32)


def spec(obst, smooth=True, beta=BETA):
    c, r = obst
    pos = [[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.0]]
    avoid = [{"op": "norm", "A": pos, "p": list(map(float, c[k])), "r": float(r[k]), "sign": 1.0}
             for k in range(len(r))]
    goal = {"op": "norm", "A": [[1.0, 0.0, -1.0, 0.0], [0.0, 1.0, 0.0, -1.0]], "p": [0.0, 0.0], "r": 0.1,
            "sign": -1.0}
    s = dict(smooth=smooth, beta=beta)
    return {"op": "and", "children": [
        dict({"op": "always", "a": 0, "b": None, "child": dict({"op": "and", "children": avoid}, **s)}, **s),
        dict({"op": "eventually", "a": 50, "b": 150, "child": goal}, **s)], **s}


def straight_line(prob):
    """[n, T, D] trajectories: the straight segment start -> goal plus the goal columns."""
    s, g = prob[:, None, 0:2], prob[:, None, 2:4]
    a = (np.arange(T, dtype=np.float32) / (T - 1))[None, :, None]
    pos = s + a * (g - s)
    return np.concatenate([pos, np.broadcast_to(g, pos.shape)], axis=2).astype(np.float32)


class Solver:
    """Batched plain gradient ascent on the smooth robustness at t = 0."""

    def __init__(self, obst, n, device, lr=0.05, check=10):
        import torch
        self.torch = torch
        self.dev = device
        self.n = n
        self.lr = lr
        self.check = check
        self.smooth = stl.Plan(spec(obst, True), D)
        self.hard = stl.Plan(spec(obst, False), D)
        self.pv_s = torch.from_numpy(self.smooth.param_vector()).to(device)
        self.pv_h = torch.from_numpy(self.hard.param_vector()).to(device)
        self.x = torch.zeros((n, T, D), dtype=torch.float32, device=device)
        G = torch.zeros((n, T), dtype=torch.float32, device=device)
        G[:, 0] = 1.0                       # d rho(x, t=0) / d x
        self.G = G
        self.graph = stl.Graph(self.smooth, self.x, self.pv_s, self.G)
        self.active = torch.ones(n, dtype=torch.int32, device=device)

    def hard_rho(self):
        return self.hard.forward(self.x, self.pv_h)[:, 0]

    def solve(self, x0, max_steps=2000, t_start=None):
        """Ascent from x0 [n, T, D].

        Returns (steps-to-success per problem (-1: not solved), timeline), the
        timeline listing (seconds since t_start, problems solved) at every
        check; t_start defaults to the call's start."""
        torch = self.torch
        t_start = time.perf_counter() if t_start is None else t_start
        self.x.copy_(x0)
        self.active.fill_(1)
        steps = torch.full((self.n,), -1, dtype=torch.int64, device=self.dev)
        ok = self.hard_rho() > 0
        steps[ok] = 0
        self.active[ok] = 0
        k = 0
        left = int(self.active.sum())
        timeline = [(time.perf_counter() - t_start, self.n - left)]
        while k < max_steps and left > 0:
            for _ in range(self.check):
                self.graph.launch()                       # smooth forward + backward (HIP graph)
                M.ascent_update(self.x, self.graph.dx, self.active, self.lr, t0=1, d_upd=2)
            k += self.check
            ok = (self.hard_rho() > 0) & (self.active > 0)
            steps[ok] = k
            self.active[ok] = 0
            left = int(self.active.sum())                 # synchronises
            timeline.append((time.perf_counter() - t_start, self.n - left))
        torch.cuda.synchronize()
        return steps.cpu().numpy(), timeline


def time_to(timeline, count):
    """First time at which at least `count` problems were solved (inf if never)."""
    for t, c in timeline:
        if c >= count:
            return t
    return float("inf")


def train_mlp(inputs, targets, device, epochs=30, batch=1024, lr=1e-3, seed=0, log=None):
    """Fit the BF16 MLP to (start, goal) -> residual waypoints with MSE + Adam."""
    import torch
    net = M.BF16MLP([4, 256, 256, 2 * T], device, seed=seed)
    X = torch.from_numpy(inputs).to(device)
    Y = torch.from_numpy(targets.reshape(len(targets), -1)).to(device)
    n = len(X)
    rng = np.random.default_rng(seed)
    loss = torch.zeros(1, dtype=torch.float32, device=device)
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(device)
        tot = 0.0
        for i in range(0, n - batch + 1, batch):
            idx = perm[i:i + batch]
            out = net.forward(X[idx], keep=True)
            g = torch.empty_like(out)
            M.mse_grad(out, Y[idx].contiguous(), g, loss)
            dW, db = net.backward(g)
            net.adam(dW, db, lr=lr)
            tot += float(loss)
        hist.append(tot / max(1, n // batch))
        if log:
            log("epoch %d loss %.5f" % (ep, hist[-1]))
    return net, hist


def propose(net, prob, device):
    """Straight line + network residual (x_0 stays at the start)."""
    import torch
    x = torch.from_numpy(straight_line(prob)).to(device)
    res = net.forward(torch.from_numpy(prob).to(device)).view(len(prob), T, 2)
    x[:, 1:, 0:2] += res[:, 1:, :]
    return x


def experiment(n_train=50_000, n_test=1000, seed=0, max_steps=2000, epochs=30, lr_ascent=0.05, check=10, log=print):
    """Data generation by plain ascent, MLP training, learned-vs-plain evaluation."""
    import torch
    dev = torch.device("cuda:0")
    obst = obstacles(seed)
    res = {"n_train_problems": n_train, "n_test": n_test, "T": T, "max_steps": max_steps, "check_every": check,
           "ascent_lr": lr_ascent}
    # 1. training data: solve n_train problems with the plain method
    tr = problems(n_train, obst, seed=20_000 + seed)
    solver = Solver(obst, n_train, dev, lr=lr_ascent, check=check)
    t0 = time.perf_counter()
    st, _ = solver.solve(torch.from_numpy(straight_line(tr)).to(dev), max_steps)
    res["datagen_s"] = time.perf_counter() - t0
    ok = st >= 0
    res["train_solved_frac"] = float(ok.mean())
    xs = solver.x[torch.from_numpy(ok).to(dev)][:, :, 0:2].cpu().numpy()
    targets = xs - straight_line(tr[ok])[:, :, 0:2]
    log("training data: %d/%d solved in %.1fs" % (ok.sum(), n_train, res["datagen_s"]))
    del solver
    # 2. train
    t0 = time.perf_counter()
    net, hist = train_mlp(tr[ok], targets.astype(np.float32), dev, epochs=epochs, seed=seed, log=log)
    torch.cuda.synchronize()
    res["train_s"] = time.perf_counter() - t0
    res["loss_first_last"] = [hist[0], hist[-1]]
    # 3. evaluate on held-out problems
    te = problems(n_test, obst, seed=30_000 + seed)
    ev = Solver(obst, n_test, dev, lr=lr_ascent, check=check)
    x_plain = torch.from_numpy(straight_line(te)).to(dev)
    ev.solve(x_plain, check)                           # warm-up (graph, allocator)
    propose(net, te[:8], dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s_plain, tl_plain = ev.solve(x_plain, max_steps, t_start=t0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x_learn = propose(net, te, dev)                    # MLP inference inside the timed region
    s_learn, tl_learn = ev.solve(x_learn, max_steps, t_start=t0)
    target = int((s_plain >= 0).sum())                 # what plain ascent reaches within max_steps

    def summary(s, tl):
        solved = s >= 0
        return {"solved_frac": float(solved.mean()),
                "median_steps": float(np.median(np.where(solved, s, max_steps))),
                "mean_steps": float(np.mean(np.where(solved, s, max_steps))),
                "wall_s": tl[-1][0],
                "s_to_plain_solved": time_to(tl, target)}

    res["plain"] = summary(s_plain, tl_plain)
    res["learned"] = summary(s_learn, tl_learn)
    log("plain %s\nlearned %s" % (res["plain"], res["learned"]))
    return res
