"""Throughput of STL robustness forward + backward on one MI355X.

Workload: B=4096 random-walk trajectories of T=2048 two-dimensional states,
formula Eventually~[a,b](x0 > 0) and~ Always~[a,b](x1 < 0.5) with smooth
sigmoid time masks (a=100, b=400, c=1, eps=1e-6, beta=10), gradients with
respect to x and the four mask bounds.  One step = stl_forward_saving +
stl_backward_saved over the whole batch (the backward reuses the two
mask-node traces the forward kept, as an autograd function does; pass
--recompute for stl_forward + stl_backward); inputs are resident in HBM and
rotate over several buffer sets so the 256 MB Infinity Cache cannot serve
them.

Prints one JSON line (metric, value, roofline of the dominant kernel, CPU
oracle baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_FWD = 12       # per signal-step: x (2 x 4 B) + root (4 B)
BYTES_BWD = 20       # per signal-step: x (8 B) + G (4 B) + dx (8 B)
METRIC = "fwd+bwd signal-steps/s (B=4096,T=2048 smooth STL); % of HBM roofline"


def cpu_baseline(n_traj=128):
    """The FP64 oracle (unchanged) on a bounded sample of the same workload."""
    import oracle
    from paper_2501_04194_amd import workloads as W
    oracle.build()
    spec, params, x = W.workload(2, B=n_traj)
    G = W.upstream_grad(102, x.shape[:2])
    p32 = {k: float(np.float32(v)) for k, v in params.items()}
    t0 = time.perf_counter()
    oracle.forward(spec, x, params=p32)
    oracle.backward(spec, x, G, params=p32)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n_traj * x.shape[1] / dt, "unit": "signal-steps/s", "cores": cores, "kind": "oracle",
            "sample": "%d of the 4096 trajectories (T=2048), forward + backward, FP64 C oracle with OpenMP, %.2f s"
                      % (n_traj, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--rotate", type=int, default=4, help="input buffer sets cycled through")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-traj", type=int, default=128)
    ap.add_argument("--recompute", action="store_true", help="backward recomputes the node traces")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (trajectories shard with no "
              "communication; see the design notes).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2501_04194_amd import stl, workloads as W

    dev = torch.device("cuda:0")
    spec, params, x = W.workload(2)
    B, T, D = x.shape
    steps_per_batch = B * T
    plan = stl.Plan(spec, D, params)
    pv = torch.from_numpy(plan.param_vector()).to(dev)
    x0 = torch.from_numpy(x).to(dev)
    G0 = torch.from_numpy(W.upstream_grad(102, (B, T))).to(dev)
    R = max(1, args.rotate)
    xs = [x0.clone() for _ in range(R)]
    Gs = [G0.clone() for _ in range(R)]
    sv = [None if args.recompute else plan.saved_buffer(xs[i]) for i in range(R)]
    del x0, G0

    def step(k):
        i = k % R
        plan.forward(xs[i], pv, saved=sv[i])
        plan.backward(xs[i], Gs[i], pv, saved=sv[i])

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e0.record(stream)
    for k in range(args.steps):
        step(k)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms = e0.elapsed_time(e1) / args.steps
    value = steps_per_batch / (ms * 1e-3)

    # per-kernel durations with events on the launch stream: forward kernel
    # alone, backward kernel alone (without the tiny parameter-reduction kernel)
    def timed(fn, n):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for k in range(n):
            evs[k][0].record(stream)
            fn(k)
            evs[k][1].record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in evs]))

    n_k = max(5, min(args.steps, 30))
    fwd_ms = timed(lambda k: plan.forward(xs[k % R], pv, saved=sv[k % R]), n_k)
    bwd_ms = timed(lambda k: plan.backward(xs[k % R], Gs[k % R], pv, want_params=False, saved=sv[k % R]), n_k)
    dom_is_bwd = bwd_ms >= fwd_ms
    dom_ms = bwd_ms if dom_is_bwd else fwd_ms
    dom_bytes = (BYTES_BWD if dom_is_bwd else BYTES_FWD) * steps_per_batch
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic_bwd_smooth_mask_B4096_T2048.json")
    if dom_is_bwd and os.path.exists(tf):
        try:
            traffic = json.load(open(tf)).get("bytes_per_launch")
        except Exception:
            traffic = None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "signal-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "smooth_mask_B4096_T2048_D2", "B": B, "T": T, "D": D,
                   "formula": "Eventually~[a,b](x0>0) and~ Always~[a,b](x1<0.5)",
                   "mask": {"a": 100.0, "b": 400.0, "c": 1.0, "eps": 1e-6}, "beta": 10.0,
                   "grads": "x and the four mask bounds", "buffer_sets": R,
                   "saved_traces": not args.recompute},
        "hbm_frac_step": (BYTES_FWD + BYTES_BWD) * value / (HBM_PEAK_GBS * 1e9),
        "kernel_ms": {"forward": fwd_ms, "backward": bwd_ms},
        "wall_s": t_wall,
        "roofline": {"bound": "hbm", "kernel": "stl_fused_bwd" if dom_is_bwd else "stl_fused_fwd",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_traj)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
