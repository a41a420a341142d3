"""GPU tests of the composed paths the benchmarks time, and of bitwise
reproducibility of the Until adjoints:
  * the ragged workload through LPT order, the autotuned launch and a HIP
    graph replayed three times, against eager calls and the FP64 oracle;
  * the autotuned launch's forward and backward against the default launch;
  * two runs of formulas with Until (smooth fp64 and scaled-pair forms, hard
    bounded and unbounded, ragged) give identical bits;
  * the interval sweep at its benchmarked size (4096 signals x 90,000
    intervals), sampled against the oracle.
"""
import numpy as np
import pytest

import oracle
from gpu_util import Gpu, assert_close
from paper_2501_04194_amd import stl, workloads as W

pytestmark = pytest.mark.gpu


def _twice(spec, D, params, x, G, offsets=None, T=None, order=None, launch=None):
    g = Gpu(spec, D, params, launch=launch)
    r1 = g.fwd(x, offsets=offsets, T=T, order=order)
    r2 = g.fwd(x, offsets=offsets, T=T, order=order)
    (d1, p1), (d2, p2) = g.bwd(x, G, offsets=offsets, T=T, order=order), g.bwd(x, G, offsets=offsets, T=T, order=order)
    assert np.array_equal(r1, r2)
    assert np.array_equal(d1, d2)
    assert p1 == p2


def _until(a, b, smooth):
    s = {"smooth": True, "beta": 10.0} if smooth else {"smooth": False}
    return dict({"op": "until", "a": a, "b": b, "left": {"op": "linear", "w": [1, 0], "c": -0.5},
                 "right": {"op": "linear", "w": [0, 1], "c": 0.1}}, **s)


def test_until_backward_bitwise_cfg1():
    spec, params, x = W.workload(1, B=64)
    G = W.upstream_grad(101, x.shape[:2])
    print("cfg1 B=64 T=%d" % x.shape[1], flush=True)
    _twice(spec, x.shape[-1], params, x, G)
    _twice(spec, x.shape[-1], params, x[:6, :700], G[:6, :700], launch=stl.Launch(512, 1, 1, 0))


def test_until_backward_bitwise_ragged():
    spec, params, xp, off = W.ragged_workload(n=60)
    G = W.upstream_grad(103, (xp.shape[0],))
    T = int(np.diff(off).max())
    order = stl.lpt_order(off)
    print("ragged n=60 T=%d" % T, flush=True)
    _twice(spec, xp.shape[-1], params, xp, G, offsets=off, T=T, order=order)


@pytest.mark.parametrize("case", ["hard_unbounded", "hard_bounded", "smooth_unbounded", "wide_range"])
def test_until_backward_bitwise_forms(case):
    rng = np.random.default_rng(31)
    x = np.cumsum(rng.normal(size=(8, 700, 2)) * 0.1, axis=1).astype(np.float32)
    spec = {"hard_unbounded": _until(0, None, False), "hard_bounded": _until(3, 40, False),
            "smooth_unbounded": _until(5, None, True), "wide_range": _until(0, 120, True)}[case]
    if case == "wide_range":
        x = x * np.float32(60.0)                  # exponent range beyond the fp64 form: scaled pairs
    G = rng.normal(size=x.shape[:2]).astype(np.float32)
    _twice(spec, 2, {}, x, G)


def test_ragged_measured_path_against_eager_and_oracle():
    """The composition the ragged benchmark times, on 200 of its trajectories
    (lengths 64..8192): LPT order, the stl_autotune launch, and forward +
    backward captured in a graph and replayed three times."""
    import torch
    spec, params, xp, off = W.ragged_workload(n=200)
    T = int(np.diff(off).max())
    G = W.upstream_grad(103, (xp.shape[0],))
    plan = stl.Plan(spec, xp.shape[-1], params)
    pv = torch.from_numpy(plan.param_vector()).cuda()
    xd, Gd = torch.from_numpy(xp).cuda(), torch.from_numpy(G).cuda()
    od = torch.from_numpy(off).cuda()
    order = torch.from_numpy(stl.lpt_order(off)).cuda()
    launch, ms = stl.autotune(plan, xd, pv, Gd, offsets=od, order=order, T=T)
    print("ragged n=200 T=%d tuned threads=%d wg_per_cu=%d global=%d (%.3f ms)"
          % (T, launch.threads, launch.wg_per_cu, launch.global_slots, ms), flush=True)
    root = plan.forward(xd, pv, offsets=od, order=order, T=T, launch=launch)
    dx, gp = plan.backward(xd, Gd, pv, offsets=od, order=order, T=T, launch=launch)
    torch.cuda.synchronize()
    gr = stl.Graph(plan, xd, pv, Gd, offsets=od, order=order, T=T, launch=launch)
    for rep in range(3):
        gr.launch()
        torch.cuda.synchronize()
        assert torch.equal(gr.root, root), rep
        assert torch.equal(gr.dx, dx), rep
        assert torch.equal(gr.gp[: gp.numel()], gp), rep
        _ = (xd * 2).sum().item()                 # other eager work between replays
    ref = oracle.forward(spec, xp, offsets=off)
    assert_close(root.cpu().numpy(), ref, what="ragged path root")
    dxr, _ = oracle.backward(spec, xp, G, offsets=off)
    dxa, _ = oracle.backward(spec, xp, np.abs(G), offsets=off)
    assert_close(dx.cpu().numpy(), dxr, scale=np.abs(dxr).max(), elem_scale=dxa, what="ragged path dx")


def test_autotuned_launch_forward_and_backward():
    import torch
    spec, params, x = W.workload(1, B=64, T=500)
    g = Gpu(spec, 4, params)
    xt = torch.from_numpy(x).cuda()
    G = torch.from_numpy(W.upstream_grad(101, x.shape[:2])).cuda()
    best, ms = stl.autotune(g.plan, xt, g.pv, G)
    r0 = g.plan.forward(xt, g.pv)
    r1 = g.plan.forward(xt, g.pv, launch=best)
    d0, _ = g.plan.backward(xt, G, g.pv)
    d1, _ = g.plan.backward(xt, G, g.pv, launch=best)
    torch.cuda.synchronize()
    assert_close(r1.cpu().numpy(), r0.cpu().numpy(), rel=2e-6, what="tuned root")
    d0 = d0.cpu().numpy()
    assert_close(d1.cpu().numpy(), d0, rel=2e-6, scale=np.abs(d0).max(), what="tuned dx")


def test_interval_sweep_benchmark_size_sampled():
    """4096 random-walk signals of T = 20 against the 300 x 300 grid of (a, b)
    fractions (90,000 intervals), the benchmarked launch: every output finite,
    and 8 signals x 3000 intervals against the oracle."""
    import torch
    T, B = 20, 4096
    gl = np.linspace(0.0, 1.0, 300)
    af, bf = np.meshgrid(gl, gl, indexing="ij")
    a = (af.ravel() * T).astype(np.float32)
    b = (bf.ravel() * T).astype(np.float32)
    rng = np.random.default_rng(6)
    x = np.cumsum(rng.normal(size=(B, T, 1)) * 0.3, axis=1).astype(np.float32)
    kw = dict(op="always", smooth=True, beta=10.0, mask_c=1.0, mask_eps=1e-6)
    xd, ad, bd = (torch.from_numpy(v).cuda() for v in (x, a, b))
    rho, ga, gb = stl.interval_sweep(xd, ad, bd, [1.0], **kw)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(rho).all()) and bool(torch.isfinite(ga).all()) and bool(torch.isfinite(gb).all())
    rows = np.array([0, 1, 517, 2048, 3000, 4093, 4094, 4095])
    cols = np.sort(rng.choice(a.size, size=3000, replace=False))
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    got = [v.index_select(0, ri).index_select(1, ci).cpu().numpy() for v in (rho, ga, gb)]
    r0, ga0, gb0 = oracle.interval_sweep(x[rows], a[cols].astype(np.float64), b[cols].astype(np.float64), [1.0], **kw)
    assert_close(got[0], r0, what="full-size sweep rho")
    sc = 1.0 / (4 * 10.0)
    assert_close(got[1], ga0, scale=sc, what="full-size sweep d/da")
    assert_close(got[2], gb0, scale=sc, what="full-size sweep d/db")


def test_ragged_forward_with_node_traces_captures_in_a_graph():
    """stl_forward on a ragged batch writing every node's trace ([n_nodes][N_total],
    N_total read from offsets on the device) neither synchronises nor copies to
    the host, so it records into a graph; three replays equal the eager call."""
    import torch
    spec, params, xp, off = W.ragged_workload(n=30)
    T = int(np.diff(off).max())
    plan = stl.Plan(spec, xp.shape[-1], params)
    pv = torch.from_numpy(plan.param_vector()).cuda()
    xd, od = torch.from_numpy(xp).cuda(), torch.from_numpy(off).cuda()
    root0, nodes0 = plan.forward(xd, pv, offsets=od, T=T, node_traces=True)     # eager (sizes the workspace)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        root1, nodes1 = plan.forward(xd, pv, offsets=od, T=T, node_traces=True)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(root1, root0), rep
        assert torch.equal(nodes1, nodes0), rep
        _ = (xd * 2).sum().item()                 # other eager work between replays
    ref = oracle.forward(spec, xp, offsets=off)
    assert_close(root1.cpu().numpy(), ref, what="captured ragged root")
