"""GPU parity of the matrix-core smooth-mask path (dense batches of a smooth
And/Or over one or two bounded smooth-mask nodes on linear predicates, D <= 2)
against the FP64 oracle, against the fp64 fused kernels and the generic
executor, and its hand-off of trajectories and masks it cannot take."""
import numpy as np
import pytest

from gpu_util import Gpu, assert_close, check_formula
from paper_2501_04194_amd import stl, workloads as W

pytestmark = pytest.mark.gpu

GENERIC = stl.Launch(256, 0, 0, 1)      # flags bit 0: generic executor only
FP64 = stl.Launch(256, 0, 0, 2)         # flags bit 1: the fp64 fused kernels


def lin(w, c=0.0):
    return {"op": "linear", "w": list(map(float, w)), "c": float(c)}


def mask(kind, child, a, b, c=1.0, eps=1e-6, beta=10.0):
    return {"op": kind, "smooth": True, "beta": beta, "child": child,
            "mask": {"a": a, "b": b, "c": c, "eps": eps}}


def agree(spec, x, params, G, other, what, rel=2e-5):
    """matrix-core path vs another path on the same inputs"""
    f = Gpu(spec, x.shape[-1], params)
    g = Gpu(spec, x.shape[-1], params, launch=other)
    assert_close(f.fwd(x), g.fwd(x), rel=rel, what=what + " root")
    (df, pf), (dg, pg) = f.bwd(x, G), g.bwd(x, G)
    assert_close(df, dg, rel=rel, scale=np.abs(dg).max(), what=what + " dx")
    for k in pg:
        assert abs(pf[k] - pg[k]) <= 1e-4 * (abs(pg[k]) + 1e-3), (what, k, pf[k], pg[k])


@pytest.mark.parametrize("T", [2048, 1500, 700, 333, 64, 17, 1])
def test_mx_headline_formula(T):
    """B = 19 (a partial group of 16), several chunks and a ragged last tile."""
    spec, params, x = W.workload(2, B=19, T=T)
    check_formula(spec, x, params=params, what="mx cfg2 T=%d" % T)


def test_mx_agrees_with_fp64_and_generic():
    spec, params, x = W.workload(2, B=20, T=900)
    G = W.upstream_grad(8, x.shape[:2])
    agree(spec, x, params, G, FP64, "mx/fp64")
    agree(spec, x, params, G, GENERIC, "mx/generic")


@pytest.mark.parametrize("T", [800, 799])
@pytest.mark.parametrize("case", range(6))
def test_mx_shapes(case, T):
    """T = 800 takes the 16-byte-load kernels, T = 799 the others."""
    rng = np.random.default_rng(70 + case)
    D = 1 if case == 3 else 2
    x = np.cumsum(rng.normal(size=(21, T, D)) * 0.05, axis=1).astype(np.float32)
    p0 = lin([1.0] * D)
    p1 = lin([-1.0] + [0.5] * (D - 1), -0.3)
    specs = [
        mask("always", p0, "a", "b"),                                                  # single mask root
        {"op": "or", "smooth": True, "beta": 7.0, "children": [
            mask("eventually", p0, 30.0, 80.0, c=2.0), mask("always", p1, 5.0, 300.0, c=0.7)]},
        {"op": "and", "smooth": True, "beta": 10.0, "children": [
            mask("always", p0, 0.0, 40.0), mask("eventually", p1, "a", "b")]},        # window from offset 0
        {"op": "and", "smooth": True, "beta": 4.0, "children": [
            mask("eventually", p0, 600.0, 900.0), mask("always", p1, "a", "b")]},     # support past the end
        mask("eventually", p1, 2000.0, 3000.0),                                       # empty support
        {"op": "or", "smooth": True, "beta": 10.0, "children": [
            mask("eventually", p0, 10.0, 44.5), mask("always", p1, 10.0, 45.0)]},      # cores of 1 and 2 steps
    ]
    params = {"a": 100.0, "b": 400.0}
    check_formula(specs[case], x, params=params, what="mx shape %d T=%d" % (case, T))


@pytest.mark.parametrize("seed", range(8))
def test_mx_random_windows(seed):
    """Two masks with seeded windows and sigmoid slopes: the derivative bands
    (about 34 / c offsets wide) cover one to three K-steps each, so the
    backward's lists of d/da and d/db tiles split differently between the
    kinds, or exceed the list and hand off (d/d bounds compared too)."""
    rng = np.random.default_rng(300 + seed)
    T = 640 if seed % 2 else 639
    x = np.cumsum(rng.normal(size=(17, T, 2)) * 0.05, axis=1).astype(np.float32)
    slopes = [0.6, 1.0, 1.7, 3.0]
    params = {}
    kids = []
    for m, (kind, pred) in enumerate([("eventually", lin([1.0, 0.0])), ("always", lin([0.0, -1.0], -0.2))]):
        a = float(rng.uniform(0.0, 150.0))
        params["a%d" % m], params["b%d" % m] = a, a + float(rng.uniform(15.0, 300.0))
        kids.append(mask(kind, pred, "a%d" % m, "b%d" % m, c=slopes[int(rng.integers(4))]))
    spec = {"op": "and" if seed % 3 else "or", "smooth": True, "beta": 10.0, "children": kids}
    check_formula(spec, x, params=params, what="mx random windows %d" % seed)


def test_mx_hands_off_wide_range_and_wide_masks():
    """A trajectory whose exponent range exceeds the staged limit, a mask
    wider than the tiles (b - a = 500) and one whose derivative bands need
    more tiles than the kernel keeps (no core, c = 0.3) all go to the generic
    executor inside the same call."""
    spec, params, x = W.workload(2, B=18, T=900)
    x[3, 450:, 0] += 25.0                       # 25 * beta * log2(e) = 361 > 200
    x[17, :300, 1] -= 16.0
    check_formula(spec, x, params=params, what="mx handoff range")
    _, _, x = W.workload(2, B=18, T=900)
    wide = {"op": "and", "smooth": True, "beta": 10.0, "children": [
        mask("eventually", lin([1, 0]), 50.0, 550.0), mask("always", lin([0, 1]), 50.0, 90.0)]}
    check_formula(wide, x, params={}, what="mx handoff wide window")
    nocore = {"op": "and", "smooth": True, "beta": 10.0, "children": [
        mask("eventually", lin([1, 0]), 20.0, 24.0, c=0.3, eps=1e-4), mask("always", lin([0, 1]), 50.0, 90.0)]}
    check_formula(nocore, x, params={}, what="mx handoff derivative tiles")


def test_mx_saved_equals_recompute_and_is_deterministic():
    """Saved pair vs recompute, bit for bit, with two trajectories handed to
    the generic executor; the saved backward runs twice after one forward
    (each call rewrites every hand-off flag it reads)."""
    import torch
    spec, params, x = W.workload(2, B=40, T=1200)
    x[5, 600:, 0] += 25.0
    x[33, :200, 1] -= 20.0
    G = W.upstream_grad(9, x.shape[:2])
    g = Gpu(spec, 2, params)
    xd, Gd = torch.from_numpy(x).cuda(), torch.from_numpy(G).cuda()
    sv = g.plan.saved_buffer(xd)
    r1 = g.plan.forward(xd, g.pv, saved=sv)
    d1, p1 = g.plan.backward(xd, Gd, g.pv, saved=sv)
    d1b, p1b = g.plan.backward(xd, Gd, g.pv, saved=sv)
    r2 = g.plan.forward(xd, g.pv)
    d2, p2 = g.plan.backward(xd, Gd, g.pv)
    d3, p3 = g.plan.backward(xd, Gd, g.pv)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2)
    assert torch.equal(d1, d2) and torch.equal(p1, p2)
    assert torch.equal(d1b, d1) and torch.equal(p1b, p1)
    assert torch.equal(d2, d3) and torch.equal(p2, p3)
    check_formula(spec, x, params=params, what="mx saved handoff")


def test_mx_graph_replay_matches_eager():
    import torch
    spec, params, x = W.workload(2, B=33, T=1000)
    g = Gpu(spec, 2, params)
    xd = torch.from_numpy(x).cuda()
    Gd = torch.from_numpy(W.upstream_grad(11, x.shape[:2])).cuda()
    root = g.plan.forward(xd, g.pv)
    dx, gp = g.plan.backward(xd, Gd, g.pv)
    torch.cuda.synchronize()
    gr = stl.Graph(g.plan, xd, g.pv, Gd)
    for _ in range(3):
        gr.launch()
        torch.cuda.synchronize()
        assert torch.equal(gr.root.view_as(root), root)
        assert torch.equal(gr.dx, dx)
        assert torch.equal(gr.gp[: gp.numel()], gp)
        _ = (xd * 2).sum().item()                    # other eager work between replays


def test_mx_full_size_sampled_against_oracle():
    """The benchmark's batch (B = 4096, T = 2048) through the pair it times
    (stl_forward_saving + stl_backward_saved): root and d/dx of 6 sampled
    trajectories against the oracle, d/da and d/db of the whole batch against
    the oracle's sums over every timestep (1e-5 of the sum of |terms|)."""
    import oracle
    import torch
    from gpu_util import REL, f32params
    spec, params, x = W.workload(2)
    params = f32params(params)
    G = W.upstream_grad(102, x.shape[:2])
    g = Gpu(spec, 2, params)
    xd, Gd = torch.from_numpy(x).cuda(), torch.from_numpy(G).cuda()
    sv = g.plan.saved_buffer(xd)
    root = g.plan.forward(xd, g.pv, saved=sv)
    dx, gp = g.plan.backward(xd, Gd, g.pv, saved=sv)
    torch.cuda.synchronize()
    root, dx = root.cpu().numpy(), dx.cpu().numpy()
    idx = [0, 1, 777, 2048, 3001, 4095]
    ref = oracle.forward(spec, x[idx], params=params)
    assert_close(root[idx], ref, what="full-size root")
    dxr, _ = oracle.backward(spec, x[idx], G[idx], params=params)
    dxa, _ = oracle.backward(spec, x[idx], np.abs(G[idx]), params=params)
    assert_close(dx[idx], dxr, scale=np.abs(dxr).max(), elem_scale=dxa, what="full-size dx")
    _, dpr = oracle.backward(spec, x, G, params=params)
    _, dpa = oracle.backward(spec, x, np.abs(G), params=params)
    got = g.plan.param_grads(gp.cpu().numpy())
    for k, v in dpr.items():
        assert abs(got[k] - v) <= REL * abs(dpa[k]) + 1e-12, (k, got[k], v, dpa[k])


def test_mx_unaligned_inputs_match_aligned():
    """x, G and the saved buffer at addresses that are not 16-byte aligned
    take the kernels with scalar loads: the same bits as the aligned call."""
    import torch
    spec, params, x = W.workload(2, B=24, T=1024)
    G = W.upstream_grad(12, x.shape[:2])
    g = Gpu(spec, 2, params)
    xa, Ga = torch.from_numpy(x).cuda(), torch.from_numpy(G).cuda()
    xu = torch.empty(x.size + 1, dtype=torch.float32, device="cuda")[1:].view(x.shape)
    Gu = torch.empty(G.size + 1, dtype=torch.float32, device="cuda")[1:].view(G.shape)
    xu.copy_(xa)
    Gu.copy_(Ga)
    assert xu.data_ptr() % 16 != 0 and Gu.data_ptr() % 16 != 0
    outs = []
    for xd, Gd in ((xa, Ga), (xu, Gu)):
        sv = g.plan.saved_buffer(xd)
        r = g.plan.forward(xd, g.pv, saved=sv)
        d, p = g.plan.backward(xd, Gd, g.pv, saved=sv)
        d2, p2 = g.plan.backward(xd, Gd, g.pv)
        outs.append((r, d, p, d2, p2))
    torch.cuda.synchronize()
    for a, b in zip(*outs):
        assert torch.equal(a, b)
