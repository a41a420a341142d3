"""GPU parity of the fused smooth-mask path (stl_forward / stl_backward pick
it for dense batches of smooth And/Or over smooth-mask nodes on linear
predicates) against the FP64 oracle and against the generic executor, and
its hand-off of trajectories it cannot take to the generic executor."""
import numpy as np
import pytest

from gpu_util import Gpu, assert_close, check_formula
from paper_2501_04194_amd import stl, workloads as W

pytestmark = pytest.mark.gpu

GENERIC = stl.Launch(256, 0, 0, 1)      # flags bit 0: no fused path
FP64 = stl.Launch(256, 0, 0, 2)         # flags bit 1: the fp64 fused kernels (not the matrix-core path)


def lin(w, c=0.0):
    return {"op": "linear", "w": list(map(float, w)), "c": float(c)}


def mask(kind, child, a, b, c=1.0, eps=1e-6, beta=10.0):
    return {"op": kind, "smooth": True, "beta": beta, "child": child,
            "mask": {"a": a, "b": b, "c": c, "eps": eps}}


def both_paths(spec, x, params, G, what):
    """fp64 fused vs generic on the same inputs: float32 rounding level agreement."""
    f = Gpu(spec, x.shape[-1], params, launch=FP64)
    g = Gpu(spec, x.shape[-1], params, launch=GENERIC)
    rf, rg = f.fwd(x), g.fwd(x)
    assert_close(rf, rg, rel=3e-6, what=what + " root fused/generic")
    (df, pf), (dg, pg) = f.bwd(x, G), g.bwd(x, G)
    assert_close(df, dg, rel=3e-6, scale=np.abs(dg).max(), what=what + " dx fused/generic")
    for k in pg:
        # both are sums over every timestep of the batch in different orders
        assert abs(pf[k] - pg[k]) <= 5e-5 * (abs(pg[k]) + 1e-3), (what, k, pf[k], pg[k])


@pytest.mark.parametrize("T", [2048, 1500, 333, 64])
def test_fused_headline_formula(T):
    spec, params, x = W.workload(2, B=6, T=T)
    check_formula(spec, x, params=params, what="fused cfg2 T=%d" % T)
    G = W.upstream_grad(7, x.shape[:2])
    both_paths(spec, x, params, G, "cfg2 T=%d" % T)


@pytest.mark.parametrize("case", range(7))
def test_fused_shapes(case):
    rng = np.random.default_rng(40 + case)
    x = np.cumsum(rng.normal(size=(5, 900, 3)) * 0.05, axis=1).astype(np.float32)
    p0, p1, p2 = lin([1, 0, 0]), lin([0, -1, 0], -0.3), lin([0.5, 0.5, 1.0], 0.1)
    specs = [
        mask("eventually", p0, "a", "b"),                                            # single mask root
        {"op": "or", "smooth": True, "beta": 7.0, "children": [
            mask("eventually", p0, "a", "b"), mask("always", p1, 30.0, 80.0, c=2.0),
            mask("eventually", p2, 5.0, 700.0, c=0.7)]},
        {"op": "and", "smooth": True, "beta": 10.0, "children": [
            mask("always", p0, "a", None), mask("eventually", p2, 0.0, 40.0)]},       # unbounded mask
        {"op": "and", "smooth": True, "beta": 10.0, "children": [
            mask("always", p0, 20.0, 24.0, c=0.3, eps=1e-4), mask("eventually", p1, "a", "b")]},  # no core
        {"op": "and", "smooth": True, "beta": 4.0, "children": [
            mask("always", p0, 880.0, 1200.0), mask("eventually", p1, "a", "b")]},   # support past the end
        mask("always", p2, 2000.0, 3000.0),                                          # empty support
        {"op": "or", "smooth": True, "beta": 10.0, "children": [
            mask("eventually", p0, 10.0, 44.5), mask("always", p1, 10.0, 45.0)]},     # cores of 1 and 2 steps
    ]
    params = {"a": 100.0, "b": 400.0}
    spec = specs[case]
    check_formula(spec, x, params=params, what="fused shape %d" % case)
    G = np.random.default_rng(3).normal(size=x.shape[:2]).astype(np.float32)
    both_paths(spec, x, params, G, "shape %d" % case)


def test_fused_hands_off_to_generic():
    """A trajectory whose signal range exceeds the fp64 exponent range, and a
    mask whose bands are wider than the fused limit, are recomputed by the
    generic executor inside the same call."""
    spec, params, x = W.workload(2, B=5, T=800)
    x[2, 400:, 0] += 300.0                # range 300 * beta * log2(e) >> 1000
    check_formula(spec, x, params=params, what="handoff range")
    # (on unshifted signals: a trace near 300 has exponents beta*log2(e)*300 ~ 4300 whose
    # float32 rounding alone is a relative error of ~2e-4 in each term)
    _, _, x = W.workload(2, B=5, T=800)
    wide = {"op": "and", "smooth": True, "beta": 10.0, "children": [
        mask("eventually", lin([1, 0]), 100.0, 400.0, c=0.02), mask("always", lin([0, 1]), 50.0, 90.0)]}
    check_formula(wide, x, params={}, what="handoff wide band")


def test_fused_grad_params_fd():
    """d/da, d/db of the fused path against central differences of its own forward."""
    import torch
    spec, params, x = W.workload(2, B=4, T=1024)
    g = Gpu(spec, 2, params)
    G = W.upstream_grad(8, x.shape[:2]).astype(np.float32)
    _, dp = g.bwd(x, G)
    for name in ("ev_a", "ev_b", "al_a", "al_b"):
        h = 0.05
        pp = dict(g.params); pp[name] += h
        pm = dict(g.params); pm[name] -= h
        fp = Gpu(spec, 2, pp).fwd(x).astype(np.float64)
        fm = Gpu(spec, 2, pm).fwd(x).astype(np.float64)
        fd = ((fp - fm) * G).sum() / (2 * h)
        assert abs(dp[name] - fd) <= 2e-3 * (abs(fd) + 1.0), (name, dp[name], fd)


def _saved_run(g, x, G, fwd_launch=None, bwd_launch=None):
    t = g.torch
    xd = t.from_numpy(np.ascontiguousarray(x)).cuda()
    Gd = t.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).cuda()
    sv = g.plan.saved_buffer(xd)
    sv.fill_(0xAB)                       # stale contents must not leak into the result
    root = g.plan.forward(xd, g.pv, saved=sv, launch=fwd_launch)
    dx, gp = g.plan.backward(xd, Gd, g.pv, saved=sv, launch=bwd_launch)
    t.cuda.synchronize()
    return root.cpu().numpy(), dx.cpu().numpy(), g.plan.param_grads(gp.cpu().numpy())


def test_saved_traces_match_recompute():
    """stl_forward_saving + stl_backward_saved give bit-identical results to
    stl_forward + stl_backward: the saved traces are the very values the
    backward would recompute.  The batch includes a trajectory handed off to
    the generic executor (its saved flag is 0)."""
    spec, params, x = W.workload(2, B=7, T=1200)
    x[4, 600:, 1] -= 250.0
    G = W.upstream_grad(9, x.shape[:2])
    g = Gpu(spec, 2, params)
    r0 = g.fwd(x)
    d0, p0 = g.bwd(x, G)
    r1, d1, p1 = _saved_run(g, x, G)
    assert np.array_equal(r0, r1)
    assert np.array_equal(d0, d1)
    for k in p0:
        assert p0[k] == p1[k], k


def test_saved_after_generic_forward_recomputes():
    """A forward that did not take a fused path flags every trajectory 0, so
    the backward does not read the buffer: it recomputes (the generic
    executor takes the flagged trajectories) and still matches the oracle."""
    import oracle
    from gpu_util import f32params
    spec, params, x = W.workload(2, B=3, T=500)
    G = W.upstream_grad(10, x.shape[:2])
    g = Gpu(spec, 2, params)
    _, d1, p1 = _saved_run(g, x, G, fwd_launch=GENERIC)
    dxr, dpr = oracle.backward(spec, x, G, params=f32params(params))
    dxa, dpa = oracle.backward(spec, x, np.abs(G), params=f32params(params))
    assert_close(d1, dxr, scale=np.abs(dxr).max(), elem_scale=dxa, what="saved after generic dx")
    for k in dpr:
        assert abs(p1[k] - dpr[k]) <= 1e-5 * abs(dpa[k]) + 1e-12, k


def test_saved_size_and_errors():
    import ctypes
    import torch
    spec, params, x = W.workload(2, B=3, T=500)
    g = Gpu(spec, 2, params)
    xd = torch.from_numpy(x).cuda()
    sv = g.plan.saved_buffer(xd)
    # flags, two [B][T] arrays, and (matrix-core path) the exponent range and
    # reference of each trajectory's two traces, padded to 256 bytes, then
    # 256 bytes of the masks' geometry
    assert sv.numel() == (256 + 2 * 3 * 500 * 4 + 3 * 2 * 3 * 4 + 255) // 256 * 256 + 256
    small = sv[:1000]
    with pytest.raises(stl.StlError, match="saved buffer too small"):
        g.plan.forward(xd, g.pv, saved=small)
    # a plan without the fused shape needs only the flag header
    p2 = stl.Plan({"op": "always", "a": 0, "b": 5, "child": lin([1, 0])}, 2)
    assert p2.saved_buffer(xd).numel() == 256
    del ctypes


def test_autograd_function_uses_saved_traces():
    """torch.autograd through StlRobustness: gradients of a loss on the trace
    equal the C-ABI backward with G = d loss / d trace."""
    import torch
    spec, params, x = W.workload(2, B=4, T=900)
    g = Gpu(spec, 2, params)
    xd = torch.from_numpy(x).cuda().requires_grad_(True)
    pv = g.pv.clone().requires_grad_(True)
    G = torch.from_numpy(W.upstream_grad(11, x.shape[:2])).cuda()
    rho = stl.robustness(g.plan, xd, pv)
    (rho * G).sum().backward()
    d0, p0 = g.bwd(x, G.cpu().numpy())
    assert np.array_equal(xd.grad.cpu().numpy(), d0)
    gp = g.plan.param_grads(pv.grad.cpu().numpy())
    for k in p0:
        assert gp[k] == p0[k], k


@pytest.mark.parametrize("generic", [False, True])
def test_tied_mask_bounds_share_parameters(generic):
    """Two mask nodes tied to the same (a, b, c, eps) names share one group of
    parameter slots in the plan; d/da and d/db sum both nodes' contributions
    (the oracle sums per name), on the fused path and on the generic executor."""
    spec = {"op": "and", "smooth": True, "beta": 10.0, "children": [
        mask("eventually", lin([1, 0]), "a", "b", c="c", eps="eps"),
        mask("always", lin([0, -1], -0.5), "a", "b", c="c", eps="eps")]}
    params = {"a": 60.0, "b": 250.0, "c": 1.0, "eps": 1e-6}
    plan = stl.Plan(spec, 2, params)
    assert plan.n_params == 7          # one shared mask group + the three beta slots (11 untied)
    _, _, x = W.workload(2, B=7, T=700)
    check_formula(spec, x, params=params, launch=GENERIC if generic else None,
                  what="tied bounds generic=%s" % generic)
