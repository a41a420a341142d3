"""GPU parity of the smooth time mask (Sec. VI) on Until and of the LAST /
CONST pads on smooth-mask Eventually / Always, against the FP64 oracle.

Until: the mask weights the Until index i (the psi index the interval
constrains) inside the outer smooth max; the hard form takes the max over the
mask support.  Pads: every support offset past the signal end contributes one
pad copy with its weight.  Calls go through the C ABI; tolerances are those of
``gpu_util`` (hard selections bit-exact).
"""
import numpy as np
import pytest

import oracle
from gpu_util import Gpu, assert_close, check_formula

pytestmark = pytest.mark.gpu

S1 = {"op": "linear", "w": [1.0], "c": 0.0}
PHI = {"op": "linear", "w": [1.0, 0.0], "c": -0.5}
PSI = {"op": "linear", "w": [0.0, 1.0], "c": 0.1}


def walk(rng, B, L, D=1, s=0.1):
    return np.cumsum(rng.normal(size=(B, L, D)) * s, axis=1).astype(np.float32)


def mask(a, b, c, eps):
    return {"a": "a", "b": None if b is None else "b", "c": c, "eps": eps}


def mparams(a, b):
    return {"a": a} if b is None else {"a": a, "b": b}


def until(m, smooth=True, left=PHI, right=PSI):
    kw = {"smooth": True, "beta": 10.0} if smooth else {}
    return dict({"op": "until", "left": left, "right": right, "mask": mask(*m)}, **kw)


# --------------------------------------------------------------------------- smooth mask on Until

UNTIL_MASKS = [
    (5.3, 60.7, 1.0, 1e-6),       # bands at both ends, interior core
    (0.0, 30.0, 1.0, 1e-6),       # sigmoid tail clipped at offset 0
    (40.0, None, 2.0, 1e-6),      # unbounded mask: walks to the end
    (20.0, 24.0, 0.3, 1e-4),      # wide bands, no flat part
    (380.0, 450.0, 1.0, 1e-6),    # support running past the end for most t
]


@pytest.mark.parametrize("m", UNTIL_MASKS)
def test_masked_until_smooth(m):
    rng = np.random.default_rng(41)
    x = walk(rng, 3, 420, D=2, s=0.1)
    check_formula(until(m), x, params=mparams(m[0], m[1]), what="masked until %s" % (m,))


def test_masked_until_sparse_gradient_and_ragged():
    rng = np.random.default_rng(42)
    m = (7.2, 90.4, 1.5, 1e-6)
    x = walk(rng, 2, 700, D=2, s=0.1)
    G = rng.normal(size=(2, 700)).astype(np.float32)
    G[rng.random(G.shape) < 0.8] = 0.0
    check_formula(until(m), x, params=mparams(7.2, 90.4), G=G, what="sparse-G masked until")
    off = np.array([0, 130, 131, 500, 777], dtype=np.int64)
    xp = walk(rng, 1, 777, D=2, s=0.1)[0]
    check_formula(until(m), xp, params=mparams(7.2, 90.4), offsets=off, T=369, what="ragged masked until")


def test_masked_until_hard_bitexact():
    # predicate constants exact in float32, so both sides select on identical values
    rng = np.random.default_rng(43)
    x = walk(rng, 3, 333, D=2, s=0.1)
    psi = {"op": "linear", "w": [0.0, 1.0], "c": 0.25}
    for m in [(5.3, 60.7, 1.0, 1e-6), (12.0, None, 2.0, 1e-6), (300.0, 400.0, 1.0, 1e-6)]:
        check_formula(until(m, smooth=False, right=psi), x, params=mparams(m[0], m[1]), bitexact_root=True,
                      what="hard masked until %s" % (m,))


def test_masked_until_wide_range_and_true_left():
    """Exponent ranges beyond the fp64 form take the scaled-pair path; with
    phi = True the masked Until equals the masked Eventually of psi."""
    rng = np.random.default_rng(44)
    x = walk(rng, 2, 300, D=2, s=0.1) * np.float32(60.0)
    check_formula(until((3.5, 44.5, 1.0, 1e-6)), x, params=mparams(3.5, 44.5), what="wide masked until")
    x = walk(rng, 2, 260, D=2, s=0.1)
    m = (4.3, 37.8, 1.5, 1e-6)
    check_formula(until(m, left={"op": "true"}), x, params=mparams(4.3, 37.8), what="true masked until")


def test_masked_until_empty_support():
    """A mask whose support lies past every trajectory: constant -rho_pad,
    zero gradients."""
    rng = np.random.default_rng(45)
    x = walk(rng, 2, 120, D=2, s=0.1)
    g = Gpu(until((500.0, 600.0, 1.0, 1e-6)), 2, mparams(500.0, 600.0))
    r = g.fwd(x)
    assert np.all(r == np.float32(-1e6))
    dx, dp = g.bwd(x, rng.normal(size=(2, 120)).astype(np.float32))
    assert np.all(dx == 0) and dp["a"] == 0 and dp["b"] == 0


def test_masked_until_in_formula():
    """A masked Until below an And with a masked Always: both masks learn."""
    rng = np.random.default_rng(46)
    x = walk(rng, 3, 500, D=2, s=0.08)
    spec = {"op": "and", "smooth": True, "beta": 5.0, "children": [
        {"op": "until", "smooth": True, "beta": 8.0, "left": PHI, "right": PSI,
         "mask": {"a": "ua", "b": "ub", "c": 1.0, "eps": 1e-6}},
        {"op": "always", "smooth": True, "beta": 8.0, "child": PSI,
         "mask": {"a": "wa", "b": "wb", "c": 0.7, "eps": 1e-6}}]}
    check_formula(spec, x, params={"ua": 10.2, "ub": 70.9, "wa": 3.1, "wb": 25.6}, what="until+always masks")


# --------------------------------------------------------------------------- pads on smooth masks

PAD_MASKS = [
    (100.0, 400.0, 1.0, 1e-6),    # headline shape: pads for the last ~413 outputs
    (10.3, 40.7, 1.0, 1e-6),
    (20.0, 24.0, 0.3, 1e-4),      # no flat part
    (600.0, 900.0, 1.0, 1e-6),    # support running past the end for every t
    (800.0, 900.0, 1.0, 1e-6),    # support entirely past the end: pads only
    (10.0, 40.0, 1.0, 0.0),       # eps = 0: the tail runs until the weights underflow
]


@pytest.mark.parametrize("m", PAD_MASKS)
@pytest.mark.parametrize("pad", ["last", "const"])
@pytest.mark.parametrize("kind", ["eventually", "always"])
def test_mask_pads_smooth(m, pad, kind):
    rng = np.random.default_rng(47)
    x = walk(rng, 3, 700, s=0.05)
    spec = {"op": kind, "smooth": True, "beta": 10.0, "child": S1, "mask": mask(*m), "pad": pad,
            "pad_value": 0.3}
    check_formula(spec, x, params=mparams(m[0], m[1]), what="mask pad %s %s %s" % (m, pad, kind))


@pytest.mark.parametrize("pad", ["last", "const"])
def test_mask_pads_hard_bitexact(pad):
    rng = np.random.default_rng(48)
    x = (rng.normal(size=(2, 500, 1))).astype(np.float32)
    for m in [(9.5, 130.5, 3.0, 1e-6), (450.0, 520.0, 1.0, 1e-6), (600.0, 700.0, 1.0, 1e-6)]:
        for kind in ("eventually", "always"):
            spec = {"op": kind, "child": S1, "mask": mask(*m), "pad": pad, "pad_value": 0.25}
            check_formula(spec, x, params=mparams(m[0], m[1]), bitexact_root=True,
                          what="hard mask pad %s %s %s" % (m, pad, kind))


def test_mask_pads_unbounded_mask_ignores_pad():
    """An unbounded mask already reaches the end: its pad policy has no effect."""
    rng = np.random.default_rng(49)
    x = walk(rng, 2, 300, s=0.05)
    m = (20.0, None, 1.0, 1e-6)
    base = {"op": "eventually", "smooth": True, "beta": 10.0, "child": S1, "mask": mask(*m)}
    r0 = Gpu(base, 1, mparams(20.0, None)).fwd(x)
    r1 = Gpu(dict(base, pad="last"), 1, mparams(20.0, None)).fwd(x)
    assert np.array_equal(r0, r1)
    check_formula(dict(base, pad="const", pad_value=5.0), x, params=mparams(20.0, None), what="unbounded+pad")


def test_mask_pads_on_the_fused_shape():
    """The smooth And of two masked windows on linear predicates normally takes
    the fused kernel; with a pad it runs on the generic executor and still
    matches the oracle."""
    rng = np.random.default_rng(50)
    x = walk(rng, 4, 900, D=2, s=0.05)
    spec = {"op": "and", "smooth": True, "beta": 10.0, "children": [
        {"op": "eventually", "smooth": True, "beta": 10.0, "child": PHI, "pad": "last",
         "mask": {"a": "ea", "b": "eb", "c": 1.0, "eps": 1e-6}},
        {"op": "always", "smooth": True, "beta": 10.0, "child": PSI,
         "mask": {"a": "la", "b": "lb", "c": 1.0, "eps": 1e-6}}]}
    check_formula(spec, x, params={"ea": 100.0, "eb": 400.0, "la": 50.0, "lb": 200.0}, what="fused shape + pad")
    ref = oracle.forward(dict(spec, children=[dict(spec["children"][0], pad="neutral"), spec["children"][1]]), x,
                         params={"ea": 100.0, "eb": 400.0, "la": 50.0, "lb": 200.0})
    got = Gpu(spec, 2, {"ea": 100.0, "eb": 400.0, "la": 50.0, "lb": 200.0}).fwd(x)
    # the pad changes the outputs whose Eventually window reaches past the end
    assert np.abs(got[:, -300:] - ref[:, -300:]).max() > 1e-4
    assert_close(got[:, :400], ref[:, :400], what="outputs away from the end")


def test_masked_until_and_pads_in_global_arenas():
    """The same operators with the slot arena in global memory (forced by the
    launch configuration, and by a trajectory too long for LDS): the Until
    sums and the pad tables then live behind global pointers."""
    from paper_2501_04194_amd import stl
    rng = np.random.default_rng(51)
    glob = stl.Launch(256, 2, 1, 0)
    x = walk(rng, 3, 420, D=2, s=0.1)
    m = (5.3, 60.7, 1.0, 1e-6)
    check_formula(until(m), x, params=mparams(m[0], m[1]), launch=glob, what="global masked until")
    check_formula(until(m, smooth=False, right={"op": "linear", "w": [0.0, 1.0], "c": 0.25}), x,
                  params=mparams(m[0], m[1]), launch=glob, bitexact_root=True, what="global hard masked until")
    xs = walk(rng, 3, 700, s=0.05)
    for pad in ("last", "const"):
        spec = {"op": "always", "smooth": True, "beta": 10.0, "child": S1, "mask": mask(100.0, 400.0, 1.0, 1e-6),
                "pad": pad, "pad_value": 0.3}
        check_formula(spec, xs, params=mparams(100.0, 400.0), launch=glob, what="global mask pad %s" % pad)
    # long trajectories: the arena does not fit in LDS at this length
    xl = walk(rng, 2, 2600, D=2, s=0.05)
    check_formula(until((12.5, 140.5, 1.0, 1e-6)), xl, params=mparams(12.5, 140.5), what="long masked until")
    spec = {"op": "eventually", "smooth": True, "beta": 10.0, "child": PHI, "mask": mask(2400.0, 2900.0, 1.0, 1e-6),
            "pad": "last"}
    check_formula(spec, xl, params=mparams(2400.0, 2900.0), what="long mask pad")


def test_mask_ext_length_one_and_two():
    """Trajectories of one and two samples: masks whose support starts past
    the end, pads that supply every term, and a masked Until with i = 0 only."""
    rng = np.random.default_rng(52)
    for L in (1, 2):
        x1 = walk(rng, 3, L, s=0.3)
        x2 = walk(rng, 3, L, D=2, s=0.3)
        cases = [
            ({"op": "eventually", "smooth": True, "beta": 10.0, "child": S1, "mask": mask(3.0, 9.0, 1.0, 1e-6),
              "pad": "last"}, x1, mparams(3.0, 9.0)),
            ({"op": "always", "smooth": True, "beta": 10.0, "child": S1, "mask": mask(0.0, 4.0, 2.0, 1e-6),
              "pad": "const", "pad_value": -0.2}, x1, mparams(0.0, 4.0)),
            ({"op": "eventually", "smooth": "softmax", "beta": 4.0, "child": S1, "a": 0, "b": 5, "pad": "last"},
             x1, {}),
            (until((0.0, 3.0, 2.0, 1e-6)), x2, mparams(0.0, 3.0)),
            (until((-3.0, 0.4, 3.0, 1e-6)), x2, mparams(-3.0, 0.4)),
        ]
        for spec, x, params in cases:
            check_formula(spec, x, params=params, what="L=%d %s" % (L, spec["op"]))


def test_graph_replay_masked_until_and_pads():
    """A formula with a masked Until and a padded smooth mask captured in a
    HIP graph: every replay matches the eager calls (to the rounding of the
    Until adjoint's cross-wave atomic sums), with eager work between replays."""
    import torch
    from paper_2501_04194_amd import stl
    rng = np.random.default_rng(53)
    x = walk(rng, 6, 500, D=2, s=0.08)
    spec = {"op": "and", "smooth": True, "beta": 5.0, "children": [
        {"op": "until", "smooth": True, "beta": 8.0, "left": PHI, "right": PSI,
         "mask": {"a": "ua", "b": "ub", "c": 1.0, "eps": 1e-6}},
        {"op": "always", "smooth": True, "beta": 8.0, "child": PSI, "pad": "last",
         "mask": {"a": "wa", "b": "wb", "c": 0.7, "eps": 1e-6}}]}
    g = Gpu(spec, 2, {"ua": 10.2, "ub": 70.9, "wa": 300.1, "wb": 525.6})
    xt = torch.from_numpy(x).cuda()
    G = torch.randn(x.shape[:2], device="cuda")
    r_e = g.plan.forward(xt, g.pv)
    d_e, p_e = g.plan.backward(xt, G, g.pv)
    gr = stl.Graph(g.plan, xt, g.pv, G)
    for rep in range(3):
        gr.launch()
        torch.cuda.synchronize()
        assert torch.equal(gr.root.view_as(r_e), r_e)
        assert torch.allclose(gr.dx, d_e, rtol=1e-5, atol=1e-6 * float(d_e.abs().max()))
        assert torch.allclose(gr.gp, p_e, rtol=1e-5, atol=1e-6 * float(p_e.abs().max()))
        xt.add_(0.01)
        r_e = g.plan.forward(xt, g.pv)
        d_e, p_e = g.plan.backward(xt, G, g.pv)
        torch.cuda.synchronize()


def test_mask_pads_ragged():
    """Pads on a smooth mask in a ragged batch: the tail past each trajectory's
    own end depends on its length (lengths 1, 37, 400, 0 and 901)."""
    rng = np.random.default_rng(54)
    off = np.array([0, 1, 38, 438, 438, 1339], dtype=np.int64)
    xp = walk(rng, 1, 1339, s=0.05)[0]
    for pad, kind in (("last", "eventually"), ("const", "always")):
        spec = {"op": kind, "smooth": True, "beta": 10.0, "child": S1, "mask": mask(20.0, 150.0, 1.0, 1e-6),
                "pad": pad, "pad_value": -0.1}
        check_formula(spec, xp, params=mparams(20.0, 150.0), offsets=off, T=901, what="ragged mask pad %s" % pad)
    spec = until((15.5, 90.5, 1.0, 1e-6))
    xp2 = walk(rng, 1, 1339, D=2, s=0.05)[0]
    check_formula(spec, xp2, params=mparams(15.5, 90.5), offsets=off, T=901, what="ragged masked until")


def test_saved_traces_with_a_padded_mask():
    """The saved-trace pair on the fused formula shape with a padded mask: the
    forward does not take the fused path, marks its saved rows invalid, and the
    backward recomputes, matching the plain pair bit for bit."""
    rng = np.random.default_rng(55)
    x = walk(rng, 4, 900, D=2, s=0.05)
    spec = {"op": "and", "smooth": True, "beta": 10.0, "children": [
        {"op": "eventually", "smooth": True, "beta": 10.0, "child": PHI, "pad": "const", "pad_value": 0.2,
         "mask": {"a": "ea", "b": "eb", "c": 1.0, "eps": 1e-6}},
        {"op": "always", "smooth": True, "beta": 10.0, "child": PSI,
         "mask": {"a": "la", "b": "lb", "c": 1.0, "eps": 1e-6}}]}
    g = Gpu(spec, 2, {"ea": 100.0, "eb": 400.0, "la": 50.0, "lb": 200.0})
    G = rng.normal(size=(4, 900)).astype(np.float32)
    r0 = g.fwd(x)
    d0, p0 = g.bwd(x, G)
    t = g.torch
    xd = t.from_numpy(x).cuda()
    sv = g.plan.saved_buffer(xd)
    sv.fill_(0xAB)
    r1 = g.plan.forward(xd, g.pv, saved=sv)
    d1, gp1 = g.plan.backward(xd, t.from_numpy(G).cuda(), g.pv, saved=sv)
    t.cuda.synchronize()
    assert np.array_equal(r0, r1.cpu().numpy())
    assert np.array_equal(d0, d1.cpu().numpy())
    p1 = g.plan.param_grads(gp1.cpu().numpy())
    for k in p0:
        assert p0[k] == p1[k], k


def test_empty_trajectory_mask_partials_with_poisoned_workspace():
    """An empty trajectory in a ragged batch writes zero mask-bound partials:
    the workspace is filled with huge values before the backward, so a
    partial left unwritten would show in d/da, d/db."""
    import torch
    rng = np.random.default_rng(56)
    off = np.array([0, 40, 40, 300], dtype=np.int64)
    xp = walk(rng, 1, 300, s=0.05)[0]
    spec = {"op": "eventually", "smooth": True, "beta": 10.0, "child": S1, "mask": mask(5.0, 30.0, 1.0, 1e-6)}
    params = mparams(5.0, 30.0)
    g = Gpu(spec, 1, params)
    g.fwd(xp, offsets=off, T=260)
    for ws in g.plan._ws.values():
        ws.fill_(0x7F)                      # every float reads 3.4e38
    torch.cuda.synchronize()
    G = rng.normal(size=300).astype(np.float32)
    dx, dp = g.bwd(xp, G, offsets=off, T=260)
    _, dp_ref = oracle.backward(spec, xp, G, params=params, offsets=off)
    _, dp_abs = oracle.backward(spec, xp, np.abs(G), params=params, offsets=off)
    for k in dp_ref:
        assert abs(dp[k] - dp_ref[k]) <= 1e-5 * abs(dp_abs[k]) + 1e-12, (k, dp[k], dp_ref[k])
