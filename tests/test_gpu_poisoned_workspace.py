"""Every operator family with the workspace filled with 3.4e38 (bytes 0x7F)
before the calls: results must not depend on what the workspace held, so a
value the kernels read without writing it first shows up against the FP64
oracle."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import Gpu, assert_close, f32params
from paper_2501_04194_amd import workloads as W

pytestmark = pytest.mark.gpu

S1 = {"op": "linear", "w": [1.0], "c": 0.0}
P0 = {"op": "linear", "w": [1.0, 0.0], "c": -0.5}
P1 = {"op": "linear", "w": [0.0, 1.0], "c": 0.1}


def _m(a, b, c=1.0, eps=1e-6):
    return {"a": a, "b": b, "c": c, "eps": eps}


CASES = [
    ("hard windows", {"op": "and", "children": [{"op": "always", "a": 3, "b": 40, "child": P0, "pad": "last"},
                                                {"op": "eventually", "a": 0, "b": None, "child": P1}]}, {}, 2),
    ("smooth windows", {"op": "or", "smooth": True, "beta": 8.0, "children": [
        {"op": "always", "a": 3, "b": 40, "smooth": True, "beta": 8.0, "child": P0, "pad": "const",
         "pad_value": 0.3},
        {"op": "eventually", "a": 5, "b": None, "smooth": True, "beta": 8.0, "child": P1}]}, {}, 2),
    ("softmax", {"op": "and", "smooth": "softmax", "beta": 4.0, "children": [
        {"op": "eventually", "a": 0, "b": 9, "smooth": "softmax", "beta": 4.0, "child": P0, "pad": "last"}, P1]},
     {}, 2),
    ("until", {"op": "until", "a": 4, "b": 90, "smooth": True, "beta": 10.0, "left": P0, "right": P1}, {}, 2),
    ("masked windows", W.cfg2_formula(), {"ev_a": 20.3, "ev_b": 90.7, "ev_c": 1.0, "ev_eps": 1e-6,
                                          "al_a": 10.2, "al_b": 60.1, "al_c": 0.7, "al_eps": 1e-6}, 2),
    ("masked window pads", {"op": "always", "smooth": True, "beta": 10.0, "child": P0, "pad": "last",
                            "mask": {"a": "a", "b": "b", "c": 1.0, "eps": 1e-6}}, {"a": 200.0, "b": 330.0}, 2),
    ("masked until", {"op": "until", "smooth": True, "beta": 10.0, "left": P0, "right": P1,
                      "mask": {"a": "a", "b": "b", "c": 1.0, "eps": 1e-6}}, {"a": 6.3, "b": 70.2}, 2),
]


def _poison(g):
    for ws in g.plan._ws.values():
        ws.fill_(0x7F)
    torch.cuda.synchronize()


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("ragged", [False, True])
def test_poisoned_workspace(case, ragged):
    name, spec, params, D = case
    rng = np.random.default_rng(60)
    params = f32params(params)
    if ragged:
        off = np.array([0, 3, 3, 250, 610], dtype=np.int64)
        x = np.cumsum(rng.normal(size=(610, D)) * 0.08, axis=0).astype(np.float32)
        kw = dict(offsets=off, T=360)
    else:
        x = np.cumsum(rng.normal(size=(3, 400, D)) * 0.08, axis=1).astype(np.float32)
        kw = {}
    g = Gpu(spec, D, params)
    g.fwd(x, **kw)
    _poison(g)
    root = g.fwd(x, **kw)
    ref = oracle.forward(spec, x, params=params, offsets=kw.get("offsets"))
    assert_close(root, ref, what=name + " root")
    G = rng.normal(size=root.shape).astype(np.float32)
    _poison(g)
    dx, dp = g.bwd(x, G, **kw)
    dxr, dpr = oracle.backward(spec, x, G, params=params, offsets=kw.get("offsets"))
    dxa, dpa = oracle.backward(spec, x, np.abs(G), params=params, offsets=kw.get("offsets"))
    assert_close(dx, dxr, scale=max(1e-30, np.abs(dxr).max()), what=name + " dx", elem_scale=dxa)
    for k, v in dpr.items():
        assert abs(dp[k] - v) <= 1e-5 * abs(dpa[k]) + 1e-12, (name, k, dp[k], v)
