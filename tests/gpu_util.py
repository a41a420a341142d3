"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded float32 inputs, and compare them.

Tolerances (written here, used by every parity test):
  * hard min/max selections: bit-exact on identical float32 inputs;
  * predicates and smooth operators: |g - r| <= 1e-5 |r| + 1e-5 S with
    S = max(1, max |r|) over the compared non-sentinel trace values;
  * d/dx: the same form with S_j = max(max |dx_ref|, |dx_abs_j|), dx_abs the
    oracle's backward on |G|: each element is a signed sum over timesteps
    whose float32 terms carry relative errors of order |z| 2^-24 (z the
    exponent of the term), so its error scales with the sum of the absolute
    terms, not with the (possibly cancelled) result;
  * d/da, d/db (sums over every timestep of the batch):
    |g - r| <= 1e-5 * sum |per-timestep terms| (the oracle's backward on |G|).
Sentinels: a reference value equal to +-1e6 (the empty-window value +-rho_pad,
or TRUE's rho_max) must match bit for bit.  Other values of sentinel
magnitude (|r| >= 1e5: what a smooth operator derives from sentinels, e.g. a
logsumexp over several of them, 1e6 +- log(K)/beta) compare at 1e-5 of their
own magnitude, and are left out of S (which would otherwise loosen the bound
of the ordinary values to 10).  A test whose smooth operators take sentinels
as operands (a logsumexp in which a sentinel dominates, so that the exact
result rounds to 1e6 in fp64) passes exact_sentinels=False: in float32 such
a value is 1e6 only to within a few units of its last place (0.0625), as the
float32 exponent beta log2(e) 1e6 = 1.4e7 carries a rounding of up to half a
unit.
"""
import numpy as np

import oracle
from paper_2501_04194_amd import stl

REL = 1e-5


def torch_mod():
    import torch
    return torch


def f32params(params):
    return {k: float(np.float32(v)) for k, v in (params or {}).items()}


SENTINEL = 1e6     # rho_pad and rho_max


def assert_close(got, ref, rel=REL, scale=None, what="", elem_scale=None, exact_sentinels=True):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    near = np.abs(ref) >= 1e5
    if near.any():
        exact = near & (np.abs(ref) == SENTINEL) if exact_sentinels else np.zeros_like(near)
        if exact.any():
            bad = got[exact] != ref[exact]
            assert not bad.any(), "%s: %d sentinel values not exact (got %r, ref %r)" % (
                what, bad.sum(), got[exact][bad][:4], ref[exact][bad][:4])
        rest = near & ~exact
        if rest.any():
            e = np.abs(got[rest] - ref[rest])
            assert np.all(np.sign(got[rest]) == np.sign(ref[rest])), "%s: sentinel sign mismatch" % what
            assert np.all(e <= rel * np.abs(ref[rest])), "%s: sentinel-scale mismatch (worst %g)" % (what, e.max())
    nz = ~near
    if not nz.any():
        return
    S = max(1.0, float(np.abs(ref[nz]).max())) if scale is None else max(float(scale), 1e-30)
    err = np.abs(got[nz] - ref[nz])
    if elem_scale is not None:
        S = np.maximum(S, np.abs(np.asarray(elem_scale, dtype=np.float64))[nz])
    bound = rel * np.abs(ref[nz]) + rel * S
    bad = err > bound
    if bad.any():
        i = np.argmax(err - bound)
        raise AssertionError("%s: %d/%d outside tolerance; worst got=%r ref=%r (S=%g)"
                             % (what, bad.sum(), bad.size, got[nz][i], ref[nz][i], np.broadcast_to(S, err.shape)[i]))


class Gpu:
    """Runs a formula on the GPU through the binding of the C ABI."""

    def __init__(self, spec, D, params=None, launch=None):
        self.torch = torch_mod()
        self.params = f32params(params)
        self.plan = stl.Plan(spec, D, self.params)
        self.pv = self.torch.from_numpy(self.plan.param_vector()).cuda()
        self.launch = launch

    def fwd(self, x, offsets=None, T=None, order=None, traces=False):
        t = self.torch
        xd = t.from_numpy(np.ascontiguousarray(x)).cuda()
        od = None if offsets is None else t.from_numpy(np.asarray(offsets, np.int64)).cuda()
        ordd = None if order is None else t.from_numpy(np.asarray(order, np.int32)).cuda()
        r = self.plan.forward(xd, self.pv, offsets=od, order=ordd, T=T, node_traces=traces, launch=self.launch)
        t.cuda.synchronize()
        if traces:
            return r[0].cpu().numpy(), r[1].cpu().numpy()
        return r.cpu().numpy()

    def bwd(self, x, G, offsets=None, T=None, order=None):
        t = self.torch
        xd = t.from_numpy(np.ascontiguousarray(x)).cuda()
        Gd = t.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).cuda()
        od = None if offsets is None else t.from_numpy(np.asarray(offsets, np.int64)).cuda()
        ordd = None if order is None else t.from_numpy(np.asarray(order, np.int32)).cuda()
        dx, gp = self.plan.backward(xd, Gd, self.pv, offsets=od, order=ordd, T=T, launch=self.launch)
        t.cuda.synchronize()
        return dx.cpu().numpy(), self.plan.param_grads(gp.cpu().numpy())


def check_formula(spec, x, params=None, G=None, grads=True, bitexact_root=False, launch=None, what="",
                  offsets=None, T=None, exact_sentinels=True):
    """Forward (and backward) parity of one formula on one batch."""
    params = f32params(params)
    g = Gpu(spec, x.shape[-1], params, launch)
    root = g.fwd(x, offsets=offsets, T=T)
    ref = oracle.forward(spec, x, params=params, offsets=offsets)
    if bitexact_root:
        assert np.array_equal(root.astype(np.float32), ref.astype(np.float32)), what + ": root not bit-exact"
    else:
        assert_close(root, ref, what=what + " root", exact_sentinels=exact_sentinels)
    if not grads:
        return g
    if G is None:
        G = np.random.default_rng(99).normal(size=root.shape).astype(np.float32)
    dx, dp = g.bwd(x, G, offsets=offsets, T=T)
    dx_ref, dp_ref = oracle.backward(spec, x, G, params=params, offsets=offsets)
    dx_abs, dp_abs = oracle.backward(spec, x, np.abs(G), params=params, offsets=offsets)
    assert_close(dx, dx_ref, scale=max(1e-30, np.abs(dx_ref).max()), what=what + " dx", elem_scale=dx_abs)
    if dp_ref:
        for k, v in dp_ref.items():
            tol = REL * abs(dp_abs[k]) + 1e-12
            assert abs(dp[k] - v) <= tol, "%s d/d%s: got %r ref %r tol %g" % (what, k, dp[k], v, tol)
    return g
