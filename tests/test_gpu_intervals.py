"""GPU parity of the interval sweep (``stl_interval_sweep``: the robustness at
t = 0 of one masked Always / Eventually for many (a, b) values, Sec. VI)
against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_close
from paper_2501_04194_amd import stl

pytestmark = pytest.mark.gpu

RHO_PAD = 1e6


def walk(rng, B, T, D=1, s=0.3):
    return np.cumsum(rng.normal(size=(B, T, D)) * s, axis=1).astype(np.float32)


def run(x, a, b, w, **kw):
    xd = torch.from_numpy(x).cuda()
    ad = torch.from_numpy(np.asarray(a, dtype=np.float32)).cuda()
    bd = torch.from_numpy(np.asarray(b, dtype=np.float32)).cuda()
    rho, ga, gb = stl.interval_sweep(xd, ad, bd, w, **kw)
    return rho.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()


def intervals(rng, N, T):
    a = rng.uniform(-8.0, T + 4.0, size=N).astype(np.float32)
    b = (a + rng.uniform(-2.0, T, size=N)).astype(np.float32)
    return a, b


@pytest.mark.parametrize("T", [20, 100, 333])
@pytest.mark.parametrize("op", ["always", "eventually"])
def test_interval_sweep_smooth(T, op):
    rng = np.random.default_rng(T)
    x = walk(rng, 3, T, D=2)
    a, b = intervals(rng, 300 if T == 20 else 90, T)
    kw = dict(c=0.1, op=op, smooth=True, beta=10.0, mask_c=1.5, mask_eps=1e-6)
    rho, ga, gb = run(x, a, b, [1.0, -0.5], **kw)
    r0, ga0, gb0 = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0, -0.5], **kw)
    assert_close(rho, r0, what="sweep rho %s T=%d" % (op, T))
    # d/da, d/db: |d rho/da| <= c/(4 beta) * (sum of |dw| E)/S; compare against that scale
    sc = 1.5 / (4 * 10.0)
    assert_close(ga, ga0, scale=sc, what="sweep d/da")
    assert_close(gb, gb0, scale=sc, what="sweep d/db")


@pytest.mark.parametrize("op", ["always", "eventually"])
def test_interval_sweep_hard_bitexact(op):
    rng = np.random.default_rng(4)
    x = walk(rng, 2, 64)
    # half-integer bounds and a steep mask: the support is an integer window
    k = rng.integers(-3, 70, size=200)
    m = k + rng.integers(-2, 40, size=200)
    a, b = (k - 0.5).astype(np.float32), (m + 0.5).astype(np.float32)
    kw = dict(op=op, smooth=False, mask_c=50.0, mask_eps=1e-6)
    rho, ga, gb = run(x, a, b, [1.0], **kw)
    r0, _, _ = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0], **kw)
    assert np.array_equal(rho.astype(np.float32), r0.astype(np.float32))
    assert not ga.any() and not gb.any()


def test_interval_sweep_trajectory_groups():
    """Batches that span several work-group trajectory groups, with a group
    size cut by the LDS capacity (T = 700: five trajectories per group)."""
    rng = np.random.default_rng(8)
    x = walk(rng, 11, 700, s=0.1)
    a, b = intervals(rng, 40, 700)
    kw = dict(op="eventually", smooth=True, beta=10.0, mask_c=0.5, mask_eps=1e-6)
    rho, ga, gb = run(x, a, b, [1.0], **kw)
    r0, ga0, gb0 = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0], **kw)
    assert_close(rho, r0, what="grouped sweep rho")
    assert_close(ga, ga0, scale=0.5 / 40, what="grouped sweep d/da")
    assert_close(gb, gb0, scale=0.5 / 40, what="grouped sweep d/db")


def test_interval_sweep_edges():
    rng = np.random.default_rng(5)
    x = walk(rng, 2, 1)
    # T = 1, intervals covering, missing and reversed
    a = np.array([-1.0, 0.0, 12.0, 3.0], dtype=np.float32)
    b = np.array([2.0, 0.5, 16.0, -3.0], dtype=np.float32)
    kw = dict(op="eventually", smooth=True, beta=10.0, mask_c=2.0, mask_eps=1e-6)
    rho, _, _ = run(x, a, b, [1.0], **kw)
    r0, _, _ = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0], **kw)
    assert_close(rho, r0, what="T=1 sweep")
    assert rho[0, 2] == -RHO_PAD and rho[0, 3] == -RHO_PAD
    # N not a multiple of the work-group size, eps = 0 (every offset in the support)
    x = walk(rng, 2, 50)
    a, b = intervals(rng, 257, 50)
    kw = dict(op="always", smooth=True, beta=3.0, mask_c=0.7, mask_eps=0.0)
    rho, ga, gb = run(x, a, b, [1.0], **kw)
    r0, ga0, gb0 = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0], **kw)
    assert_close(rho, r0, what="eps=0 sweep")
    assert_close(ga, ga0, scale=0.7 / 12, what="eps=0 d/da")
    # empty batch / no intervals, and argument errors
    xd = torch.from_numpy(x).cuda()
    e = torch.zeros(0, dtype=torch.float32, device="cuda")
    assert stl.interval_sweep(xd, e, e, [1.0])[0].shape == (2, 0)
    one = torch.ones(3, dtype=torch.float32, device="cuda")
    with pytest.raises(stl.StlError, match="mask_c"):
        stl.interval_sweep(xd, one, one, [1.0], mask_c=0.0)
    with pytest.raises(stl.StlError, match="T must be"):
        stl.interval_sweep(torch.zeros((1, 5000, 1), device="cuda"), one, one, [1.0])


@pytest.mark.parametrize("T,B,N", [(20, 37, 500), (17, 16, 300), (32, 21, 200), (61, 18, 150)])
@pytest.mark.parametrize("op", ["always", "eventually"])
def test_interval_sweep_batched_matrix_cores(T, B, N, op):
    """Batches of 16 or more trajectories with T <= 64 take the matrix-core
    path (16 x 16 tiles of trajectories x intervals): ragged tiles on both
    sides, T not a multiple of 4, every K-step count."""
    rng = np.random.default_rng(100 + T)
    x = walk(rng, B, T, D=2, s=0.2)
    a, b = intervals(rng, N, T)
    kw = dict(c=0.1, op=op, smooth=True, beta=10.0, mask_c=1.5, mask_eps=1e-6)
    rho, ga, gb = run(x, a, b, [1.0, -0.5], **kw)
    r0, ga0, gb0 = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0, -0.5], **kw)
    assert_close(rho, r0, what="batched sweep rho %s T=%d" % (op, T))
    sc = 1.5 / (4 * 10.0)
    assert_close(ga, ga0, scale=sc, what="batched sweep d/da")
    assert_close(gb, gb0, scale=sc, what="batched sweep d/db")


def test_interval_sweep_batched_range_fallback_and_eps0():
    """Traces whose exponent range exceeds fp32 against the trajectory's
    largest term: intervals whose support only sees terms far below it are
    redone against their own reference.  eps = 0 keeps every offset; it is
    checked on a trace of moderate range: the kernels' fp32 weights end near
    e^-87 (the oracle's fp64 ones near e^-745), and a weight past that point
    could only matter against a term more than e^87 above the others."""
    rng = np.random.default_rng(9)
    B, T = 20, 40
    for s, eps in ((2.0, 1e-6), (0.3, 0.0)):   # s = 2: beta log2(e) |du| reaches well past 126
        x = walk(rng, B, T, s=s)
        a, b = intervals(rng, 300, T)
        kw = dict(op="eventually", smooth=True, beta=10.0, mask_c=2.0, mask_eps=eps)
        rho, ga, gb = run(x, a, b, [1.0], **kw)
        r0, ga0, gb0 = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0], **kw)
        assert_close(rho, r0, what="range sweep rho eps=%g" % eps)
        assert_close(ga, ga0, scale=2.0 / 40, what="range sweep d/da")
        assert_close(gb, gb0, scale=2.0 / 40, what="range sweep d/db")


@pytest.mark.parametrize("B", [1, 3])
def test_interval_sweep_maximum_length(B):
    """T = 4096, the sweep's maximum: the whole trace's terms fill the LDS
    array of one work-group; intervals near both ends and past the end."""
    rng = np.random.default_rng(40 + B)
    x = walk(rng, B, 4096, s=0.05)
    a = np.array([0.0, 100.0, 1999.5, 3000.5, 4090.0, 4200.0, -50.0, 10.0, 2047.0, 4000.0, 512.0, 3500.0],
                 dtype=np.float32)
    b = np.array([5.0, 1500.0, 2010.5, 4200.0, 5000.0, 4300.0, 30.0, 4095.0, 2049.0, 4095.5, 1024.0, 3400.0],
                 dtype=np.float32)
    for op in ("eventually", "always"):
        kw = dict(op=op, smooth=True, beta=10.0, mask_c=1.0, mask_eps=1e-6)
        rho, ga, gb = run(x, a, b, [1.0], **kw)
        r0, ga0, gb0 = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), [1.0], **kw)
        assert_close(rho, r0, what="T=4096 sweep rho %s" % op)
        assert_close(ga, ga0, scale=1.0 / 40, what="T=4096 d/da")
        assert_close(gb, gb0, scale=1.0 / 40, what="T=4096 d/db")
    kw = dict(op="always", smooth=False, mask_c=50.0, mask_eps=1e-6)
    rho, _, _ = run(x, np.floor(a) - 0.5, np.floor(b) + 0.5, [1.0], **kw)
    r0, _, _ = oracle.interval_sweep(x, (np.floor(a) - 0.5).astype(np.float64), (np.floor(b) + 0.5).astype(np.float64),
                                     [1.0], **kw)
    assert np.array_equal(rho.astype(np.float32), r0.astype(np.float32))


def test_interval_sweep_batched_wide_state():
    """The matrix-core path with the widest state (D = 16): each lane's
    predicate reads 16 strided coefficients per offset."""
    rng = np.random.default_rng(12)
    B, T, D = 19, 24, 16
    x = walk(rng, B, T, D=D, s=0.05)
    w = list(rng.normal(size=D) * 0.3)
    a, b = intervals(rng, 130, T)
    kw = dict(c=-0.05, op="always", smooth=True, beta=10.0, mask_c=1.2, mask_eps=1e-6)
    rho, ga, gb = run(x, a, b, w, **kw)
    r0, ga0, gb0 = oracle.interval_sweep(x, a.astype(np.float64), b.astype(np.float64), w, **kw)
    assert_close(rho, r0, what="D=16 batched sweep rho")
    assert_close(ga, ga0, scale=1.2 / 40, what="D=16 d/da")
    assert_close(gb, gb0, scale=1.2 / 40, what="D=16 d/db")
