"""GPU parity of the warm-start kernels (BF16 MFMA matrix product, casts,
ReLU mask, column sums, MSE gradient, Adam, ascent step) against the FP64
oracle that rounds to BF16 at the same points, and the warm-start gain.

Tolerances: products accumulate in FP32 on the GPU and in FP64 in the
oracle, so a value that lands within FP32 rounding of a BF16 rounding tie may
round to the neighbouring BF16 value (one BF16 ulp, 2^-8 relative).  Tests
require FP32-level agreement (1e-5 of the scale) for at least 99% of the
elements and one-BF16-ulp agreement (2^-7 of the scale) for all of them.
"""
import numpy as np
import pytest

from oracle import mlp_oracle as MO

pytestmark = pytest.mark.gpu


def bits_to_f32(u16):
    return (np.asarray(u16).astype(np.uint16).astype(np.uint32) << 16).view(np.float32)


def to_bf16_dev(torch, a):
    from paper_2501_04194_amd import mlp as M
    x = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    y = torch.empty(x.shape, dtype=torch.int16, device="cuda")
    M.cast_bf16(x, y)
    return y


def close_mostly(got, ref, what, frac=0.99):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = max(1e-30, np.abs(ref).max())
    err = np.abs(got - ref)
    assert np.all(err <= 2.0 ** -7 * scale), "%s: max err %g (scale %g)" % (what, err.max(), scale)
    assert np.mean(err <= 1e-5 * scale) >= frac, "%s: only %.4f within 1e-5" % (what, np.mean(err <= 1e-5 * scale))


def test_cast_bf16_round_to_nearest_even():
    import torch
    x = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, np.pi, -2.5, 0.0, 1e-30, 3.3e38], dtype=np.float32)
    r = bits_to_f32(to_bf16_dev(torch, x).cpu().numpy())
    assert np.array_equal(r, MO.bf16(x.astype(np.float64)).astype(np.float32))
    y = np.random.default_rng(0).normal(size=100_000).astype(np.float32) * 10
    r = bits_to_f32(to_bf16_dev(torch, y).cpu().numpy())
    assert np.array_equal(r, MO.bf16(y.astype(np.float64)).astype(np.float32))


@pytest.mark.parametrize("shape", [(1, 1, 1), (70, 33, 4), (64, 64, 16), (129, 200, 300), (1000, 400, 256),
                                   (5, 7, 0)])
def test_bf16_gemm_against_float64(shape):
    import torch
    from paper_2501_04194_amd import mlp as M
    Mm, N, K = shape
    rng = np.random.default_rng(sum(shape))
    A = MO.bf16(rng.normal(size=(Mm, K)))
    B = MO.bf16(rng.normal(size=(K, N)))
    bias = rng.normal(size=N).astype(np.float32)
    ref = A @ B + bias
    for transA in (False, True):
        Ad = to_bf16_dev(torch, A.T if transA else A)
        Bd = to_bf16_dev(torch, B)
        sam, sak = (1, Mm) if transA else (K, 1)
        c32 = torch.zeros((Mm, N), dtype=torch.float32, device="cuda")
        c16 = torch.zeros((Mm, N), dtype=torch.int16, device="cuda")
        M.gemm(Ad, Bd, Mm, N, K, sam, sak, N, 1, bias=torch.from_numpy(bias).cuda(), c32=c32, ldc32=N, c16=c16,
               ldc16=N)
        torch.cuda.synchronize()
        got = c32.cpu().numpy()
        scale = np.abs(A) @ np.abs(B) + np.abs(bias)
        assert np.all(np.abs(got - ref) <= 1e-6 * (scale + 1)), shape
        g16 = bits_to_f32(c16.cpu().numpy())
        assert np.all(np.abs(g16 - MO.bf16(got)) == 0)          # epilogue rounding of the FP32 result
    # ReLU epilogue and accumulation into C
    c32 = torch.ones((Mm, N), dtype=torch.float32, device="cuda")
    M.gemm(to_bf16_dev(torch, A), to_bf16_dev(torch, B), Mm, N, K, K, 1, N, 1, relu=True, c32=c32, ldc32=N, beta=True)
    torch.cuda.synchronize()
    np.testing.assert_allclose(c32.cpu().numpy(), 1 + np.maximum(A @ B, 0), rtol=1e-5, atol=1e-5)


def test_mlp_forward_backward_adam_vs_oracle():
    import torch
    from paper_2501_04194_amd import mlp as M
    rng = np.random.default_rng(5)
    sizes = [4, 48, 40, 30]
    W = [(rng.normal(size=(sizes[l + 1], sizes[l])) / np.sqrt(sizes[l]), rng.normal(size=sizes[l + 1]) * 0.1)
         for l in range(3)]
    net = M.BF16MLP(sizes, torch.device("cuda:0"), weights=W)
    X = rng.normal(size=(150, 4)).astype(np.float32)
    Y = rng.normal(size=(150, 30)).astype(np.float32)
    out = net.forward(torch.from_numpy(X).cuda(), keep=True)
    Wn = net.numpy_weights()
    ref, acts = MO.forward(X.astype(np.float64), Wn)
    close_mostly(out.cpu().numpy(), ref, "forward")
    g = torch.empty_like(out)
    loss = torch.zeros(1, device="cuda")
    M.mse_grad(out, torch.from_numpy(Y).cuda(), g, loss)
    lref, gref = MO.mse(out.cpu().numpy().astype(np.float64), Y)
    assert float(loss) == pytest.approx(lref, rel=1e-5)
    np.testing.assert_allclose(g.cpu().numpy(), gref, rtol=1e-5, atol=1e-9)
    dW, db = net.backward(g)
    # oracle backward on the GPU's own forward activations and gradient
    acts_gpu = [bits_to_f32(a.cpu().numpy()).astype(np.float64) for a in net._acts]
    dWr, dbr = MO.backward(g.cpu().numpy().astype(np.float64), Wn, acts_gpu)
    for l in range(3):
        close_mostly(dW[l].cpu().numpy(), dWr[l], "dW%d" % l)
        close_mostly(db[l].cpu().numpy(), dbr[l], "db%d" % l)
    w0 = net.W[1].cpu().numpy().astype(np.float64)
    net.adam(dW, db, lr=1e-2)
    w1, _, _ = MO.adam(w0, dW[1].cpu().numpy().astype(np.float64), np.zeros_like(w0), np.zeros_like(w0), 1, lr=1e-2)
    np.testing.assert_allclose(net.W[1].cpu().numpy(), w1, rtol=1e-6, atol=1e-6)
    assert np.array_equal(bits_to_f32(net.W16[1].cpu().numpy()), MO.bf16(net.W[1].cpu().numpy()).astype(np.float32))


def test_ascent_update_and_colsum():
    import torch
    from paper_2501_04194_amd import mlp as M
    rng = np.random.default_rng(6)
    x = rng.normal(size=(5, 7, 4)).astype(np.float32)
    dx = rng.normal(size=(5, 7, 4)).astype(np.float32)
    act = np.array([1, 0, 1, 1, 0], dtype=np.int32)
    xd = torch.from_numpy(x).cuda()
    M.ascent_update(xd, torch.from_numpy(dx).cuda(), torch.from_numpy(act).cuda(), 0.25, t0=1, d_upd=2)
    ref = x.copy()
    for n in range(5):
        if act[n]:
            ref[n, 1:, :2] += np.float32(0.25) * dx[n, 1:, :2]
    assert np.array_equal(xd.cpu().numpy(), ref)
    a = rng.normal(size=(33, 17)).astype(np.float32)
    out = torch.empty(17, device="cuda")
    M.colsum(torch.from_numpy(a).cuda(), 33, 17, 17, out)
    np.testing.assert_allclose(out.cpu().numpy(), a.astype(np.float64).sum(0), rtol=1e-5, atol=1e-5)


def test_warmstart_gain():
    """At the configuration's size (50,000 training problems, 1,000 held out):
    on held-out problems the learned proposal needs fewer ascent steps
    (median) than plain ascent from the straight line, solves at least as
    many problems, and reaches the number plain ascent solves within its step
    budget in less wall time (MLP inference included)."""
    from paper_2501_04194_amd import warmstart as WS
    res = WS.experiment(n_train=50_000, n_test=1000, epochs=30, log=print)
    print(res)
    assert res["learned"]["median_steps"] < res["plain"]["median_steps"]
    assert res["learned"]["s_to_plain_solved"] < res["plain"]["s_to_plain_solved"]
    assert res["learned"]["solved_frac"] >= res["plain"]["solved_frac"] - 0.02
