"""Pins of the warm-start network oracle (CPU)."""
import numpy as np
import pytest

from oracle import mlp_oracle as MO


def test_bf16_rounding_closed_forms():
    # 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 -> even (1)
    assert MO.bf16(1 + 2.0 ** -8) == 1.0
    assert MO.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6          # tie -> even mantissa
    assert MO.bf16(1 + 2.0 ** -8 + 2.0 ** -20) == 1 + 2.0 ** -7  # above the tie
    assert MO.bf16(-3.0) == -3.0 and MO.bf16(0.0) == 0.0
    assert MO.bf16(np.pi) == 3.140625                          # 0b11.0010010 (8 bits)
    x = np.random.default_rng(0).normal(size=1000)
    r = MO.bf16(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)      # half an ulp of 8 bits
    assert np.array_equal(MO.bf16(r), r)                       # idempotent


def test_forward_equals_plain_matmul_on_bf16_operands():
    rng = np.random.default_rng(1)
    W = [(MO.bf16(rng.normal(size=(16, 4))), rng.normal(size=16)),
         (MO.bf16(rng.normal(size=(5, 16))), rng.normal(size=5))]
    X = MO.bf16(rng.normal(size=(7, 4)))
    out, acts = MO.forward(X, W)
    h = MO.bf16(np.maximum(X @ W[0][0].T + W[0][1], 0))
    assert np.array_equal(acts[1], h)
    np.testing.assert_allclose(out, h @ W[1][0].T + W[1][1], rtol=1e-14, atol=1e-14)


def test_backward_matches_finite_differences_without_rounding():
    rng = np.random.default_rng(2)
    W = [(rng.normal(size=(8, 4)) * 0.5, rng.normal(size=8) * 0.1),
         (rng.normal(size=(6, 8)) * 0.5, rng.normal(size=6) * 0.1),
         (rng.normal(size=(3, 6)) * 0.5, rng.normal(size=3) * 0.1)]
    X = rng.normal(size=(5, 4))
    T = rng.normal(size=(5, 3))
    out, acts = MO.forward(X, W, rounding=False)
    loss, dOut = MO.mse(out, T)
    dW, db = MO.backward(dOut, W, acts, rounding=False)
    h = 1e-6
    for l in range(3):
        for idx in [(0, 0), (1, 2), (2, 1)]:
            Wp = [(w.copy(), b.copy()) for w, b in W]
            Wm = [(w.copy(), b.copy()) for w, b in W]
            Wp[l][0][idx] += h
            Wm[l][0][idx] -= h
            fd = (MO.mse(MO.forward(X, Wp, False)[0], T)[0] - MO.mse(MO.forward(X, Wm, False)[0], T)[0]) / (2 * h)
            assert dW[l][idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)
        Wp = [(w.copy(), b.copy()) for w, b in W]
        Wm = [(w.copy(), b.copy()) for w, b in W]
        Wp[l][1][1] += h
        Wm[l][1][1] -= h
        fd = (MO.mse(MO.forward(X, Wp, False)[0], T)[0] - MO.mse(MO.forward(X, Wm, False)[0], T)[0]) / (2 * h)
        assert db[l][1] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    # with bias correction the first step is lr * g / (|g| + eps)
    w, m, v = MO.adam(np.array([1.0, 2.0]), np.array([0.5, -3.0]), np.zeros(2), np.zeros(2), 1, lr=0.1)
    np.testing.assert_allclose(w, [1.0 - 0.1, 2.0 + 0.1], rtol=1e-7)
