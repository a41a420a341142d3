"""BF16 multilayer perceptron trained and run with the library's own kernels
(include/stlmi_mlp.h): every matrix product is stl_bf16_gemm (MFMA, FP32
accumulation), the optimiser is stl_adam_step on FP32 master weights.
PyTorch only allocates the device buffers.

Layer l maps h_{l-1} [N, I] to h_l = act(h_{l-1} W_l^T + b_l) with W_l
[O, I] row-major; hidden activations are kept in BF16, the output in FP32.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import stl

_c = None


def _lib():
    global _c
    if _c is not None:
        return _c
    L = stl.lib()
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.stl_bf16_gemm.argtypes = [vp, i64, i64, vp, i64, i64, i32, i32, i32, vp, i32, vp, i64, i32, vp, i64, vp]
    L.stl_cast_bf16.argtypes = [vp, vp, i64, vp]
    L.stl_relu_grad_bf16.argtypes = [vp, vp, vp, i64, vp]
    L.stl_colsum.argtypes = [vp, i32, i32, i64, vp, vp]
    L.stl_mse_grad.argtypes = [vp, vp, vp, vp, i64, vp]
    L.stl_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, vp]
    L.stl_ascent_update.argtypes = [vp, vp, vp, i64, i32, i32, i32, i32, f32, vp]
    for f in ("stl_bf16_gemm", "stl_cast_bf16", "stl_relu_grad_bf16", "stl_colsum", "stl_mse_grad",
              "stl_adam_step", "stl_ascent_update"):
        getattr(L, f).restype = ctypes.c_int
    _c = L
    return L


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _s(torch, dev):
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def gemm(A, B, M, N, K, sam, sak, sbk, sbn, bias=None, relu=False, c32=None, ldc32=0, beta=False, c16=None,
         ldc16=0):
    import torch
    stl._check(_lib().stl_bf16_gemm(_p(A), sam, sak, _p(B), sbk, sbn, M, N, K, _p(bias), int(relu), _p(c32), ldc32,
                                    int(beta), _p(c16), ldc16, _s(torch, A.device)))


def cast_bf16(x, y):
    import torch
    stl._check(_lib().stl_cast_bf16(_p(x), _p(y), x.numel(), _s(torch, x.device)))


def relu_grad_bf16(g, h, g16):
    import torch
    stl._check(_lib().stl_relu_grad_bf16(_p(g), _p(h), _p(g16), g.numel(), _s(torch, g.device)))


def colsum(x, rows, cols, ld, out):
    import torch
    stl._check(_lib().stl_colsum(_p(x), rows, cols, ld, _p(out), _s(torch, x.device)))


def mse_grad(y, t, g, loss):
    import torch
    stl._check(_lib().stl_mse_grad(_p(y), _p(t), _p(g), _p(loss), y.numel(), _s(torch, y.device)))


def adam_step(w, g, m, v, w16, lr, b1, b2, eps, step):
    import torch
    stl._check(_lib().stl_adam_step(_p(w), _p(g), _p(m), _p(v), _p(w16), w.numel(), lr, b1, b2, eps, step,
                                    _s(torch, w.device)))


def ascent_update(x, dx, active, lr, t0=1, d_upd=2):
    import torch
    N, T, D = x.shape
    stl._check(_lib().stl_ascent_update(_p(x), _p(dx), _p(active), N, T, D, t0, d_upd, lr, _s(torch, x.device)))


class BF16MLP:
    """MLP with FP32 master weights, BF16 compute copies and Adam state."""

    def __init__(self, sizes, device, seed=0, weights=None):
        import torch
        self.sizes = list(sizes)
        self.dev = device
        rng = np.random.default_rng(seed)
        self.W, self.b = [], []
        for l in range(len(sizes) - 1):
            I, O = sizes[l], sizes[l + 1]
            if weights is not None:
                w, b = weights[l]
            else:
                lim = np.sqrt(6.0 / (I + O))                      # Glorot-uniform initialisation
                w = rng.uniform(-lim, lim, size=(O, I))
                b = np.zeros(O)
            self.W.append(torch.tensor(np.asarray(w, np.float32), device=device))
            self.b.append(torch.tensor(np.asarray(b, np.float32), device=device))
        self.W16 = [torch.empty(w.shape, dtype=torch.int16, device=device) for w in self.W]
        for w, w16 in zip(self.W, self.W16):
            cast_bf16(w, w16)
        self.mW = [torch.zeros_like(w) for w in self.W]
        self.vW = [torch.zeros_like(w) for w in self.W]
        self.mb = [torch.zeros_like(b) for b in self.b]
        self.vb = [torch.zeros_like(b) for b in self.b]
        self.step_count = 0

    @property
    def n_layers(self):
        return len(self.W)

    def forward(self, X, keep=False):
        """X [N, sizes[0]] float32 -> [N, sizes[-1]] float32 (activations kept for backward)."""
        import torch
        N = X.shape[0]
        h16 = torch.empty((N, self.sizes[0]), dtype=torch.int16, device=self.dev)
        cast_bf16(X.contiguous(), h16)
        acts = [h16]
        out = None
        for l in range(self.n_layers):
            I, O = self.sizes[l], self.sizes[l + 1]
            last = l == self.n_layers - 1
            if last:
                out = torch.empty((N, O), dtype=torch.float32, device=self.dev)
                gemm(acts[-1], self.W16[l], N, O, I, I, 1, 1, I, bias=self.b[l], c32=out, ldc32=O)
            else:
                hn = torch.empty((N, O), dtype=torch.int16, device=self.dev)
                gemm(acts[-1], self.W16[l], N, O, I, I, 1, 1, I, bias=self.b[l], relu=True, c16=hn, ldc16=O)
                acts.append(hn)
        if keep:
            self._acts = acts
        return out

    def backward(self, dOut):
        """Gradients (dW, db) of the loss, dOut = d loss / d out [N, O_last] (FP32).

        Per layer, from the last: the gradient with respect to the
        pre-activation is rounded to BF16 (after the ReLU mask of a hidden
        layer); dW = g^T h_in and db = column sums of g (both FP32), and the
        gradient passed down is g W (FP32)."""
        import torch
        acts = self._acts
        N = dOut.shape[0]
        dW = [None] * self.n_layers
        db = [None] * self.n_layers
        g32 = dOut.contiguous()
        for l in range(self.n_layers - 1, -1, -1):
            I, O = self.sizes[l], self.sizes[l + 1]
            g16 = torch.empty((N, O), dtype=torch.int16, device=self.dev)
            relu_grad_bf16(g32, None if l == self.n_layers - 1 else acts[l + 1], g16)
            dW[l] = torch.empty((O, I), dtype=torch.float32, device=self.dev)
            gemm(g16, acts[l], O, I, N, 1, O, I, 1, c32=dW[l], ldc32=I)          # g^T [O,N] h [N,I]
            db[l] = torch.empty(O, dtype=torch.float32, device=self.dev)
            # widen the BF16 gradient exactly (product with the identity) and sum its rows
            wide = torch.empty((N, O), dtype=torch.float32, device=self.dev)
            gemm(g16, self._eye16(O), N, O, O, O, 1, O, 1, c32=wide, ldc32=O)
            colsum(wide, N, O, O, db[l])
            if l > 0:
                g32 = torch.empty((N, I), dtype=torch.float32, device=self.dev)
                gemm(g16, self.W16[l], N, I, O, O, 1, I, 1, c32=g32, ldc32=I)   # g [N,O] W [O,I]
        return dW, db

    def _eye16(self, n):
        import torch
        if not hasattr(self, "_eyes"):
            self._eyes = {}
        if n not in self._eyes:
            e = torch.eye(n, dtype=torch.float32, device=self.dev)
            e16 = torch.empty((n, n), dtype=torch.int16, device=self.dev)
            cast_bf16(e, e16)
            self._eyes[n] = e16
        return self._eyes[n]

    def adam(self, dW, db, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        for l in range(self.n_layers):
            adam_step(self.W[l], dW[l], self.mW[l], self.vW[l], self.W16[l], lr, b1, b2, eps, self.step_count)
            adam_step(self.b[l], db[l], self.mb[l], self.vb[l], None, lr, b1, b2, eps, self.step_count)

    def numpy_weights(self):
        return [(w.cpu().numpy().astype(np.float64), b.cpu().numpy().astype(np.float64))
                for w, b in zip(self.W, self.b)]
