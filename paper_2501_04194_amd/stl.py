"""Python binding of the C ABI in ``include/stlmi.h`` (argument marshalling only).

Every operator runs in the HIP kernels of ``libstlmi.so``; this module turns a
formula description (see ``workloads.py`` for the format) into the library's
node array, owns the parameter-vector layout, allocates workspaces with the
PyTorch caching allocator and passes raw device pointers and the current HIP
stream to ``stl_compile`` / ``stl_forward`` / ``stl_backward``.  There is no
fallback: if the library or a GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstlmi.so")

STL_TRUE, STL_PRED_LINEAR, STL_PRED_NORM, STL_NOT, STL_AND, STL_OR, STL_EVENTUALLY, STL_ALWAYS, STL_UNTIL = range(9)
PADS = {"neutral": 0, "last": 1, "const": 2}
MAX_D = 16


class StlError(RuntimeError):
    pass


class Node(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("n_child", ctypes.c_int32), ("child_off", ctypes.c_int32),
                ("smooth", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32),
                ("mask_param", ctypes.c_int32), ("mask_unbounded", ctypes.c_int32),
                ("beta_param", ctypes.c_int32), ("pred", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("pad_value", ctypes.c_float)]


class Pred(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int32), ("w", ctypes.c_float * MAX_D),
                ("c", ctypes.c_float), ("A", ctypes.c_float * (4 * MAX_D)), ("p", ctypes.c_float * 4),
                ("r", ctypes.c_float), ("sign", ctypes.c_float)]


class Batch(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("B", ctypes.c_int64), ("T", ctypes.c_int64), ("D", ctypes.c_int32),
                ("pad0", ctypes.c_int32), ("offsets", ctypes.c_void_p), ("order", ctypes.c_void_p)]


class Launch(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32), ("global_slots", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class IntervalDesc(ctypes.Structure):
    """stl_interval_desc"""
    _fields_ = [("op", ctypes.c_int32), ("smooth", ctypes.c_int32), ("beta", ctypes.c_float),
                ("mask_c", ctypes.c_float), ("mask_eps", ctypes.c_float), ("D", ctypes.c_int32),
                ("w", ctypes.c_float * 16), ("c", ctypes.c_float), ("rho_pad", ctypes.c_float)]


_lib = None

EXPORTS = ["stl_compile", "stl_plan_destroy", "stl_plan_info", "stl_workspace_size", "stl_forward",
           "stl_backward", "stl_saved_size", "stl_forward_saving", "stl_backward_saved", "stl_last_error",
           "stl_lpt_order", "stl_autotune", "stl_graph_capture", "stl_graph_launch", "stl_graph_destroy",
           "stl_interval_sweep", "stl_pstl_descent", "stl_forward_static"]


def lib():
    """Load libstlmi.so (built by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise StlError("libstlmi.so is not built: run paper_2501_04194_amd/build.py (or __graft_entry__.build())")
    L = _bind(ctypes.CDLL(LIB_PATH))
    _lib = L
    return L


def _signatures():
    vp, i32, i64, sz, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_float
    B, La = ctypes.POINTER(Batch), ctypes.POINTER(Launch)
    return {
        "stl_compile": [ctypes.POINTER(Node), i32, ctypes.POINTER(i32), i32, i32, ctypes.POINTER(Pred), i32, i32, i32,
                        f32, f32, ctypes.POINTER(vp)],
        "stl_plan_destroy": [vp],
        "stl_plan_info": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "stl_workspace_size": [vp, B, La, ctypes.POINTER(sz), ctypes.POINTER(sz)],
        "stl_forward": [vp, B, vp, vp, vp, vp, sz, La, vp],
        "stl_backward": [vp, B, vp, vp, vp, vp, vp, sz, La, vp],
        "stl_saved_size": [vp, B, ctypes.POINTER(sz)],
        "stl_forward_saving": [vp, B, vp, vp, vp, sz, vp, sz, La, vp],
        "stl_backward_saved": [vp, B, vp, vp, sz, vp, vp, vp, vp, sz, La, vp],
        "stl_forward_static": [vp, B, vp, vp, vp, La, vp],
        "stl_last_error": [],
        "stl_lpt_order": [ctypes.POINTER(i64), i64, ctypes.POINTER(i32)],
        "stl_autotune": [vp, B, vp, vp, vp, vp, vp, vp, sz, vp, La, ctypes.POINTER(f32)],
        "stl_graph_capture": [vp, B, vp, vp, vp, vp, vp, vp, sz, La, vp, ctypes.POINTER(vp)],
        "stl_graph_launch": [vp, vp],
        "stl_graph_destroy": [vp],
        "stl_interval_sweep": [ctypes.POINTER(IntervalDesc), vp, i64, i64, vp, vp, i64, vp, vp, vp, vp],
        "stl_pstl_descent": [ctypes.POINTER(IntervalDesc), vp, i64, i64, f32, f32, f32, f32, i32, f32, f32, vp, vp,
                             vp],
    }


def _bind(L):
    """Argument and result types of the entry points L exports: every one of
    EXPORTS for libstlmi.so; a library with a subset of them (a host-only
    build of the plan compiler) gets those it has."""
    for name, args in _signatures().items():
        try:
            f = getattr(L, name)
        except AttributeError:
            continue
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "stl_last_error" else ctypes.c_int
    return L


def _check(status):
    if status != 0:
        raise StlError("stlmi error %d: %s" % (status, lib().stl_last_error().decode()))


# --------------------------------------------------------------------------- formula -> node array

class _Emitter:
    """Post-order node array (children left to right, root last)."""

    def __init__(self, D):
        self.D = D
        self.nodes, self.child_idx, self.preds = [], [], []
        self.slots = []          # parameter slots: (name or None, literal value or None)
        self.mask_groups = {}    # (a, b, c, eps) names -> first slot of their group

    def slot(self, v):
        self.slots.append((v, None) if isinstance(v, str) else (None, float(v)))
        return len(self.slots) - 1

    def mask(self, nd, m):
        """Smooth time-interval mask (Sec. VI): (a, b, c, eps) in four
        consecutive parameter slots.  Masks whose four entries are the same
        parameter names (tied bounds) share one group of slots."""
        key = (m["a"], m.get("b"), m["c"], m.get("eps", 1e-6))
        nd.mask_unbounded = 1 if m.get("b") is None else 0
        if all(isinstance(v, str) for v in key) and key in self.mask_groups:
            nd.mask_param = self.mask_groups[key]
            return
        nd.mask_param = self.slot(m["a"])
        self.slot(0.0 if m.get("b") is None else m["b"])
        self.slot(m["c"])
        self.slot(m.get("eps", 1e-6))
        if all(isinstance(v, str) for v in key):
            self.mask_groups[key] = nd.mask_param

    def emit(self, f):
        op = f["op"]
        nd = Node()
        nd.mask_param = -1
        nd.beta_param = -1
        nd.pred = -1
        nd.b = -1
        kids = []
        if op == "true":
            nd.op = STL_TRUE
        elif op in ("linear", "norm"):
            p = Pred()
            if op == "linear":
                nd.op = p.kind = STL_PRED_LINEAR
                if len(f["w"]) != self.D:
                    raise ValueError("linear predicate width must equal D")
                for d, v in enumerate(f["w"]):
                    p.w[d] = float(v)
                p.c = float(f.get("c", 0.0))
            else:
                nd.op = p.kind = STL_PRED_NORM
                A = f["A"]
                p.m = len(A)
                for i, row in enumerate(A):
                    if len(row) != self.D:
                        raise ValueError("norm predicate row width must equal D")
                    for d, v in enumerate(row):
                        p.A[i * self.D + d] = float(v)
                for i, v in enumerate(f.get("p", [0.0] * p.m)):
                    p.p[i] = float(v)
                p.r = float(f.get("r", 0.0))
                p.sign = float(f.get("sign", 1.0))
            nd.pred = len(self.preds)
            self.preds.append(p)
        elif op == "not":
            nd.op = STL_NOT
            kids = [self.emit(f["child"])]
        elif op in ("and", "or"):
            nd.op = STL_AND if op == "and" else STL_OR
            kids = [self.emit(c) for c in f["children"]]
        elif op in ("eventually", "always"):
            nd.op = STL_EVENTUALLY if op == "eventually" else STL_ALWAYS
            kids = [self.emit(f["child"])]
            if "mask" in f:
                self.mask(nd, f["mask"])
            else:
                nd.a = int(f.get("a", 0))
                nd.b = -1 if f.get("b") is None else int(f["b"])
            nd.pad = PADS[f.get("pad", "neutral")]
            nd.pad_value = float(f.get("pad_value", 0.0))
        elif op == "until":
            nd.op = STL_UNTIL
            kids = [self.emit(f["left"]), self.emit(f["right"])]
            if "mask" in f:
                self.mask(nd, f["mask"])
            else:
                nd.a = int(f.get("a", 0))
                nd.b = -1 if f.get("b") is None else int(f["b"])
        else:
            raise ValueError("unknown op %r" % op)
        sm = f.get("smooth", False)
        nd.smooth = 2 if sm == "softmax" else (1 if sm else 0)
        if nd.smooth:
            nd.beta_param = self.slot(f.get("beta", 10.0))
        nd.n_child = len(kids)
        nd.child_off = len(self.child_idx)
        self.child_idx.extend(kids)
        self.nodes.append(nd)
        return len(self.nodes) - 1


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A compiled formula (``stl_compile``) plus its parameter layout."""

    def __init__(self, spec, D, params=None, rho_max=1e6, rho_pad=1e6):
        em = _Emitter(D)
        root = em.emit(spec)
        n = len(em.nodes)
        self.D = D
        self.n_nodes = n
        self.slots = em.slots
        self.n_params = len(em.slots)
        self.param_names = sorted({nm for nm, _ in em.slots if nm is not None})
        self.defaults = dict(params or {})
        nodes = (Node * n)(*em.nodes)
        ci = (ctypes.c_int32 * max(1, len(em.child_idx)))(*em.child_idx)
        preds = (Pred * max(1, len(em.preds)))(*em.preds)
        h = ctypes.c_void_p()
        _check(lib().stl_compile(nodes, n, ci, len(em.child_idx), root, preds, len(em.preds), D, self.n_params,
                                 float(rho_max), float(rho_pad), ctypes.byref(h)))
        self._h = h
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.stl_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    # parameter vector ------------------------------------------------------
    def param_vector(self, params=None):
        """float32 numpy vector of every parameter slot (names from `params`)."""
        vals = dict(self.defaults)
        vals.update(params or {})
        out = np.zeros(max(1, self.n_params), dtype=np.float32)
        for i, (nm, lit) in enumerate(self.slots):
            out[i] = vals[nm] if nm is not None else lit
        return out

    def param_grads(self, gvec):
        """{name: gradient} summed over the slots that carry the name."""
        g = np.asarray(gvec, dtype=np.float64)
        res = {}
        for i, (nm, _) in enumerate(self.slots):
            if nm is not None:
                res[nm] = res.get(nm, 0.0) + float(g[i])
        return res

    # batches ---------------------------------------------------------------
    def _batch(self, x, offsets=None, order=None, T=None):
        b = Batch()
        b.x = x.data_ptr()
        b.D = self.D
        if offsets is None:
            if x.dim() != 3 or x.shape[2] != self.D:
                raise ValueError("dense x must be [B, T, D]")
            b.B, b.T = x.shape[0], x.shape[1]
            b.offsets = None
        else:
            if x.dim() != 2 or x.shape[1] != self.D:
                raise ValueError("ragged x must be [N_total, D]")
            if T is None:
                raise ValueError("ragged batches need T (an upper bound on the lengths)")
            b.B, b.T = offsets.shape[0] - 1, int(T)
            b.offsets = offsets.data_ptr()
        b.order = None if order is None else order.data_ptr()
        return b

    def workspace(self, torch, batch, launch=None, device=None):
        fw, bw = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().stl_workspace_size(self._h, ctypes.byref(batch), None if launch is None else ctypes.byref(launch),
                                        ctypes.byref(fw), ctypes.byref(bw)))
        need = max(fw.value, bw.value, 256)
        key = str(device)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws

    def saved_buffer(self, x, offsets=None, T=None):
        """Device buffer for the mask-node traces kept between forward and backward (``stl_saved_size``)."""
        import torch
        bt = self._batch(x, offsets, None, T)
        n = ctypes.c_size_t()
        _check(lib().stl_saved_size(self._h, ctypes.byref(bt), ctypes.byref(n)))
        return torch.empty(max(256, n.value), dtype=torch.uint8, device=x.device)

    def forward(self, x, pvec, offsets=None, order=None, T=None, node_traces=False, launch=None, saved=None):
        """Root robustness trace (float32) and optionally every node trace.

        ``saved`` (from ``saved_buffer``): also keep the mask-node traces for
        ``backward(..., saved=...)`` (``stl_forward_saving``)."""
        import torch
        _require_gpu(torch, x)
        x = x.contiguous()
        bt = self._batch(x, offsets, order, T)
        N = x.shape[0] * x.shape[1] if offsets is None else x.shape[0]
        root = torch.empty(N, dtype=torch.float32, device=x.device)
        nodes = torch.empty((self.n_nodes, N), dtype=torch.float32, device=x.device) if node_traces else None
        ws = self.workspace(torch, bt, launch, x.device)
        lp = None if launch is None else ctypes.byref(launch)
        if saved is not None:
            if node_traces:
                raise ValueError("node_traces and saved cannot be combined")
            _check(lib().stl_forward_saving(self._h, ctypes.byref(bt), _ptr(pvec), _ptr(root), _ptr(saved),
                                            saved.numel(), _ptr(ws), ws.numel(), lp, _stream(torch, x.device)))
        else:
            _check(lib().stl_forward(self._h, ctypes.byref(bt), _ptr(pvec), _ptr(root), _ptr(nodes), _ptr(ws),
                                     ws.numel(), lp, _stream(torch, x.device)))
        if offsets is None:
            root = root.view(x.shape[0], x.shape[1])
            if nodes is not None:
                nodes = nodes.view(self.n_nodes, x.shape[0], x.shape[1])
        return (root, nodes) if node_traces else root

    def forward_static(self, x, pvec, offsets=None, order=None, T=None, node_traces=False, launch=None):
        """``forward`` through ``stl_forward_static``: the library's fixed
        device workspace instead of one allocated here (the root and node
        traces are still allocated by the caller, i.e. here)."""
        import torch
        _require_gpu(torch, x)
        x = x.contiguous()
        bt = self._batch(x, offsets, order, T)
        N = x.shape[0] * x.shape[1] if offsets is None else x.shape[0]
        root = torch.empty(N, dtype=torch.float32, device=x.device)
        nodes = torch.empty((self.n_nodes, N), dtype=torch.float32, device=x.device) if node_traces else None
        lp = None if launch is None else ctypes.byref(launch)
        _check(lib().stl_forward_static(self._h, ctypes.byref(bt), _ptr(pvec), _ptr(root), _ptr(nodes), lp,
                                        _stream(torch, x.device)))
        if offsets is None:
            root = root.view(x.shape[0], x.shape[1])
            if nodes is not None:
                nodes = nodes.view(self.n_nodes, x.shape[0], x.shape[1])
        return (root, nodes) if node_traces else root

    def backward(self, x, G, pvec, offsets=None, order=None, T=None, launch=None, want_params=True, saved=None):
        """(dx, dparams-vector) for the upstream gradient G of the root trace.

        ``saved``: the buffer filled by ``forward(..., saved=...)`` on the
        same x and parameters (``stl_backward_saved``)."""
        import torch
        _require_gpu(torch, x)
        x = x.contiguous()
        G = G.contiguous()
        bt = self._batch(x, offsets, order, T)
        dx = torch.empty_like(x)
        gp = torch.empty(max(1, self.n_params), dtype=torch.float32, device=x.device) if want_params else None
        ws = self.workspace(torch, bt, launch, x.device)
        lp = None if launch is None else ctypes.byref(launch)
        if saved is not None:
            _check(lib().stl_backward_saved(self._h, ctypes.byref(bt), _ptr(pvec), _ptr(saved), saved.numel(),
                                            _ptr(G), _ptr(dx), _ptr(gp), _ptr(ws), ws.numel(), lp,
                                            _stream(torch, x.device)))
        else:
            _check(lib().stl_backward(self._h, ctypes.byref(bt), _ptr(pvec), _ptr(G), _ptr(dx), _ptr(gp), _ptr(ws),
                                      ws.numel(), lp, _stream(torch, x.device)))
        return dx, gp


def _require_gpu(torch, x):
    if not x.is_cuda:
        raise StlError("stlmi runs on the GPU only: move the tensors to a HIP device")
    if x.dtype != torch.float32:
        raise StlError("x must be float32")


def interval_sweep(x, a, b, w, c=0.0, op="always", smooth=True, beta=10.0, mask_c=1.0, mask_eps=1e-6,
                   rho_pad=1e6, grads=True):
    """Robustness at t = 0 of op_{mask(a_n, b_n)}(w . x - c) for every trajectory of
    x [B, T, D] and every interval n (``stl_interval_sweep``): returns rho [B, N]
    and, with ``grads``, d rho / d a and d rho / d b [B, N] (a, b in timesteps)."""
    import torch
    _require_gpu(torch, x)
    x = x.contiguous()
    a = a.contiguous()
    b = b.contiguous()
    if a.dtype != torch.float32 or b.dtype != torch.float32 or a.shape != b.shape or a.dim() != 1:
        raise ValueError("a and b must be float32 vectors of one length")
    B, T, D = x.shape
    if len(w) != D:
        raise ValueError("predicate width must equal D")
    d = IntervalDesc()
    d.op = STL_ALWAYS if op == "always" else STL_EVENTUALLY
    d.smooth = 1 if smooth else 0
    d.beta, d.mask_c, d.mask_eps = float(beta), float(mask_c), float(mask_eps)
    d.D = D
    for k, v in enumerate(w):
        d.w[k] = float(v)
    d.c, d.rho_pad = float(c), float(rho_pad)
    N = a.shape[0]
    rho = torch.empty((B, N), dtype=torch.float32, device=x.device)
    ga = torch.empty_like(rho) if grads else None
    gb = torch.empty_like(rho) if grads else None
    _check(lib().stl_interval_sweep(ctypes.byref(d), _ptr(x), B, T, _ptr(a), _ptr(b), N, _ptr(rho), _ptr(ga),
                                    _ptr(gb), _stream(torch, x.device)))
    return (rho, ga, gb) if grads else rho


def pstl_descent(x, logits, steps, lr=1e-2, gamma=0.1, c_range=(1.0, 20.0), beta_range=(1.0, 20.0), w=(1.0,),
                 c=0.0, op="always", mask_eps=1e-6, want_loss=False):
    """Gradient descent on the pSTL loss in one launch (``stl_pstl_descent``):
    logits (a float32 device tensor [2], p_a and p_b) is updated in place;
    returns the per-step loss tensor when ``want_loss``."""
    import torch
    _require_gpu(torch, x)
    x = x.contiguous()
    B, T, D = x.shape
    d = IntervalDesc()
    d.op = STL_ALWAYS if op == "always" else STL_EVENTUALLY
    d.smooth = 1
    d.mask_eps = float(mask_eps)
    d.D = D
    for k, v in enumerate(w):
        d.w[k] = float(v)
    d.c = float(c)
    loss = torch.empty(max(1, steps), dtype=torch.float32, device=x.device) if want_loss else None
    _check(lib().stl_pstl_descent(ctypes.byref(d), _ptr(x), B, T, float(c_range[0]), float(c_range[1]),
                                  float(beta_range[0]), float(beta_range[1]), int(steps), float(lr), float(gamma),
                                  _ptr(logits), _ptr(loss), _stream(torch, x.device)))
    return loss


def lpt_order(offsets_host):
    """Longest-first processing order for a ragged batch (``stl_lpt_order``)."""
    off = np.ascontiguousarray(offsets_host, dtype=np.int64)
    B = len(off) - 1
    order = np.zeros(max(1, B), dtype=np.int32)
    _check(lib().stl_lpt_order(off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), B,
                               order.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
    return order[:B]


def autotune(plan, x, pvec, G, offsets=None, order=None, T=None):
    """Pick the fastest launch configuration (``stl_autotune``); returns (Launch, ms)."""
    import torch
    x = x.contiguous()
    bt = plan._batch(x, offsets, order, T)
    N = x.shape[0] * x.shape[1] if offsets is None else x.shape[0]
    root = torch.empty(N, dtype=torch.float32, device=x.device)
    dx = torch.empty_like(x)
    gp = torch.empty(max(1, plan.n_params), dtype=torch.float32, device=x.device)
    fw, bw = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().stl_workspace_size(plan.handle, ctypes.byref(bt), None, ctypes.byref(fw), ctypes.byref(bw)))
    biggest = 0
    for nt in (128, 256, 512):
        for wpc in (0, 1, 2, 4, 8):
            l = Launch(nt, wpc, 0, 0)
            a, b = ctypes.c_size_t(), ctypes.c_size_t()
            _check(lib().stl_workspace_size(plan.handle, ctypes.byref(bt), ctypes.byref(l), ctypes.byref(a),
                                            ctypes.byref(b)))
            biggest = max(biggest, a.value, b.value)
    ws = torch.empty(biggest, dtype=torch.uint8, device=x.device)
    best = Launch()
    ms = ctypes.c_float()
    _check(lib().stl_autotune(plan.handle, ctypes.byref(bt), _ptr(pvec), _ptr(root), _ptr(G.contiguous()), _ptr(dx),
                              _ptr(gp), _ptr(ws), ws.numel(), _stream(torch, x.device), ctypes.byref(best),
                              ctypes.byref(ms)))
    return best, ms.value


class Graph:
    """Forward + backward captured once into a HIP graph (``stl_graph_capture``)."""

    def __init__(self, plan, x, pvec, G, offsets=None, order=None, T=None, launch=None):
        import torch
        self.plan = plan
        self.x = x
        self.pvec = pvec
        self.G = G
        bt = plan._batch(x, offsets, order, T)
        self._bt = bt
        N = x.shape[0] * x.shape[1] if offsets is None else x.shape[0]
        self.root = torch.empty(N, dtype=torch.float32, device=x.device)
        self.dx = torch.empty_like(x)
        self.gp = torch.empty(max(1, plan.n_params), dtype=torch.float32, device=x.device)
        self.ws = plan.workspace(torch, bt, launch, x.device).clone()
        self._keep = (offsets, order, launch)
        h = ctypes.c_void_p()
        _check(lib().stl_graph_capture(plan.handle, ctypes.byref(bt), _ptr(pvec), _ptr(self.root), _ptr(G), _ptr(self.dx),
                                       _ptr(self.gp), _ptr(self.ws), self.ws.numel(),
                                       None if launch is None else ctypes.byref(launch), _stream(torch, x.device),
                                       ctypes.byref(h)))
        self._h = h

    def launch(self):
        import torch
        _check(lib().stl_graph_launch(self._h, _stream(torch, self.x.device)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.stl_graph_destroy(h)
            self._h = None


def make_autograd():
    import torch

    class StlRobustness(torch.autograd.Function):
        """Robustness trace with a hand-written backward.

        Saves x, the parameter vector and the mask-node traces of the fused
        path (``stl_forward_saving`` / ``stl_backward_saved``); anything else
        is recomputed on chip in the backward kernel.
        """

        @staticmethod
        def forward(ctx, plan, x, pvec):
            ctx.plan = plan
            x = x.contiguous()
            saved = plan.saved_buffer(x)
            ctx.save_for_backward(x, pvec, saved)
            return plan.forward(x, pvec, saved=saved)

        @staticmethod
        def backward(ctx, G):
            x, pvec, saved = ctx.saved_tensors
            dx, gp = ctx.plan.backward(x, G, pvec, saved=saved)
            return None, dx, gp[: pvec.numel()]

    return StlRobustness


_autograd = None


def robustness(plan, x, pvec):
    """Differentiable robustness trace [B, T] of a dense batch x [B, T, D]."""
    global _autograd
    if _autograd is None:
        _autograd = make_autograd()
    return _autograd.apply(plan, x, pvec)
