"""FP64 CPU oracle for STL robustness traces and gradients.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark; never by the GPU library.  It shares no
code with the GPU path.  The arithmetic lives in ``stl_oracle.c`` (plain loops
over each window, straight from the definitions of arXiv 2501.04194
Sec. III-B, III-C, IV-B, IV-C and VI); this module builds it, turns a formula
description into the C node array and marshals arrays.

``literal_mask.py`` next to this file is a second, independent reference for
tiny signals: it builds the unrolled arrays and masks of Sec. IV literally.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

O_TRUE, O_LINEAR, O_NORM, O_NOT, O_AND, O_OR, O_EV, O_ALW, O_UNTIL = range(9)
PADS = {"neutral": 0, "last": 1, "const": 2}
OMAXCH, OMAXD = 16, 16

RHO_MAX = 1e6   # value of True (Sec. III-B: rho_max > 0)
RHO_PAD = 1e6   # magnitude of the empty-window value


class ONode(ctypes.Structure):
    _fields_ = [
        ("op", ctypes.c_int), ("nch", ctypes.c_int), ("ch", ctypes.c_int * OMAXCH),
        ("smooth", ctypes.c_int), ("beta", ctypes.c_double),
        ("a", ctypes.c_int), ("b", ctypes.c_int),
        ("masked", ctypes.c_int), ("ma", ctypes.c_double), ("mb", ctypes.c_double),
        ("mc", ctypes.c_double), ("meps", ctypes.c_double), ("mb_inf", ctypes.c_int),
        ("pad", ctypes.c_int), ("pad_value", ctypes.c_double),
        ("D", ctypes.c_int), ("w", ctypes.c_double * OMAXD), ("c", ctypes.c_double),
        ("m", ctypes.c_int), ("A", ctypes.c_double * (4 * OMAXD)), ("p", ctypes.c_double * 4),
        ("r", ctypes.c_double), ("sign", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        # STL_ORACLE_LIB: another build of stl_oracle.c (the host sanitizer test's)
        lib = ctypes.CDLL(os.environ.get("STL_ORACLE_LIB") or build())
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_longlong)
        np_ = ctypes.POINTER(ONode)
        lib.orc_forward.argtypes = [np_, ctypes.c_int, dp, lp, ctypes.c_longlong, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, ip, dp, dp]
        lib.orc_backward.argtypes = [np_, ctypes.c_int, dp, lp, ctypes.c_longlong, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, ip, dp, dp, dp, dp]
        lib.orc_backward_nodes.argtypes = [np_, ctypes.c_int, dp, lp, ctypes.c_longlong,
                                           ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp,
                                           dp, dp]
        lib.orc_mask_weights.argtypes = [np_, ctypes.c_int, dp, dp, dp]
        lib.orc_sizeof_node.restype = ctypes.c_int
        assert lib.orc_sizeof_node() == ctypes.sizeof(ONode), "ONode layout mismatch"
        _lib = lib
    return _lib


def _val(v, params):
    if isinstance(v, str):
        return float(params[v])
    return float(v)


class Compiled:
    """Post-order node array of a formula plus the names of its learnable mask bounds."""

    def __init__(self, spec, params, D):
        self.nodes = []
        self.mask_names = []   # per node index: (name_a, name_b) or None
        self.D = D
        self.params = dict(params or {})
        self.root = self._emit(spec)
        n = len(self.nodes)
        self.arr = (ONode * n)(*self.nodes)

    def _mask(self, nd, m):
        """Smooth time-interval mask (Sec. VI) on a temporal node; returns
        the names of its learnable bounds."""
        nd.masked = 1
        nd.ma = _val(m["a"], self.params)
        nd.mb_inf = 1 if m.get("b") is None else 0
        nd.mb = 0.0 if nd.mb_inf else _val(m["b"], self.params)
        nd.mc = _val(m["c"], self.params)
        nd.meps = _val(m.get("eps", 1e-6), self.params)
        return (m["a"] if isinstance(m["a"], str) else None,
                m.get("b") if isinstance(m.get("b"), str) else None)

    def _emit(self, f):
        op = f["op"]
        nd = ONode()
        nd.D = self.D
        nd.b = -1
        names = None
        kids = []
        if op == "true":
            nd.op = O_TRUE
        elif op == "linear":
            nd.op = O_LINEAR
            w = f["w"]
            if len(w) != self.D or self.D > OMAXD:
                raise ValueError("linear predicate width must equal D")
            for d in range(self.D):
                nd.w[d] = float(w[d])
            nd.c = float(f.get("c", 0.0))
        elif op == "norm":
            nd.op = O_NORM
            A = f["A"]
            nd.m = len(A)
            if nd.m > 4:
                raise ValueError("norm predicate supports at most 4 rows")
            for i, row in enumerate(A):
                if len(row) != self.D:
                    raise ValueError("norm predicate row width must equal D")
                for d in range(self.D):
                    nd.A[i * self.D + d] = float(row[d])
            p = f.get("p", [0.0] * nd.m)
            for i in range(nd.m):
                nd.p[i] = float(p[i])
            nd.r = float(f.get("r", 0.0))
            nd.sign = float(f.get("sign", 1.0))
        elif op == "not":
            nd.op = O_NOT
            kids = [self._emit(f["child"])]
        elif op in ("and", "or"):
            nd.op = O_AND if op == "and" else O_OR
            kids = [self._emit(c) for c in f["children"]]
            if not 1 <= len(kids) <= OMAXCH:
                raise ValueError("and/or takes 1..16 children")
        elif op in ("eventually", "always"):
            nd.op = O_EV if op == "eventually" else O_ALW
            kids = [self._emit(f["child"])]
            if "mask" in f:
                names = self._mask(nd, f["mask"])
            else:
                nd.a = int(f.get("a", 0))
                b = f.get("b")
                nd.b = -1 if b is None else int(b)
                if nd.a < 0 or (nd.b >= 0 and nd.b < nd.a):
                    raise ValueError("bad interval")
            nd.pad = PADS[f.get("pad", "neutral")]
            nd.pad_value = float(f.get("pad_value", 0.0))
        elif op == "until":
            nd.op = O_UNTIL
            kids = [self._emit(f["left"]), self._emit(f["right"])]
            if "mask" in f:
                names = self._mask(nd, f["mask"])
            else:
                nd.a = int(f.get("a", 0))
                b = f.get("b")
                nd.b = -1 if b is None else int(b)
                if nd.a < 0 or (nd.b >= 0 and nd.b < nd.a):
                    raise ValueError("bad interval")
        else:
            raise ValueError("unknown op %r" % op)
        sm = f.get("smooth", False)
        nd.smooth = 2 if sm == "softmax" else (1 if sm else 0)
        if nd.smooth == 2 and (op not in ("and", "or", "eventually", "always") or "mask" in f):
            raise ValueError("the softmax-weighted form applies to and/or and unmasked windows")
        nd.beta = _val(f.get("beta", 10.0), self.params)
        nd.nch = len(kids)
        for i, k in enumerate(kids):
            nd.ch[i] = k
        self.nodes.append(nd)
        self.mask_names.append(names)
        return len(self.nodes) - 1


def _dense(x):
    x = np.asarray(x)
    if x.ndim != 3:
        raise ValueError("dense x must be [B, T, D]")
    B, T, D = x.shape
    off = np.arange(B + 1, dtype=np.int64) * T
    return x.reshape(B * T, D), off, (B, T)


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def forward(spec, x, params=None, offsets=None, leaf_traces=None, all_nodes=False,
            rho_max=RHO_MAX, rho_pad=RHO_PAD):
    """Robustness traces in float64.

    x: [B, T, D] (dense) or [N_total, D] with ``offsets`` (int64, B+1).
    leaf_traces: optional {node_index: trace array shaped like the output}
    that replaces the computed trace of those nodes.
    Returns the root trace ([B, T] or [N_total]); with all_nodes=True also the
    list of every node trace (post-order, root last).
    """
    lib = _load()
    shape = None
    if offsets is None:
        xf, off, shape = _dense(x)
    else:
        xf, off = np.asarray(x), np.asarray(offsets, dtype=np.int64)
    D = xf.shape[1]
    comp = Compiled(spec, params, D)
    n = len(comp.nodes)
    xd = np.ascontiguousarray(xf, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    Ntot = int(off[-1])
    traces = np.zeros((n, Ntot), dtype=np.float64)
    om, ot = None, None
    if leaf_traces:
        om = np.zeros(n, dtype=np.int32)
        ot = np.zeros((n, Ntot), dtype=np.float64)
        for i, tr in leaf_traces.items():
            om[i] = 1
            ot[i] = np.asarray(tr, dtype=np.float64).reshape(-1)
    err = lib.orc_forward(comp.arr, n, _ptr(xd, ctypes.c_double), _ptr(off, ctypes.c_longlong),
                          len(off) - 1, D, rho_max, rho_pad,
                          None if om is None else _ptr(om, ctypes.c_int),
                          None if ot is None else _ptr(ot, ctypes.c_double),
                          _ptr(traces, ctypes.c_double))
    if err:
        raise MemoryError("oracle forward failed")
    rs = (lambda a: a.reshape(shape)) if shape else (lambda a: a)
    if all_nodes:
        return rs(traces[-1]), [rs(traces[i]) for i in range(n)]
    return rs(traces[-1])


def backward(spec, x, G, params=None, offsets=None, leaf_traces=None, node_adjoints=False,
             rho_max=RHO_MAX, rho_pad=RHO_PAD):
    """Gradient of sum(G * root_trace) w.r.t. x (float64) and the named mask bounds.

    Returns (dx, dparams) with dparams = {name: value}; with node_adjoints=True
    also the adjoint of every node trace (post-order).
    """
    lib = _load()
    shape = None
    if offsets is None:
        xf, off, shape = _dense(x)
    else:
        xf, off = np.asarray(x), np.asarray(offsets, dtype=np.int64)
    D = xf.shape[1]
    comp = Compiled(spec, params, D)
    n = len(comp.nodes)
    xd = np.ascontiguousarray(xf, dtype=np.float64)
    off = np.ascontiguousarray(off, dtype=np.int64)
    B = len(off) - 1
    Ntot = int(off[-1])
    Gd = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(-1))
    if Gd.shape[0] != Ntot:
        raise ValueError("G has the wrong size")
    dx = np.zeros((Ntot, D), dtype=np.float64)
    dpt = np.zeros((B, n, 2), dtype=np.float64)
    adj = None
    if node_adjoints:
        if leaf_traces:
            raise ValueError("node_adjoints with leaf_traces is not supported")
        adj = np.zeros((n, Ntot), dtype=np.float64)
        err = lib.orc_backward_nodes(comp.arr, n, _ptr(xd, ctypes.c_double),
                                     _ptr(off, ctypes.c_longlong), B, D, rho_max, rho_pad,
                                     _ptr(Gd, ctypes.c_double), _ptr(dx, ctypes.c_double),
                                     _ptr(dpt, ctypes.c_double), _ptr(adj, ctypes.c_double))
    else:
        om, ot = None, None
        if leaf_traces:
            om = np.zeros(n, dtype=np.int32)
            ot = np.zeros((n, Ntot), dtype=np.float64)
            for i, tr in leaf_traces.items():
                om[i] = 1
                ot[i] = np.asarray(tr, dtype=np.float64).reshape(-1)
        err = lib.orc_backward(comp.arr, n, _ptr(xd, ctypes.c_double), _ptr(off, ctypes.c_longlong),
                               B, D, rho_max, rho_pad,
                               None if om is None else _ptr(om, ctypes.c_int),
                               None if ot is None else _ptr(ot, ctypes.c_double),
                               _ptr(Gd, ctypes.c_double), _ptr(dx, ctypes.c_double),
                               _ptr(dpt, ctypes.c_double))
    if err:
        raise MemoryError("oracle backward failed")
    tot = np.zeros((n, 2))
    for b in range(B):            # fixed trajectory order
        tot += dpt[b]
    dparams = {}
    for i, names in enumerate(comp.mask_names):
        if names is None:
            continue
        if names[0]:
            dparams[names[0]] = dparams.get(names[0], 0.0) + tot[i, 0]
        if names[1]:
            dparams[names[1]] = dparams.get(names[1], 0.0) + tot[i, 1]
    dx = dx.reshape(shape + (D,)) if shape else dx
    if node_adjoints:
        rs = (lambda a: a.reshape(shape)) if shape else (lambda a: a)
        return dx, dparams, [rs(adj[i]) for i in range(n)]
    return dx, dparams


def mask_weights(a, b, c, eps, L):
    """(w, dw/da, dw/db) of the smooth mask (Sec. VI) for offsets 0..L-1."""
    lib = _load()
    nd = ONode()
    nd.op = O_EV
    nd.masked = 1
    nd.ma, nd.mc, nd.meps = float(a), float(c), float(eps)
    nd.mb_inf = 1 if b is None else 0
    nd.mb = 0.0 if b is None else float(b)
    w = np.zeros(L)
    da = np.zeros(L)
    db = np.zeros(L)
    lib.orc_mask_weights(ctypes.byref(nd), L, _ptr(w, ctypes.c_double), _ptr(da, ctypes.c_double),
                         _ptr(db, ctypes.c_double))
    return w, da, db


def node_count(spec, D, params=None):
    return len(Compiled(spec, params, D).nodes)


def interval_sweep(x, a, b, w, c=0.0, op="always", smooth=True, beta=10.0, mask_c=1.0, mask_eps=1e-6,
                   rho_pad=RHO_PAD):
    """Robustness at t = 0 of op_{mask(a_n, b_n)}(w . x - c) for every
    trajectory of x [B, T, D] and every interval n, with d/da_n and d/db_n
    (Sec. VI: the masked form evaluated for many time-interval values).

    Plain composition of the pinned single-formula oracle: one forward and one
    backward (upstream gradient 1 at t = 0) per trajectory and interval.
    Returns (rho, drho_da, drho_db), each [B, N] float64."""
    x = np.asarray(x, dtype=np.float32)
    B, T, D = x.shape
    N = len(a)
    rho, ga, gb = np.zeros((B, N)), np.zeros((B, N)), np.zeros((B, N))
    spec = {"op": op, "smooth": bool(smooth), "beta": float(beta),
            "child": {"op": "linear", "w": [float(v) for v in w], "c": float(c)},
            "mask": {"a": "a", "b": "b", "c": float(mask_c), "eps": float(mask_eps)}}
    G = np.zeros((1, T), dtype=np.float32)
    G[0, 0] = 1.0
    for n in range(N):
        params = {"a": float(a[n]), "b": float(b[n])}
        r = forward(spec, x, params=params, rho_pad=rho_pad)
        rho[:, n] = r[:, 0]
        for k in range(B):
            _, dp = backward(spec, x[k:k + 1], G, params=params, rho_pad=rho_pad)
            ga[k, n], gb[k, n] = dp.get("a", 0.0), dp.get("b", 0.0)
    return rho, ga, gb
