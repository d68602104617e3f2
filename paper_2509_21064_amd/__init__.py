"""PDBO hot path on MI355X: Python binding of libpdbo (include/pdbo.h).

The functions below carry the names of the C entry points and only marshal
arguments (numpy arrays for host data, torch tensors for device data, the
current torch stream); every step of Alg. 1 runs in the HIP kernels of the
library.  There is no CPU path: a missing libpdbo.so raises on first use.

Instances are duck-typed: a QUBO has ``n`` and either a dense int32 ``Q`` or CSR
``row_ptr``/``col_idx``/``vals``, plus ``c`` (int64 or None); a MaxSAT formula
has ``n``, ``lits`` (m, k) DIMACS int32 and ``w`` (m,) int32.  Parameters are a
dict with B, alpha, beta, y0, delta, scale, g ("quad"/"entropy"), and
optionally precision ("fp32"/"bf16"/"fp8"/"i8"), eval_every, tile, graph_chunk.
Starting points x0 are float64 arrays of shape (B, n), or None: then the
library draws them with its Philox4x32-10 generator keyed by params["seed"].
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from ._abi import (PDBO_BF16, PDBO_CSR, PDBO_DENSE, PDBO_FP8, PDBO_FP32, PDBO_G_ENTROPY, PDBO_I8,
                   PDBO_G_QUAD, PDBO_K_ARGMIN, PDBO_K_EVAL, PDBO_K_INCR, PDBO_K_PERSISTENT, PDBO_K_STEP,
                   PdboError, check, load)

__all__ = [
    "load", "PdboError", "Context", "qubo_gda_init", "qubo_gda_step", "qubo_gda_result",
    "qubo_gda_get_state", "qubo_gda_set_state", "qubo_gda_restart", "qubo_gda_objectives", "qubo_gda_grad",
    "qubo_gda_eval", "qubo_gda_eval_noalloc", "qubo_dual_bound", "qubo_gda_trace", "qubo_gda_solve",
    "qubo_gda_objectives_f64", "qubo_gda_eval_f64", "qubo_gda_trace_f64",
    "qubo_gda_batch_init", "qubo_gda_batch_result",
    "qubo_gda_batch_solve", "kcut_gda_init", "maxsat_gda_init", "maxsat_gda_step", "maxsat_gda_result",
    "maxsat_gda_solve", "maxsat_lagrangian_fwd", "maxsat_lagrangian_bwd", "MaxSATLagrangian",
    "PDBO_FP32", "PDBO_BF16", "PDBO_FP8", "PDBO_I8", "PDBO_K_STEP", "PDBO_K_EVAL", "PDBO_K_ARGMIN",
    "PDBO_K_PERSISTENT", "PDBO_K_INCR",
]

_PREC = {"fp32": PDBO_FP32, "bf16": PDBO_BF16, "fp8": PDBO_FP8, "i8": PDBO_I8}
_G = {"quad": PDBO_G_QUAD, "entropy": PDBO_G_ENTROPY, "poly": _abi.PDBO_G_POLY}
_DUAL = {"vector": _abi.PDBO_DUAL_VECTOR, "scalar": _abi.PDBO_DUAL_SCALAR}


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _current_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # torch without a GPU: the library uses the null stream
        pass
    return None


class _Keep:
    """Holds the numpy buffers a ctypes struct points into."""

    def __init__(self):
        self.bufs = []

    def arr(self, a, dtype):
        if a is None:
            return None
        b = np.ascontiguousarray(a, dtype=dtype)
        self.bufs.append(b)
        return b


def _is_real(q) -> bool:
    """Float weights (Q or vals, or c, of a floating dtype) take PDBO_W_F64."""
    w = q.Q if getattr(q, "Q", None) is not None else q.vals
    c = getattr(q, "c", None)
    return np.asarray(w).dtype.kind == "f" or (c is not None and np.asarray(c).dtype.kind == "f")


def _qubo_struct(q, keep: _Keep) -> _abi.pdbo_qubo:
    s = _abi.pdbo_qubo()
    s.n = int(q.n)
    real = _is_real(q)
    s.wtype = _abi.PDBO_W_F64 if real else _abi.PDBO_W_INT32
    wt = np.float64 if real else np.int32
    if getattr(q, "Q", None) is not None:
        s.format = PDBO_DENSE
        w = _ptr(keep.arr(q.Q, wt))
        s.nnz = 0
    else:
        s.format = PDBO_CSR
        s.row_ptr = _ptr(keep.arr(q.row_ptr, np.int32))
        s.col_idx = _ptr(keep.arr(q.col_idx, np.int32))
        w = _ptr(keep.arr(q.vals, wt))
        s.nnz = int(len(q.col_idx))
    c = getattr(q, "c", None)
    cp = None if c is None else _ptr(keep.arr(c, np.float64 if real else np.int64))
    if real:
        s.qd, s.cd = w, cp
    else:
        s.q, s.c = w, cp
    return s


def _maxsat_struct(f, keep: _Keep) -> _abi.pdbo_maxsat:
    s = _abi.pdbo_maxsat()
    lits = keep.arr(f.lits, np.int32)
    s.n, s.m, s.k = int(f.n), int(lits.shape[0]), int(lits.shape[1])
    s.lits = _ptr(lits)
    s.w = _ptr(keep.arr(f.w, np.int32)) if getattr(f, "w", None) is not None else None
    return s


def _params_struct(p: dict, x0, keep: _Keep) -> _abi.pdbo_params:
    s = _abi.pdbo_params()
    s.B = int(p["B"])
    s.g_kind = _G[p.get("g", "quad")]
    s.precision = _PREC[p.get("precision", "fp32")]
    s.eval_every = int(p.get("eval_every", 1))
    s.alpha, s.beta, s.y0 = float(p["alpha"]), float(p["beta"]), float(p["y0"])
    s.delta, s.scale = float(p["delta"]), float(p.get("scale", 1.0))
    s.tile = int(p.get("tile", 0))
    s.graph_chunk = int(p.get("graph_chunk", 0))
    s.g_degree = int(p.get("g_degree", 1))
    s.dual_kind = _DUAL[p.get("dual", "vector")]
    s.x0 = _ptr(keep.arr(x0, np.float64)) if x0 is not None else None
    s.seed = int(p.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF
    return s


def _result_dict(r: _abi.pdbo_result, best_x) -> dict:
    return dict(best_obj=int(r.best_obj), best_obj_f64=float(r.best_obj_f64),
                best_restart=int(r.best_restart), best_iter=int(r.best_iter),
                time_to_best_s=float(r.time_to_best_s), steps_done=int(r.steps_done), best_x=best_x)


class Context:
    """Owner of a pdbo_ctx*; the methods call the entry points of the same name."""

    def __init__(self, handle, n, B, kind, ninst=1, ns=None, k=1):
        self.h = handle
        self.n, self.B, self.kind, self.ninst = n, B, kind, ninst
        self.ns = ns or [n]
        self.k = k  # values per node of x (Max-k-Cut: the k logits)

    def __del__(self):
        self.destroy()

    def destroy(self):
        if getattr(self, "h", None):
            load().pdbo_destroy(self.h)
            self.h = None

    def step(self, nsteps):
        return qubo_gda_step(self, nsteps)

    def result(self):
        return qubo_gda_result(self)

    def get_state(self):
        return qubo_gda_get_state(self)

    def set_state(self, x=None, y=None, t=0):
        return qubo_gda_set_state(self, x, y, t)

    def objectives(self):
        return qubo_gda_objectives(self)

    def objectives_f64(self):
        return qubo_gda_objectives_f64(self)

    def eval_f64(self, xr):
        return qubo_gda_eval_f64(self, xr)

    def trace_f64(self, cap=4096):
        return qubo_gda_trace_f64(self, cap)

    def restart(self, x0):
        return qubo_gda_restart(self, x0)

    def grad(self, x):
        return qubo_gda_grad(self, x)

    def eval(self, xr):
        return qubo_gda_eval(self, xr)

    def trace(self, cap=4096):
        return qubo_gda_trace(self, cap)

    def timing(self, enable=True, classes=None, stride=1):
        """Kernel timing on (all classes, or the PDBO_K_* classes listed) or off;
        with stride > 1 only every stride-th launch of a class is timed."""
        if classes is not None and enable:
            mask = 0
            for k in classes:
                mask |= 1 << int(k)
            check(load().pdbo_timing_classes(self.h, mask), self.h)
        else:
            check(load().pdbo_timing(self.h, int(bool(enable))), self.h)
        check(load().pdbo_timing_stride(self.h, int(stride)), self.h)

    def kernel_time(self, which):
        ms, cnt = ctypes.c_double(), ctypes.c_int64()
        check(load().pdbo_kernel_time(self.h, which, ctypes.byref(ms), ctypes.byref(cnt)), self.h)
        return ms.value, cnt.value

    @property
    def tile_name(self):
        return load().pdbo_tile_name(self.h).decode()


def qubo_gda_init(q, params: dict, x0, stream=None) -> Context:
    lib, keep = load(), _Keep()
    prob = _qubo_struct(q, keep)
    par = _params_struct(params, x0, keep)
    h = ctypes.c_void_p()
    st = lib.qubo_gda_init(ctypes.byref(prob), ctypes.byref(par),
                           stream if stream is not None else _current_stream(), ctypes.byref(h))
    check(st)
    return Context(h, int(q.n), int(params["B"]), "qubo")


def qubo_gda_step(ctx: Context, nsteps: int):
    check(load().qubo_gda_step(ctx.h, int(nsteps)), ctx.h)


def qubo_gda_result(ctx: Context) -> dict:
    bx = np.zeros(ctx.n, dtype=np.uint8)
    r = _abi.pdbo_result()
    r.best_x = _ptr(bx)
    check(load().qubo_gda_result(ctx.h, ctypes.byref(r)), ctx.h)
    return _result_dict(r, bx)


def _xshape(ctx):
    return (ctx.B, ctx.n) if ctx.k == 1 else (ctx.B, ctx.n, ctx.k)


def qubo_gda_get_state(ctx: Context):
    x = np.zeros(_xshape(ctx), dtype=np.float32)
    y = np.zeros((ctx.B, ctx.n), dtype=np.float32)
    t = ctypes.c_int64()
    check(load().qubo_gda_get_state(ctx.h, _ptr(x), _ptr(y), ctypes.byref(t)), ctx.h)
    return x, y, t.value


def qubo_gda_set_state(ctx: Context, x=None, y=None, t=0):
    xa = None if x is None else np.ascontiguousarray(x, dtype=np.float32)
    ya = None if y is None else np.ascontiguousarray(y, dtype=np.float32)
    check(load().qubo_gda_set_state(ctx.h, _ptr(xa), _ptr(ya), int(t)), ctx.h)


def qubo_gda_restart(ctx: Context, x0=None):
    """x0 None: the library's generator with the parameters' seed."""
    xa = None
    if x0 is not None:
        xa = np.ascontiguousarray(x0, dtype=np.float64)
        if xa.shape != _xshape(ctx):
            raise ValueError(f"x0 must have shape {_xshape(ctx)}")
    check(load().qubo_gda_restart(ctx.h, _ptr(xa)), ctx.h)


def qubo_gda_objectives(ctx: Context) -> np.ndarray:
    F = np.zeros(ctx.B, dtype=np.int64)
    check(load().qubo_gda_objectives(ctx.h, _ptr(F)), ctx.h)
    return F


def qubo_gda_objectives_f64(ctx: Context) -> np.ndarray:
    F = np.zeros(ctx.B, dtype=np.float64)
    check(load().qubo_gda_objectives_f64(ctx.h, _ptr(F)), ctx.h)
    return F


def qubo_gda_grad(ctx: Context, x) -> np.ndarray:
    xa = np.ascontiguousarray(x, dtype=np.float32)
    G = np.zeros(_xshape(ctx), dtype=np.float32)
    check(load().qubo_gda_grad(ctx.h, _ptr(xa), _ptr(G)), ctx.h)
    return G


def qubo_gda_eval(ctx: Context, xr) -> np.ndarray:
    xa = np.ascontiguousarray(xr, dtype=np.uint8)
    xa = xa.reshape(-1, ctx.n)
    F = np.zeros(xa.shape[0], dtype=np.int64)
    check(load().qubo_gda_eval(ctx.h, _ptr(xa), int(xa.shape[0]), _ptr(F)), ctx.h)
    return F


def qubo_gda_eval_f64(ctx: Context, xr) -> np.ndarray:
    xa = np.ascontiguousarray(xr, dtype=np.uint8)
    xa = xa.reshape(-1, ctx.n)
    F = np.zeros(xa.shape[0], dtype=np.float64)
    check(load().qubo_gda_eval_f64(ctx.h, _ptr(xa), int(xa.shape[0]), _ptr(F)), ctx.h)
    return F


def qubo_gda_eval_noalloc(ctx: Context, xr, F, stream=None):
    """Exact objectives of the rounded rows of the device uint8 tensor xr (nb, n)
    into the device int64 tensor F (nb,), enqueued on the current torch stream
    (or `stream`), with no device allocation by the library."""
    assert xr.is_cuda and F.is_cuda and xr.is_contiguous() and F.is_contiguous()
    assert xr.dim() == 2 and xr.shape[1] == ctx.n and F.shape == (xr.shape[0],)
    s = _current_stream() if stream is None else ctypes.c_void_p(stream.cuda_stream)
    check(load().qubo_gda_eval_noalloc(ctx.h, ctypes.c_void_p(xr.data_ptr()), int(xr.shape[0]),
                                       ctypes.c_void_p(F.data_ptr()), s), ctx.h)
    return F


def qubo_dual_bound(ctx: Context, iters: int, ybar: float = 0.0) -> dict:
    """Certified lower bound on min F from the Lagrangian at y = ybar 1 (valid
    when that Lagrangian is convex); see pdbo.h."""
    lb = ctypes.c_double()
    val = np.zeros(3, dtype=np.float64)
    x = np.zeros(ctx.n, dtype=np.float32)
    check(load().qubo_dual_bound(ctx.h, float(ybar), int(iters), ctypes.byref(lb), _ptr(val), _ptr(x)),
          ctx.h)
    return dict(lower_bound=lb.value, value=float(val[0]), gap=float(val[1]),
                rounding=float(val[2]), x=x)


def qubo_gda_trace(ctx: Context, cap: int = 4096) -> dict:
    t = np.zeros(cap, dtype=np.int64)
    F = np.zeros(cap, dtype=np.int64)
    b = np.zeros(cap, dtype=np.int32)
    sec = np.zeros(cap, dtype=np.float64)
    ln = ctypes.c_int32()
    check(load().qubo_gda_trace(ctx.h, int(cap), _ptr(t), _ptr(F), _ptr(b), _ptr(sec),
                                ctypes.byref(ln)), ctx.h)
    k = ln.value
    return dict(t=t[:k], F=F[:k], b=b[:k], sec=sec[:k])


def qubo_gda_trace_f64(ctx: Context, cap: int = 4096) -> dict:
    t = np.zeros(cap, dtype=np.int64)
    F = np.zeros(cap, dtype=np.float64)
    b = np.zeros(cap, dtype=np.int32)
    sec = np.zeros(cap, dtype=np.float64)
    ln = ctypes.c_int32()
    check(load().qubo_gda_trace_f64(ctx.h, int(cap), _ptr(t), _ptr(F), _ptr(b), _ptr(sec),
                                    ctypes.byref(ln)), ctx.h)
    k = ln.value
    return dict(t=t[:k], F=F[:k], b=b[:k], sec=sec[:k])


def qubo_gda_solve(q, params: dict, x0, T: int, stream=None) -> dict:
    lib, keep = load(), _Keep()
    prob = _qubo_struct(q, keep)
    par = _params_struct(params, x0, keep)
    bx = np.zeros(int(q.n), dtype=np.uint8)
    r = _abi.pdbo_result()
    r.best_x = _ptr(bx)
    check(lib.qubo_gda_solve(ctypes.byref(prob), ctypes.byref(par), int(T),
                             stream if stream is not None else _current_stream(), ctypes.byref(r)))
    return _result_dict(r, bx)


def _batch_arrays(qs, params_list, x0s, keep):
    k = len(qs)
    probs = (_abi.pdbo_qubo * k)(*[_qubo_struct(q, keep) for q in qs])
    pars = (_abi.pdbo_params * k)(*[_params_struct(p, x, keep) for p, x in zip(params_list, x0s)])
    return k, probs, pars


def qubo_gda_batch_init(qs, params_list, x0s, grouped=True, stream=None) -> Context:
    lib, keep = load(), _Keep()
    k, probs, pars = _batch_arrays(qs, params_list, x0s, keep)
    h = ctypes.c_void_p()
    check(lib.qubo_gda_batch_init(k, probs, pars, int(bool(grouped)),
                                  stream if stream is not None else _current_stream(),
                                  ctypes.byref(h)))
    return Context(h, int(qs[0].n), int(params_list[0]["B"]), "batch", k, [int(q.n) for q in qs])


def qubo_gda_batch_result(ctx: Context, inst: int) -> dict:
    bx = np.zeros(ctx.ns[inst], dtype=np.uint8)
    r = _abi.pdbo_result()
    r.best_x = _ptr(bx)
    check(load().qubo_gda_batch_result(ctx.h, int(inst), ctypes.byref(r)), ctx.h)
    return _result_dict(r, bx)


def qubo_gda_batch_solve(qs, params_list, x0s, T: int, grouped=True, stream=None) -> list:
    lib, keep = load(), _Keep()
    k, probs, pars = _batch_arrays(qs, params_list, x0s, keep)
    bxs = [np.zeros(int(q.n), dtype=np.uint8) for q in qs]
    res = (_abi.pdbo_result * k)()
    for i in range(k):
        res[i].best_x = _ptr(bxs[i])
    check(lib.qubo_gda_batch_solve(k, probs, pars, int(T), int(bool(grouped)),
                                   stream if stream is not None else _current_stream(), res))
    return [_result_dict(res[i], bxs[i]) for i in range(k)]


def kcut_gda_init(graph, params: dict, x0=None, stream=None) -> Context:
    """graph: n, k, symmetric CSR row_ptr / col_idx / w (int32); x0: (B, n, k)
    logits or None (the library's generator)."""
    lib, keep = load(), _Keep()
    g = _abi.pdbo_kcut()
    g.n, g.k = int(graph.n), int(graph.k)
    g.row_ptr = _ptr(keep.arr(graph.row_ptr, np.int32))
    col = keep.arr(graph.col_idx, np.int32)
    g.col_idx = _ptr(col)
    g.w = _ptr(keep.arr(graph.w, np.int32))
    g.nnz = int(len(col))
    par = _params_struct(params, x0, keep)
    h = ctypes.c_void_p()
    check(lib.kcut_gda_init(ctypes.byref(g), ctypes.byref(par),
                            stream if stream is not None else _current_stream(), ctypes.byref(h)))
    return Context(h, int(graph.n), int(params["B"]), "kcut", k=int(graph.k))


def maxsat_gda_init(f, params: dict, x0, stream=None) -> Context:
    lib, keep = load(), _Keep()
    prob = _maxsat_struct(f, keep)
    par = _params_struct(params, x0, keep)
    h = ctypes.c_void_p()
    check(lib.maxsat_gda_init(ctypes.byref(prob), ctypes.byref(par),
                              stream if stream is not None else _current_stream(), ctypes.byref(h)))
    return Context(h, int(f.n), int(params["B"]), "maxsat")


def maxsat_gda_step(ctx: Context, nsteps: int):
    check(load().maxsat_gda_step(ctx.h, int(nsteps)), ctx.h)


def maxsat_gda_result(ctx: Context) -> dict:
    return qubo_gda_result(ctx)


def maxsat_gda_solve(f, params: dict, x0, T: int, stream=None) -> dict:
    lib, keep = load(), _Keep()
    prob = _maxsat_struct(f, keep)
    par = _params_struct(params, x0, keep)
    bx = np.zeros(int(f.n), dtype=np.uint8)
    r = _abi.pdbo_result()
    r.best_x = _ptr(bx)
    check(lib.maxsat_gda_solve(ctypes.byref(prob), ctypes.byref(par), int(T),
                               stream if stream is not None else _current_stream(), ctypes.byref(r)))
    return _result_dict(r, bx)


def _dev_f32(t):
    import torch
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError("expected a contiguous float32 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def maxsat_lagrangian_fwd(ctx: Context, x, y):
    """L[b] = f(x_b)/s + sum_i y_bi g(x_bi) for (nb, n) float32 GPU tensors."""
    import torch
    L = torch.empty(x.shape[0], device=x.device, dtype=torch.float32)
    stream = ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    check(load().maxsat_lagrangian_fwd(ctx.h, _dev_f32(x), _dev_f32(y), int(x.shape[0]),
                                       _dev_f32(L), stream), ctx.h)
    return L


def maxsat_lagrangian_bwd(ctx: Context, x, y, dL):
    import torch
    dx = torch.empty_like(x)
    dy = torch.empty_like(y)
    stream = ctypes.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    check(load().maxsat_lagrangian_bwd(ctx.h, _dev_f32(x), _dev_f32(y), _dev_f32(dL),
                                       int(x.shape[0]), _dev_f32(dx), _dev_f32(dy), stream), ctx.h)
    return dx, dy


def _autograd_class():
    import torch

    class _MaxSATLagrangian(torch.autograd.Function):
        """L(x, y) of a MaxSAT context with the hand-written HIP adjoint as backward."""

        @staticmethod
        def forward(fctx, x, y, pctx):
            x = x.contiguous()
            y = y.contiguous()
            fctx.save_for_backward(x, y)
            fctx.pctx = pctx
            return maxsat_lagrangian_fwd(pctx, x, y)

        @staticmethod
        def backward(fctx, dL):
            x, y = fctx.saved_tensors
            dx, dy = maxsat_lagrangian_bwd(fctx.pctx, x, y, dL.contiguous().float())
            return dx, dy, None

    return _MaxSATLagrangian


class _LazyAutograd:
    _cls = None

    def apply(self, x, y, pctx):
        if _LazyAutograd._cls is None:
            _LazyAutograd._cls = _autograd_class()
        return _LazyAutograd._cls.apply(x, y, pctx)


MaxSATLagrangian = _LazyAutograd()
