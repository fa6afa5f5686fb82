"""Python binding of librm.so: argument marshalling only.

Each function has the name of the C entry point it calls (include/rm.h) and takes
torch CUDA (HIP) tensors for the device pointers.  Shapes, dtypes, devices and
contiguity are checked here; every computation happens in the HIP kernels.
"""
import ctypes
import weakref

import numpy as np
import torch

from . import _lib
from ._lib import (RM_EDIVERGED, RM_ENOTCONV, RM_F32, RM_F64, RM_FD5_HELMHOLTZ, RM_MOM, RM_NAG, RM_NAGEX,
                   RM_OK, RM_Q1_ANISO, RM_RICHARDSON, RM_TO_TOL, RM_UNROLL)

STREAM_SHAPE = 9  # kernel shape id of the row-streaming sweep (rm_plan_set_kernel)

__all__ = [
    "RMError", "Context", "Plan", "rm_tune", "rm_apply_A", "rm_residual", "rm_solve", "rm_solve_adjoint",
    "rm_twogrid_solve", "rm_twogrid_adjoint", "rm_fgmres",
    "rm_meta_forward", "rm_meta_backward", "rm_meta_param_count", "solve_opts",
    "rm_symbolnet_param_count", "rm_symbolnet_forward", "rm_symbolnet_backward",
    "RM_Q1_ANISO", "RM_FD5_HELMHOLTZ", "RM_RICHARDSON", "RM_NAG", "RM_MOM", "RM_NAGEX", "RM_F32", "RM_F64",
    "RM_UNROLL", "RM_TO_TOL", "RM_OK", "RM_ENOTCONV", "RM_EDIVERGED",
]


class RMError(RuntimeError):
    def __init__(self, status, where):
        lib = _lib.load()
        msg = lib.rm_last_error().decode()
        super().__init__(f"{where}: {lib.rm_status_string(status).decode()} ({msg})")
        self.status = status


def _check(status, where):
    if status != RM_OK:
        raise RMError(status, where)


_DT = {torch.float32: RM_F32, torch.float64: RM_F64}


def _ptr(t, dtype=None, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """rm_create / rm_destroy; enqueues on the given (default: current) torch stream."""

    def __init__(self, device=0, stream=None):
        self.lib = _lib.load()
        dev = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(dev)
        self.stream = stream
        self.device = device
        h = ctypes.c_void_p()
        _check(self.lib.rm_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)), "rm_create")
        self.handle = h
        self._plans = weakref.WeakSet()

    def close(self):
        """Free the context's remaining plans, then the context itself."""
        if getattr(self, "handle", None):
            for plan in list(getattr(self, "_plans", ())):
                plan.close()
            self.lib.rm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Plan:
    """rm_plan: a batch of instances.  ``n`` list of sizes; Q1 instances take eps and
    theta, Helmholtz instances take kappa."""

    def __init__(self, ctx, n, eps=None, theta=None, kappa=None, op=RM_Q1_ANISO, offsets=None):
        """offsets: optional B + 1 element offsets of the instances in every vector
        (rm_plan; None = packed back to back)."""
        self.ctx = ctx
        self.lib = ctx.lib
        B = len(n)
        arr = (_lib.rm_instance * B)()
        for b in range(B):
            arr[b].n = int(n[b])
            arr[b].op = op
            arr[b].eps = float(eps[b]) if eps is not None else 1.0
            arr[b].theta = float(theta[b]) if theta is not None else 0.0
            arr[b].kappa = float(kappa[b]) if kappa is not None else 0.0
        off_in = None
        if offsets is not None:
            if len(offsets) != B + 1:
                raise ValueError(f"offsets must have {B + 1} entries")
            off_in = (ctypes.c_int64 * (B + 1))(*[int(o) for o in offsets])
        h = ctypes.c_void_p()
        _check(self.lib.rm_plan(ctx.handle, B, arr, off_in, ctypes.byref(h)), "rm_plan")
        self.handle = h
        ctx._plans.add(self)
        self.B = B
        self.n = [int(k) for k in n]
        self.P = int(self.lib.rm_plan_points(h))
        off = (ctypes.c_int64 * (B + 1))()
        _check(self.lib.rm_plan_offsets(h, off), "rm_plan_offsets")
        self.offsets = np.frombuffer(off, dtype=np.int64).copy()

    def set_kernel(self, shape, T, n=0, cw=0):
        """rm_plan_set_kernel: (variant, T, tile width) for the size class n (n <= 0: all);
        shape -1 = one launch per inner step; shape STREAM_SHAPE = the row-streaming
        kernel, whose cw is the height of its row windows; cw <= 0 = the cost model's
        width."""
        _check(self.lib.rm_plan_set_kernel(self.handle, n, shape, T, cw), "rm_plan_set_kernel")

    def get_kernel(self, n):
        sh, T, cw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.rm_plan_get_kernel(self.handle, n, ctypes.byref(sh), ctypes.byref(T), ctypes.byref(cw)),
               "rm_plan_get_kernel")
        return sh.value, T.value, cw.value

    def set_tail_kernel(self, shape, T, n=0, cw=0):
        """rm_plan_set_tail_kernel: the configuration the refined solve switches to once
        few instances are still active."""
        _check(self.lib.rm_plan_set_tail_kernel(self.handle, n, shape, T, cw), "rm_plan_set_tail_kernel")

    def get_tail_kernel(self, n):
        sh, T, cw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self.lib.rm_plan_get_tail_kernel(self.handle, n, ctypes.byref(sh), ctypes.byref(T),
                                                ctypes.byref(cw)), "rm_plan_get_tail_kernel")
        return sh.value, T.value, cw.value

    def set_tail_switch(self, frac):
        """rm_plan_set_tail_switch: active fraction below which the tails run (< 0: measured)."""
        _check(self.lib.rm_plan_set_tail_switch(self.handle, float(frac)), "rm_plan_set_tail_switch")

    def set_mixed(self, on):
        """rm_plan_set_mixed: advance every class that runs the 8-step row pipeline in one
        launch per chunk of steps (same results as one launch per class)."""
        _check(self.lib.rm_plan_set_mixed(self.handle, 1 if on else 0), "rm_plan_set_mixed")

    def get_mixed(self):
        on = ctypes.c_int32()
        _check(self.lib.rm_plan_get_mixed(self.handle, ctypes.byref(on)), "rm_plan_get_mixed")
        return bool(on.value)

    def coarse_points(self):
        """rm_plan_coarse_points: total coarse points of the two-grid cycle (-1 if the
        plan's sizes do not qualify)."""
        return int(self.lib.rm_plan_coarse_points(self.handle))

    def coarse_offsets(self):
        off = (ctypes.c_int64 * self.B)()
        _check(self.lib.rm_plan_coarse_offsets(self.handle, off), "rm_plan_coarse_offsets")
        return np.frombuffer(off, dtype=np.int64).copy()

    def coefficients(self):
        c = (ctypes.c_double * (5 * self.B))()
        g = (ctypes.c_double * self.B)()
        _check(self.lib.rm_plan_coefficients(self.handle, c, g), "rm_plan_coefficients")
        return np.frombuffer(c).reshape(self.B, 5).copy(), np.frombuffer(g).copy()

    def close(self):
        if getattr(self, "handle", None):
            self.lib.rm_plan_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_opts(mode=RM_UNROLL, dtype=RM_F32, m=16, K=0, ckpt_every=0, max_outer=100000, max_rounds=8,
               check_every=4, tol=1e-10, tol_inner=1e-3, graph=False, jacobi=False, ssor=None, hist_len=0):
    """rm_solve_opts; ssor = the SSOR relaxation factor (None: no SSOR preconditioning);
    hist_len = rows of the refined solve's per-outer-iteration history."""
    o = _lib.rm_solve_opts()
    o.mode, o.dtype, o.m, o.K, o.ckpt_every = mode, dtype, m, K, ckpt_every
    o.max_outer, o.max_rounds, o.check_every = max_outer, max_rounds, check_every
    o.flags = ((_lib.RM_FLAG_GRAPH if graph else 0) | (_lib.RM_FLAG_JACOBI if jacobi else 0)
               | (_lib.RM_FLAG_SSOR if ssor is not None else 0))
    o.hist_len = hist_len
    o.tol, o.tol_inner = tol, tol_inner
    o.relax = 1.0 if ssor is None else float(ssor)
    return o


def rm_tune(ctx, plan, method, m, omega, alpha, b, cache_path=None):
    """Autotune every size class of the plan on its data; returns the summed us per step."""
    us = ctypes.c_double()
    na = 2 if method == RM_NAGEX else 1
    _check(ctx.lib.rm_tune(ctx.handle, plan.handle, method, m, _ptr(omega, torch.float32, plan.B * m, "omega"),
                           _ptr(alpha, torch.float32, na * plan.B * m, "alpha") if alpha is not None else None,
                           _ptr(b, torch.float32, plan.P, "b"),
                           cache_path.encode() if cache_path else None, ctypes.byref(us)), "rm_tune")
    return us.value


def rm_apply_A(ctx, plan, x, y):
    dt = _DT[x.dtype]
    _check(ctx.lib.rm_apply_A(ctx.handle, plan.handle, dt, _ptr(x, x.dtype, plan.P, "x"),
                              _ptr(y, x.dtype, plan.P, "y")), "rm_apply_A")
    return y


def rm_residual(ctx, plan, b, x, r=None, r2=None, b2=None, rel2=None):
    dt = _DT[b.dtype]
    _check(ctx.lib.rm_residual(ctx.handle, plan.handle, dt, _ptr(b, b.dtype, plan.P, "b"),
                               _ptr(x, b.dtype, plan.P, "x"), _ptr(r, b.dtype, plan.P, "r"),
                               _ptr(r2, torch.float64, plan.B, "r2"), _ptr(b2, torch.float64, plan.B, "b2"),
                               _ptr(rel2, torch.float32, plan.B, "rel2")), "rm_residual")


def rm_solve(ctx, plan, method, opts, omega, alpha, b, x, ckpt=None, hist=None):
    """UNROLL: returns None (asynchronous).  TO_TOL: blocks and returns a dict of
    per-instance numpy arrays (outer_iters, rounds, relres, inst_status and history
    [max_rounds + 1, B]) plus 'status'; hist (TO_TOL) is a device double tensor of
    opts.hist_len * B elements."""
    m = opts.m
    na = 2 if method == RM_NAGEX else 1
    om = _ptr(omega, torch.float32, plan.B * m, "omega")
    al = _ptr(alpha, torch.float32, na * plan.B * m, "alpha") if alpha is not None else None
    if opts.mode == RM_UNROLL:
        vdt = torch.float32 if opts.dtype == RM_F32 else torch.float64
        ck = None
        if ckpt is not None:
            ck = _ptr(ckpt, vdt, (opts.K // opts.ckpt_every) * 2 * plan.P, "ckpt")
        hs = _ptr(hist, torch.float64, (opts.K // m) * plan.B, "hist") if hist is not None else None
        st = ctx.lib.rm_solve(ctx.handle, plan.handle, method, ctypes.byref(opts), om, al,
                              _ptr(b, vdt, plan.P, "b"), _ptr(x, vdt, plan.P, "x"), ck, hs, None)
        _check(st, "rm_solve")
        return None
    B = plan.B
    outer = (ctypes.c_int32 * B)()
    rounds = (ctypes.c_int32 * B)()
    relres = (ctypes.c_double * B)()
    status = (ctypes.c_int32 * B)()
    nh = (opts.max_rounds + 1) * B
    history = (ctypes.c_double * nh)()
    rep = _lib.rm_report(outer, rounds, relres, status, history)
    hs = _ptr(hist, torch.float64, opts.hist_len * B, "hist") if hist is not None else None
    st = ctx.lib.rm_solve(ctx.handle, plan.handle, method, ctypes.byref(opts), om, al,
                          _ptr(b, torch.float64, plan.P, "b"), _ptr(x, torch.float64, plan.P, "x"),
                          None, hs, ctypes.byref(rep))
    if st not in (RM_OK, RM_ENOTCONV, RM_EDIVERGED):
        _check(st, "rm_solve")
    return {
        "status": st,
        "outer_iters": np.frombuffer(outer, dtype=np.int32).copy(),
        "rounds": np.frombuffer(rounds, dtype=np.int32).copy(),
        "relres": np.frombuffer(relres, dtype=np.float64).copy(),
        "inst_status": np.frombuffer(status, dtype=np.int32).copy(),
        "history": np.frombuffer(history, dtype=np.float64).reshape(opts.max_rounds + 1, B).copy(),
    }


def rm_solve_adjoint(ctx, plan, method, opts, omega, alpha, b, ckpt, d_omega, d_alpha, g_uK=None,
                     g_loss=None, d_b=None, loss=None):
    m = opts.m
    P, B = plan.P, plan.B
    na = 2 if method == RM_NAGEX else 1
    st = ctx.lib.rm_solve_adjoint(
        ctx.handle, plan.handle, method, ctypes.byref(opts),
        _ptr(omega, torch.float32, B * m, "omega"),
        _ptr(alpha, torch.float32, na * B * m, "alpha") if alpha is not None else None,
        _ptr(b, torch.float32, P, "b"),
        _ptr(ckpt, torch.float32, (opts.K // opts.ckpt_every) * 2 * P, "ckpt"),
        _ptr(g_uK, torch.float32, P, "g_uK"), _ptr(g_loss, torch.float32, B, "g_loss"),
        _ptr(d_omega, torch.float32, B * m, "d_omega"), _ptr(d_alpha, torch.float32, na * B * m, "d_alpha"),
        _ptr(d_b, torch.float32, P, "d_b"), _ptr(loss, torch.float32, B, "loss"))
    _check(st, "rm_solve_adjoint")


def rm_twogrid_solve(ctx, plan, method, opts, omega, alpha, symbol, b, x, ckpt=None, hist=None):
    """K = opts.K two-grid cycles in FP32 from u = x (asynchronous)."""
    m, K, P, B = opts.m, opts.K, plan.P, plan.B
    na = 2 if method == RM_NAGEX else 1
    Pc = plan.coarse_points()
    st = ctx.lib.rm_twogrid_solve(
        ctx.handle, plan.handle, method, ctypes.byref(opts),
        _ptr(omega, torch.float32, B * m, "omega"),
        _ptr(alpha, torch.float32, na * B * m, "alpha") if alpha is not None else None,
        _ptr(symbol, torch.float32, Pc, "symbol"), _ptr(b, torch.float32, P, "b"), _ptr(x, torch.float32, P, "x"),
        _ptr(ckpt, torch.float32, K * P, "ckpt"), _ptr(hist, torch.float64, K * B, "hist"))
    _check(st, "rm_twogrid_solve")


def rm_twogrid_adjoint(ctx, plan, method, opts, omega, alpha, symbol, b, ckpt, d_omega, d_alpha, d_symbol,
                       g_uK=None, g_loss=None, d_b=None, loss=None):
    m, K, P, B = opts.m, opts.K, plan.P, plan.B
    na = 2 if method == RM_NAGEX else 1
    Pc = plan.coarse_points()
    st = ctx.lib.rm_twogrid_adjoint(
        ctx.handle, plan.handle, method, ctypes.byref(opts),
        _ptr(omega, torch.float32, B * m, "omega"),
        _ptr(alpha, torch.float32, na * B * m, "alpha") if alpha is not None else None,
        _ptr(symbol, torch.float32, Pc, "symbol"), _ptr(b, torch.float32, P, "b"),
        _ptr(ckpt, torch.float32, K * P, "ckpt"),
        _ptr(g_uK, torch.float32, P, "g_uK"), _ptr(g_loss, torch.float32, B, "g_loss"),
        _ptr(d_omega, torch.float32, B * m, "d_omega"), _ptr(d_alpha, torch.float32, na * B * m, "d_alpha"),
        _ptr(d_symbol, torch.float32, Pc, "d_symbol"), _ptr(d_b, torch.float32, P, "d_b"),
        _ptr(loss, torch.float32, B, "loss"))
    _check(st, "rm_twogrid_adjoint")


def rm_fgmres(ctx, plan, b, x, restart=20, max_iter=200, tol=1e-6, method=RM_NAG, inner=None, omega=None,
              alpha=None, symbol=None):
    """Batched FGMRES; blocks and returns the per-instance report like rm_solve(TO_TOL)."""
    B = plan.B
    fo = _lib.rm_fgmres_opts(restart, max_iter, tol)
    om = al = sy = None
    if inner is not None:
        m = inner.m
        na = 2 if method == RM_NAGEX else 1
        om = _ptr(omega, torch.float32, B * m, "omega")
        al = _ptr(alpha, torch.float32, na * B * m, "alpha") if alpha is not None else None
        sy = _ptr(symbol, torch.float32, plan.coarse_points(), "symbol") if symbol is not None else None
    outer = (ctypes.c_int32 * B)()
    rounds = (ctypes.c_int32 * B)()
    relres = (ctypes.c_double * B)()
    status = (ctypes.c_int32 * B)()
    rep = _lib.rm_report(outer, rounds, relres, status, None)
    st = ctx.lib.rm_fgmres(ctx.handle, plan.handle, ctypes.byref(fo), method,
                           ctypes.byref(inner) if inner is not None else None, om, al, sy,
                           _ptr(b, torch.float64, plan.P, "b"), _ptr(x, torch.float64, plan.P, "x"),
                           ctypes.byref(rep))
    if st not in (RM_OK, RM_ENOTCONV, RM_EDIVERGED):
        _check(st, "rm_fgmres")
    return {
        "status": st,
        "outer_iters": np.frombuffer(outer, dtype=np.int32).copy(),
        "rounds": np.frombuffer(rounds, dtype=np.int32).copy(),
        "relres": np.frombuffer(relres, dtype=np.float64).copy(),
        "inst_status": np.frombuffer(status, dtype=np.int32).copy(),
    }


def rm_meta_param_count(m):
    return int(_lib.load().rm_meta_param_count(m))


def rm_meta_forward(ctx, plan, m, params, omega, alpha):
    _check(ctx.lib.rm_meta_forward(ctx.handle, plan.handle, m,
                                   _ptr(params, torch.float32, rm_meta_param_count(m), "params"),
                                   _ptr(omega, torch.float32, plan.B * m, "omega"),
                                   _ptr(alpha, torch.float32, plan.B * m, "alpha")), "rm_meta_forward")


def rm_meta_backward(ctx, plan, m, params, d_omega, d_alpha, d_params):
    npar = rm_meta_param_count(m)
    _check(ctx.lib.rm_meta_backward(ctx.handle, plan.handle, m, _ptr(params, torch.float32, npar, "params"),
                                    _ptr(d_omega, torch.float32, plan.B * m, "d_omega"),
                                    _ptr(d_alpha, torch.float32, plan.B * m, "d_alpha"),
                                    _ptr(d_params, torch.float32, npar, "d_params")), "rm_meta_backward")


def rm_symbolnet_param_count():
    return int(_lib.load().rm_symbolnet_param_count())


def rm_symbolnet_forward(ctx, plan, params, symbol):
    """symbol (device float [Pc]) of every instance from the symbol network's params."""
    _check(ctx.lib.rm_symbolnet_forward(ctx.handle, plan.handle,
                                        _ptr(params, torch.float32, rm_symbolnet_param_count(), "params"),
                                        _ptr(symbol, torch.float32, plan.coarse_points(), "symbol")),
           "rm_symbolnet_forward")


def rm_symbolnet_backward(ctx, plan, params, d_symbol, d_params):
    npar = rm_symbolnet_param_count()
    _check(ctx.lib.rm_symbolnet_backward(ctx.handle, plan.handle, _ptr(params, torch.float32, npar, "params"),
                                         _ptr(d_symbol, torch.float32, plan.coarse_points(), "d_symbol"),
                                         _ptr(d_params, torch.float32, npar, "d_params")),
           "rm_symbolnet_backward")
