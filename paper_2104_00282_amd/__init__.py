"""MI355X price discovery for fungible resource allocation.

Python face of the C ABI in include/resalloc.h.  PyTorch supplies device
memory only; every step of the method runs in libresalloc.so (gfx950 HIP).
``_capi`` holds the ctypes declarations under the C names; ``Context`` and
``Problem`` below are conveniences that marshal torch tensors into them.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref

import numpy as np

from . import _capi
from ._capi import (RA_EDEVICE, RA_EINVAL, RA_ENOMEM, RA_ENOTCONV, RA_ENUMERIC, RA_EUNSUPPORTED,
                    RA_F32, RA_F64, RA_OK, RA_UTIL_ALPHA_FAIR, RA_UTIL_CAPLIN, RA_UTIL_LOG,
                    RAError, ra_create,
                    ra_destroy, ra_dual_eval, ra_get_allocation, ra_last_error, ra_problem_create,
                    ra_problem_destroy, ra_solve, ra_solve_info, ra_solve_opts,
                    ra_solve_opts_default, ra_status_string, ra_set_kernel_timing,
                    ra_get_kernel_timing, ra_batch_solve, ra_stream_read_ms,
                    ra_probe_first_vertex_ms,
                    ra_batch_set_shape, ra_batch_tuning)

__all__ = [
    "Context", "Problem", "RAError", "ra_create", "ra_destroy", "ra_status_string",
    "ra_last_error", "ra_problem_create", "ra_problem_destroy", "ra_dual_eval",
    "ra_solve_opts_default", "ra_solve", "ra_get_allocation", "ra_solve_opts", "ra_solve_info",
    "ra_set_kernel_timing", "ra_get_kernel_timing", "ra_batch_solve", "batch_solve", "MLP",
    "ra_stream_read_ms", "ra_probe_first_vertex_ms", "ra_batch_set_shape", "ra_batch_tuning",
]


# Handles still open at interpreter exit are closed before torch and the HIP
# runtime are torn down (problems first, then contexts).
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    objs = list(_LIVE)
    for o in objs:
        if not isinstance(o, Context):
            o.close()
    for o in objs:
        o.close()


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _hbuf(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Context:
    """A library context on one HIP device with its own stream."""

    def __init__(self, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        self.device = device
        self.handle = ra_create(device, None)
        _LIVE.add(self)

    def set_batch_shape(self, tile_floats, rows=(0, 0, 0, 0), blocks_per_cu=0):
        """Fix the batched launch shape (tile_floats 0: back to the autotuner)."""
        ra_batch_set_shape(self.handle, tile_floats, rows, blocks_per_cu)

    def batch_tuning(self):
        """The autotuner's record of its last tuning (dict; {} if none)."""
        import json
        txt = ra_batch_tuning(self.handle)
        return json.loads(txt) if txt else {}

    def close(self):
        if self.handle:
            ra_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    """A resource allocation problem on the device (tensors are kept alive).

    T: (n, m) float32/float64 CUDA tensor; w, c: (n,) of T's dtype; kind:
    (n,) uint8 (0 = log, 1 = capped linear) or None; R: m limits.
    """

    def __init__(self, ctx, T, w, c=None, kind=None, R=None, eps=1e-3, validate=True):
        import torch
        if T.dim() != 2 or not T.is_cuda:
            raise ValueError("T must be a 2-D device tensor")
        if T.dtype not in (torch.float32, torch.float64):
            raise TypeError("T must be float32 or float64")
        self.ctx = ctx
        self.T = T.contiguous()
        self.n, self.m = self.T.shape
        self.dtype = self.T.dtype
        self.w = w.to(self.dtype).contiguous()
        self.c = None if c is None else c.to(self.dtype).contiguous()
        self.kind = None if kind is None else kind.to(torch.uint8).contiguous()
        self.R = np.ascontiguousarray(np.asarray(R, dtype=np.float64))
        self.eps = float(eps)
        torch.cuda.synchronize(self.T.device)
        self.handle = ra_problem_create(
            ctx.handle, self.n, self.m, RA_F32 if self.dtype == torch.float32 else RA_F64,
            _dptr(self.T), _dptr(self.w), _dptr(self.c), _dptr(self.kind), _hbuf(self.R),
            self.eps, 1 if validate else 0)
        _LIVE.add(self)

    def close(self):
        if getattr(self, "handle", None):
            ra_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dual_eval(self, p, lower_bound=False, support=False, j1=False):
        """g(p), grad = R - r, and optionally U(X~), the per-job support
        (j_pair int16 (n, 2), x_pair (n, 2)) and the first vertex j1 (n,)."""
        import torch
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
        g = ctypes.c_double()
        grad = np.zeros(self.m)
        lb = ctypes.c_double() if lower_bound else None
        dev = self.T.device
        jp = torch.empty((self.n, 2), dtype=torch.int16, device=dev) if support else None
        xp = torch.empty((self.n, 2), dtype=self.dtype, device=dev) if support else None
        jv = torch.empty(self.n, dtype=torch.int16, device=dev) if j1 else None
        ra_dual_eval(self.ctx.handle, self.handle, _hbuf(p), ctypes.byref(g), _hbuf(grad),
                     ctypes.byref(lb) if lb is not None else None, _dptr(jp), _dptr(xp),
                     _dptr(jv))
        out = {"g": g.value, "grad": grad, "r": self.R - grad}
        if lb is not None:
            out["lower_bound"] = lb.value
        if support:
            out["j_pair"], out["x_pair"] = jp, xp
        if j1:
            out["j1"] = jv
        return out

    def solve(self, p0=None, tol_rel=1e-6, max_iter=500, lbfgs_mem=10, method=0, use_graph=True,
              verbose=False, max_evals=0, stall_evals=0, init_step=0.0, paper_init=False,
              tol_abs=0.0, device_loop=False, stall_restarts=0):
        """Price discovery; returns (p, info dict, status).  paper_init starts
        from the paper's data-dependent prices (ra_init_prices) unless p0 is
        given."""
        o = ra_solve_opts_default()
        o.stall_restarts = stall_restarts
        o.init_step = init_step
        o.tol_abs = tol_abs
        o.device_loop = 1 if device_loop else 0
        o.max_evals = max_evals
        o.stall_evals = stall_evals
        o.tol_rel = tol_rel
        o.max_iter = max_iter
        o.lbfgs_mem = lbfgs_mem
        o.method = method
        o.use_graph = 1 if use_graph else 0
        o.verbose = 1 if verbose else 0
        p = np.ones(self.m)
        if p0 is not None:
            p = np.ascontiguousarray(np.asarray(p0, dtype=np.float64)).copy()
            o.init = 1
        elif paper_init:
            o.init = 2
        info = ra_solve_info()
        st = ra_solve(self.ctx.handle, self.handle, o, _hbuf(p), info)
        return p, {f: getattr(info, f) for f, _ in ra_solve_info._fields_}, st

    def features(self):
        """Warm-start feature vector (8 m + 16 floats, device tensor)."""
        import torch
        f = torch.empty(8 * self.m + 16, dtype=torch.float32, device=self.T.device)
        _capi.check(self.ctx.handle, _capi.lib().ra_features(self.ctx.handle, self.handle, _dptr(f)))
        return f

    def set_demands(self, d):
        """Per-job demands d (device tensor of the problem's dtype, n values
        > 0), or None to remove them (ra_problem_set_demands)."""
        if d is not None:
            d = d.to(self.dtype).contiguous()
            self._demands = d
        else:
            self._demands = None
        _capi.check(self.ctx.handle, _capi.lib().ra_problem_set_demands(
            self.ctx.handle, self.handle, _dptr(d) if d is not None else None))

    def set_demand_vectors(self, D):
        """Per-job demand vectors D (device tensor of the problem's dtype,
        n x m, entries > 0), or None to remove them
        (ra_problem_set_demand_vectors).  The library borrows D: the problem
        keeps a reference to it until it is replaced or removed."""
        if D is not None:
            D = D.to(self.dtype).contiguous()
            if tuple(D.shape) != (self.n, self.m):
                raise ValueError("demand vectors must have shape (n, m)")
        _capi.check(self.ctx.handle, _capi.lib().ra_problem_set_demand_vectors(
            self.ctx.handle, self.handle, _dptr(D) if D is not None else None))
        self._demand_vectors = D

    def init_prices(self):
        """The paper's data-dependent starting prices (ra_init_prices)."""
        p = np.zeros(self.m)
        _capi.check(self.ctx.handle, _capi.lib().ra_init_prices(self.ctx.handle, self.handle,
                                                                _hbuf(p)))
        return p

    def predict_prices(self, mlp):
        """Starting prices predicted by the network (ra_predict_prices)."""
        p = np.zeros(self.m)
        _capi.check(self.ctx.handle, _capi.lib().ra_predict_prices(self.ctx.handle, self.handle,
                                                                   mlp.handle, _hbuf(p)))
        return p

    def solve_learned(self, mlp, tol_rel=1e-6, max_iter=500, lbfgs_mem=10, use_graph=True,
                      max_evals=0, stall_evals=0, fallback_window=5, init_step=0.0,
                      stall_restarts=0, warm_stall_restarts=-1, warm_stall_evals=0):
        """Price discovery from the network's predicted prices (ra_solve_learned).
        warm_stall_restarts >= 0: the warm run's own stall restarts, after which
        a warm run that stalls short of tol_rel is followed by a solve from
        p = 1 (info["restarted"] == 2); warm_stall_evals > 0: the warm run's
        own stall window."""
        o = ra_solve_opts_default()
        o.stall_restarts = stall_restarts
        o.warm_stall_restarts = warm_stall_restarts
        o.warm_stall_evals = warm_stall_evals
        o.init_step = init_step
        o.tol_rel = tol_rel
        o.max_iter = max_iter
        o.lbfgs_mem = lbfgs_mem
        o.use_graph = 1 if use_graph else 0
        o.max_evals = max_evals
        o.stall_evals = stall_evals
        p = np.zeros(self.m)
        info = ra_solve_info()
        st = _capi.lib().ra_solve_learned(self.ctx.handle, self.handle, mlp.handle,
                                         ctypes.byref(o), fallback_window, _hbuf(p),
                                         ctypes.byref(info))
        _capi.check(self.ctx.handle, st, (RA_OK, RA_ENOTCONV))
        return p, {f: getattr(info, f) for f, _ in ra_solve_info._fields_}, st

    def allocation(self, p):
        """Dense feasible allocation X~ (n, m) at prices p."""
        import torch
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float64))
        X = torch.empty((self.n, self.m), dtype=self.dtype, device=self.T.device)
        ra_get_allocation(self.ctx.handle, self.handle, _hbuf(p), _dptr(X))
        return X


def batch_solve(problems, p0=None, tol_rel=1e-6, tol_each=None, max_iter=500, lbfgs_mem=10,
                method=0, use_graph=True, max_evals=0, stall_evals=0, init_step=0.0,
                paper_init=False, tol_abs=0.0, stall_restarts=0):
    """Solve several Problems of one Context together (ra_batch_solve).
    Returns (list of price arrays, list of info dicts, status)."""
    if not problems:
        raise ValueError("no problems")
    ctx = problems[0].ctx
    B = len(problems)
    o = ra_solve_opts_default()
    o.tol_rel = tol_rel
    o.max_iter = max_iter
    o.lbfgs_mem = lbfgs_mem
    o.method = method
    o.use_graph = 1 if use_graph else 0
    o.max_evals = max_evals
    o.stall_evals = stall_evals
    o.init_step = init_step
    o.tol_abs = tol_abs
    o.stall_restarts = stall_restarts
    ms = [pr.m for pr in problems]
    offs = np.concatenate([[0], np.cumsum(ms)]).astype(np.int64)
    p = np.ones(int(offs[-1]))
    if p0 is not None:
        for b, pb in enumerate(p0):
            p[offs[b]:offs[b + 1]] = np.asarray(pb, dtype=np.float64)
        o.init = 1
    elif paper_init:
        o.init = 2
    handles = (ctypes.c_void_p * B)(*[pr.handle for pr in problems])
    infos = (ra_solve_info * B)()
    tol = None
    if tol_each is not None:
        tol = np.ascontiguousarray(np.asarray(tol_each, dtype=np.float64))
    st = ra_batch_solve(ctx.handle, B, handles, o, _hbuf(tol) if tol is not None else None,
                        _hbuf(p), infos)
    out_p = [p[offs[b]:offs[b + 1]].copy() for b in range(B)]
    out_i = [{f: getattr(infos[b], f) for f, _ in ra_solve_info._fields_} for b in range(B)]
    return out_p, out_i, st


class MLP:
    """Warm-start network (ra_mlp_*): in_dim -> hidden -> hidden -> out_dim."""

    def __init__(self, ctx, in_dim, hidden, out_dim, seed=0, handle=None):
        self.ctx = ctx
        self.in_dim, self.hidden, self.out_dim = in_dim, hidden, out_dim
        if handle is None:
            h = ctypes.c_void_p()
            _capi.check(ctx.handle, _capi.lib().ra_mlp_create(ctx.handle, in_dim, hidden, out_dim,
                                                             seed, ctypes.byref(h)))
            handle = h
        self.handle = handle
        _LIVE.add(self)

    @classmethod
    def load(cls, ctx, path):
        h = ctypes.c_void_p()
        _capi.check(ctx.handle, _capi.lib().ra_mlp_load(ctx.handle, path.encode(), ctypes.byref(h)))
        import struct
        with open(path, "rb") as f:
            f.read(8)
            D, H, O = struct.unpack("<3i", f.read(12))
        return cls(ctx, D, H, O, handle=h)

    def save(self, path):
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_save(self.handle, path.encode()))

    def close(self):
        if getattr(self, "handle", None):
            _capi.lib().ra_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def num_params(self):
        k = ctypes.c_int64()
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_num_params(self.handle, ctypes.byref(k)))
        return k.value

    def get_params(self):
        a = np.empty(self.num_params(), dtype=np.float32)
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_get_params(self.handle, _hbuf(a)))
        return a

    def set_params(self, a):
        a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
        assert a.size == self.num_params()
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_set_params(self.handle, _hbuf(a)))

    def set_normalization(self, x_mean, x_std, y_mean, y_std):
        arrs = [np.ascontiguousarray(np.asarray(v, dtype=np.float32))
                for v in (x_mean, x_std, y_mean, y_std)]
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_set_normalization(
            self.handle, *[_hbuf(a) for a in arrs]))

    def forward(self, X):
        import torch
        X = X.to(torch.float32).contiguous()
        Y = torch.empty((X.shape[0], self.out_dim), dtype=torch.float32, device=X.device)
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_forward(self.ctx.handle, self.handle,
                                                               X.shape[0], _dptr(X), _dptr(Y)))
        return Y

    def gradients(self, X, Ty):
        g = np.empty(self.num_params(), dtype=np.float32)
        loss = ctypes.c_double()
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_gradients(
            self.ctx.handle, self.handle, X.shape[0], _dptr(X.contiguous()),
            _dptr(Ty.contiguous()), _hbuf(g), ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, X, Ty, lr):
        loss = ctypes.c_double()
        _capi.check(self.ctx.handle, _capi.lib().ra_mlp_train_step(
            self.ctx.handle, self.handle, X.shape[0], _dptr(X.contiguous()),
            _dptr(Ty.contiguous()), lr, ctypes.byref(loss)))
        return loss.value
