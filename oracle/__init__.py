"""FP64 CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It never touches the HIP library and
the HIP library never touches it.

``oracle.c`` is the slow, plain implementation of the paper's method (see
its header); this module loads it with ctypes (compiling it with gcc first
when the shared object is missing) and wraps it for numpy arrays.
``oracle.brute`` holds independent tiny-case routes (grid search, LP via
scipy, water-filling) that pin the C oracle.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LOG = 0
CAPLIN = 1


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc and OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_p = ctypes.c_void_p


class _Job(ctypes.Structure):
    _fields_ = [("t", _d), ("v", _d), ("jlo", _i32), ("jhi", _i32), ("xlo", _d), ("xhi", _d),
                ("j1", _i32), ("margin1", _d), ("marginx", _d)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol_rel", _d), ("max_iter", _i32), ("mem", _i32), ("method", _i32),
                ("verbose", _i32), ("tol_abs", _d)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", _i32), ("evals", _i32), ("status", _i32), ("g", _d), ("U", _d),
                ("rel_gap", _d)]


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        L.orc_utility.restype = _d
        L.orc_utility.argtypes = [ctypes.c_int, _d, _d, _d, _d]
        L.orc_segment_argmax.restype = _d
        L.orc_segment_argmax.argtypes = [ctypes.c_int, _d, _d, _d, _d, _d, _d]
        L.orc_cost.restype = _d
        L.orc_cost.argtypes = [ctypes.c_int, _p, _p, _d]
        L.orc_subproblem.restype = None
        L.orc_subproblem.argtypes = [ctypes.c_int, _p, _p, ctypes.c_int, _d, _d, _d,
                                     ctypes.POINTER(_Job)]
        L.orc_dual_eval.restype = ctypes.c_int
        L.orc_dual_eval.argtypes = [_i64, ctypes.c_int, ctypes.c_int, _p, _p, _p, _p, _d, _p, _p,
                                    _p, _p, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_lower_bound.restype = _d
        L.orc_lower_bound.argtypes = [_i64, ctypes.c_int, ctypes.c_int, _p, _p, _p, _p, _d, _p,
                                      _p, _p, _p, _p, _p, _p]
        L.orc_solve.restype = ctypes.c_int
        L.orc_solve.argtypes = [_i64, ctypes.c_int, ctypes.c_int, _p, _p, _p, _p, _d, _p,
                                ctypes.POINTER(SolveOpts), _p, ctypes.POINTER(SolveInfo)]
        L.orc_dual_eval_d.restype = ctypes.c_int
        L.orc_dual_eval_d.argtypes = L.orc_dual_eval.argtypes + [_p, ctypes.c_int]
        L.orc_dual_eval_m.restype = ctypes.c_int
        L.orc_dual_eval_m.argtypes = L.orc_dual_eval.argtypes + [_p, _p, ctypes.c_int]
        L.orc_solve_d.restype = ctypes.c_int
        L.orc_solve_d.argtypes = L.orc_solve.argtypes + [_p, ctypes.c_int]
        L.orc_init_prices.restype = ctypes.c_int
        L.orc_init_prices.argtypes = [_i64, ctypes.c_int, ctypes.c_int, _p, _p, _p, _p, _d, _p, _p]
        L.orc_first_vertex.restype = None
        L.orc_first_vertex.argtypes = [_i64, ctypes.c_int, ctypes.c_int, _p, _p, _p]
        L.orc_init_prices_d.restype = ctypes.c_int
        L.orc_init_prices_d.argtypes = L.orc_init_prices.argtypes + [_p, ctypes.c_int]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def utility(kind, w, c, eps, t):
    return lib().orc_utility(int(kind), float(w), float(c), float(eps), float(t))


def segment_argmax(kind, w, c, eps, alpha, gamma, delta):
    return lib().orc_segment_argmax(int(kind), float(w), float(c), float(eps), float(alpha),
                                    float(gamma), float(delta))


def cost(a, p, t):
    a = np.ascontiguousarray(a, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    return lib().orc_cost(len(a), _ptr(a), _ptr(p), float(t))


def subproblem(a, p, kind, w, c, eps):
    """One job's optimum: dict(t, v, jlo, jhi, xlo, xhi, j1, margin1, marginx)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    J = _Job()
    lib().orc_subproblem(len(a), _ptr(a), _ptr(p), int(kind), float(w), float(c), float(eps),
                         ctypes.byref(J))
    return {f: getattr(J, f) for f, _ in _Job._fields_}


def _tdt(T):
    if T.dtype == np.float32:
        return 0
    if T.dtype == np.float64:
        return 1
    raise TypeError("T must be float32 or float64")


class DualResult:
    """g(p), r, sum of net utilities, and (optionally) per-job results."""

    def __init__(self, g, r, sumv, jobs):
        self.g = g
        self.r = r
        self.sumv = sumv
        self.jobs = jobs

    @property
    def grad(self):
        return self._R - self.r


def _demands(d, n, m):
    """(array, columns) for optional demands: n scalars, or an n x m matrix
    of per-job demand vectors."""
    if d is None:
        return None, 0
    dd = np.ascontiguousarray(d, dtype=np.float64)
    if dd.shape == (n,):
        return dd, 1
    if dd.shape == (n, m):
        return dd, m
    raise ValueError("demands must have shape (n,) or (n, m)")


def dual_eval(T, w, c, kind, eps, R, p, per_job=False, d=None):
    """Dual function value, usage r and (per_job) the per-job optimum.
    d: optional per-job demands, n scalars or n x m vectors (usage limit
    sum_i d_i * x_i <= R)."""
    T = np.ascontiguousarray(T)
    n, m = T.shape
    tdt = _tdt(T)
    w = np.ascontiguousarray(w, dtype=T.dtype)
    c = np.ascontiguousarray(c, dtype=T.dtype)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    R = np.ascontiguousarray(R, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    g = ctypes.c_double()
    sv = ctypes.c_double()
    r = np.zeros(m)
    jobs = None
    outs = [None] * 9
    if per_job:
        jobs = {
            "jlo": np.empty(n, np.int32), "jhi": np.empty(n, np.int32),
            "xlo": np.empty(n), "xhi": np.empty(n), "t": np.empty(n), "v": np.empty(n),
            "j1": np.empty(n, np.int32), "margin1": np.empty(n), "marginx": np.empty(n),
        }
        outs = [jobs[k] for k in ("jlo", "jhi", "xlo", "xhi", "t", "v", "j1", "margin1",
                                  "marginx")]
    dd, dc = _demands(d, n, m)
    rc = lib().orc_dual_eval_m(n, m, tdt, _ptr(T), _ptr(w), _ptr(c), _ptr(kind), float(eps),
                               _ptr(R), _ptr(p), ctypes.byref(g), _ptr(r), ctypes.byref(sv),
                               *[_ptr(o) for o in outs], _ptr(dd), dc)
    if rc != 0:
        raise MemoryError("oracle dual_eval failed")
    res = DualResult(g.value, r, sv.value, jobs)
    res._R = R
    return res


def lower_bound(T, w, c, kind, eps, R, r, jobs):
    """U(X~) of the column-scaled allocation, and sum_i u(t_i) - u(t~_i)."""
    T = np.ascontiguousarray(T)
    n, m = T.shape
    du = ctypes.c_double()
    w = np.ascontiguousarray(w, dtype=T.dtype)
    c = np.ascontiguousarray(c, dtype=T.dtype)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    R = np.ascontiguousarray(R, dtype=np.float64)
    r = np.ascontiguousarray(r, dtype=np.float64)
    U = lib().orc_lower_bound(n, m, _tdt(T), _ptr(T), _ptr(w), _ptr(c), _ptr(kind), float(eps),
                              _ptr(R), _ptr(r), _ptr(jobs["jlo"]), _ptr(jobs["jhi"]),
                              _ptr(jobs["xlo"]), _ptr(jobs["xhi"]), ctypes.byref(du))
    return U, du.value


def solve(T, w, c, kind, eps, R, p0=None, tol_rel=1e-6, max_iter=500, mem=10, method=0,
          tol_abs=0.0, d=None):
    """Algorithm 2 with the oracle's projected L-BFGS; returns (p, info dict)."""
    T = np.ascontiguousarray(T)
    n, m = T.shape
    w = np.ascontiguousarray(w, dtype=T.dtype)
    c = np.ascontiguousarray(c, dtype=T.dtype)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    R = np.ascontiguousarray(R, dtype=np.float64)
    p = np.ones(m) if p0 is None else np.array(p0, dtype=np.float64)
    opts = SolveOpts(tol_rel, max_iter, mem, method, 0, tol_abs)
    info = SolveInfo()
    dd, dc = _demands(d, n, m)
    rc = lib().orc_solve_d(n, m, _tdt(T), _ptr(T), _ptr(w), _ptr(c), _ptr(kind), float(eps),
                           _ptr(R), ctypes.byref(opts), _ptr(p), ctypes.byref(info), _ptr(dd), dc)
    if rc != 0:
        raise RuntimeError("oracle solve failed (%d)" % rc)
    return p, {f: getattr(info, f) for f, _ in SolveInfo._fields_}


def init_prices(T, w, c, kind, eps, R, d=None):
    """The paper's data-dependent starting prices (eq. e-initialization);
    with demands d (n or n x m), each job's term is divided by its demand."""
    T = np.ascontiguousarray(T)
    n, m = T.shape
    w = np.ascontiguousarray(w, dtype=T.dtype)
    c = np.ascontiguousarray(c, dtype=T.dtype)
    kind = np.ascontiguousarray(kind, dtype=np.uint8)
    R = np.ascontiguousarray(R, dtype=np.float64)
    p = np.zeros(m)
    dd, dc = _demands(d, n, m)
    rc = lib().orc_init_prices_d(n, m, _tdt(T), _ptr(T), _ptr(w), _ptr(c), _ptr(kind),
                                 float(eps), _ptr(R), _ptr(p), _ptr(dd), dc)
    if rc != 0:
        raise RuntimeError("oracle init_prices failed (%d)" % rc)
    return p


def dense_allocation(n, m, jobs):
    """Dense n x m allocation from the per-job support."""
    X = np.zeros((n, m))
    idx = np.arange(n)
    lo = jobs["jlo"] >= 0
    X[idx[lo], jobs["jlo"][lo]] += jobs["xlo"][lo]
    hi = jobs["jhi"] >= 0
    X[idx[hi], jobs["jhi"][hi]] += jobs["xhi"][hi]
    return X


def first_vertex(T, p):
    """Each job's first envelope vertex decided in T's element type (the key
    a_ij * (1/p_j) rounded to it; lowest index on equal keys; -1 if none)."""
    T = np.ascontiguousarray(T)
    n, m = T.shape
    p = np.ascontiguousarray(p, dtype=np.float64)
    j1 = np.empty(n, np.int32)
    lib().orc_first_vertex(n, m, _tdt(T), _ptr(T), _ptr(p), _ptr(j1))
    return j1


def num_threads():
    return lib().orc_num_threads()
