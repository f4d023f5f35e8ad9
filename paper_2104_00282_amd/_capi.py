"""ctypes declarations of the C ABI in include/resalloc.h (same names).

This module only marshals arguments: every step of the method runs in the
HIP library.  Importing it fails loudly when libresalloc.so is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libresalloc.so")

RA_OK = 0
RA_EINVAL = 1
RA_ENOMEM = 2
RA_EDEVICE = 3
RA_ENUMERIC = 4
RA_ENOTCONV = 5
RA_EUNSUPPORTED = 6

RA_F32 = 0
RA_F64 = 1
RA_UTIL_LOG = 0
RA_UTIL_CAPLIN = 1
RA_UTIL_ALPHA_FAIR = 2
RA_MAX_RESOURCES = 256

_vp = ctypes.c_void_p
_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_int = ctypes.c_int
_st = ctypes.c_int


class ra_solve_opts(ctypes.Structure):
    _fields_ = [("tol_rel", _d), ("max_iter", _i32), ("lbfgs_mem", _i32), ("method", _i32),
                ("init", _i32), ("use_graph", _i32), ("verbose", _i32), ("max_evals", _i32),
                ("stall_evals", _i32), ("init_step", _d), ("tol_abs", _d),
                ("device_loop", _i32), ("stall_restarts", _i32),
                ("warm_stall_restarts", _i32), ("warm_stall_evals", _i32)]


class ra_solve_info(ctypes.Structure):
    _fields_ = [("iters", _i32), ("dual_evals", _i32), ("fell_back", _i32), ("converged", _i32),
                ("g", _d), ("U_lb", _d), ("rel_gap", _d), ("seconds", _d),
                ("restarted", _i32), ("warm_evals", _i32)]


# name -> (restype, argtypes)
PROTOTYPES = {
    "ra_create": (_st, [ctypes.POINTER(_vp), _int, _vp]),
    "ra_destroy": (_st, [_vp]),
    "ra_status_string": (ctypes.c_char_p, [_st]),
    "ra_last_error": (ctypes.c_char_p, [_vp]),
    "ra_problem_create": (_st, [_vp, ctypes.POINTER(_vp), _i64, _i32, _int, _vp, _vp, _vp, _vp,
                                _vp, _d, _int]),
    "ra_problem_destroy": (_st, [_vp]),
    "ra_dual_eval": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "ra_dual_eval_noalloc": (_st, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "ra_solve_opts_default": (None, [ctypes.POINTER(ra_solve_opts)]),
    "ra_solve": (_st, [_vp, _vp, ctypes.POINTER(ra_solve_opts), _vp,
                       ctypes.POINTER(ra_solve_info)]),
    "ra_get_allocation": (_st, [_vp, _vp, _vp, _vp]),
    "ra_batch_solve": (_st, [_vp, _i32, _vp, ctypes.POINTER(ra_solve_opts), _vp, _vp,
                             _vp]),
    "ra_batch_set_shape": (_st, [_vp, _i32, ctypes.POINTER(_i32), _i32]),
    "ra_batch_tuning": (_st, [_vp, ctypes.c_char_p, ctypes.c_size_t,
                              ctypes.POINTER(ctypes.c_size_t)]),
    "ra_features": (_st, [_vp, _vp, _vp]),
    "ra_predict_prices": (_st, [_vp, _vp, _vp, _vp]),
    "ra_init_prices": (_st, [_vp, _vp, _vp]),
    "ra_problem_set_demands": (_st, [_vp, _vp, _vp]),
    "ra_problem_set_demand_vectors": (_st, [_vp, _vp, _vp]),
    "ra_stream_read_ms": (_st, [_vp, _vp, _i64, _i32, ctypes.POINTER(_d)]),
    "ra_probe_first_vertex_ms": (_st, [_vp, _vp, _i64, ctypes.POINTER(_d), _i32, _i32, _vp,
                                       ctypes.POINTER(_d)]),
    "ra_mlp_create": (_st, [_vp, _i32, _i32, _i32, ctypes.c_uint64, ctypes.POINTER(_vp)]),
    "ra_mlp_destroy": (_st, [_vp]),
    "ra_mlp_num_params": (_st, [_vp, ctypes.POINTER(_i64)]),
    "ra_mlp_get_params": (_st, [_vp, _vp]),
    "ra_mlp_set_params": (_st, [_vp, _vp]),
    "ra_mlp_set_normalization": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "ra_mlp_forward": (_st, [_vp, _vp, _i32, _vp, _vp]),
    "ra_mlp_gradients": (_st, [_vp, _vp, _i32, _vp, _vp, _vp, ctypes.POINTER(_d)]),
    "ra_mlp_train_step": (_st, [_vp, _vp, _i32, _vp, _vp, ctypes.c_float, ctypes.POINTER(_d)]),
    "ra_mlp_save": (_st, [_vp, ctypes.c_char_p]),
    "ra_mlp_load": (_st, [_vp, ctypes.c_char_p, ctypes.POINTER(_vp)]),
    "ra_solve_learned": (_st, [_vp, _vp, _vp, ctypes.POINTER(ra_solve_opts), _i32, _vp,
                               ctypes.POINTER(ra_solve_info)]),
    "ra_set_kernel_timing": (_st, [_vp, _int]),
    "ra_get_kernel_timing": (_st, [_vp, ctypes.POINTER(_d), ctypes.POINTER(_i64)]),
}

_lib = None


def lib():
    """Load libresalloc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libresalloc.so is not built (run __graft_entry__.build() or "
                              "python paper_2104_00282_amd/build.py): " + LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class RAError(RuntimeError):
    def __init__(self, status, detail=""):
        self.status = status
        msg = lib().ra_status_string(status).decode()
        super().__init__("%s (%d)%s" % (msg, status, (": " + detail) if detail else ""))


def ra_status_string(status):
    return lib().ra_status_string(status).decode()


def ra_last_error(ctx):
    return lib().ra_last_error(ctx).decode()


def ra_create(device_ordinal=0, hip_stream=None):
    h = _vp()
    st = lib().ra_create(ctypes.byref(h), device_ordinal, hip_stream)
    if st != RA_OK:
        raise RAError(st, "ra_create")
    return h


def ra_destroy(ctx):
    return lib().ra_destroy(ctx)


def ra_problem_create(ctx, n, m, dtype, T, w, c, kind, R, eps, validate):
    h = _vp()
    st = lib().ra_problem_create(ctx, ctypes.byref(h), n, m, dtype, T, w, c, kind, R, eps,
                                 validate)
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return h


def ra_problem_destroy(prob):
    return lib().ra_problem_destroy(prob)


def ra_dual_eval(ctx, prob, p, g, grad, lower_bound, j_pair, x_pair, j1):
    st = lib().ra_dual_eval(ctx, prob, p, g, grad, lower_bound, j_pair, x_pair, j1)
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return st


def ra_solve_opts_default():
    o = ra_solve_opts()
    lib().ra_solve_opts_default(ctypes.byref(o))
    return o


def ra_solve(ctx, prob, opts, p_inout, info):
    st = lib().ra_solve(ctx, prob, ctypes.byref(opts) if opts is not None else None, p_inout,
                        ctypes.byref(info) if info is not None else None)
    if st not in (RA_OK, RA_ENOTCONV):
        raise RAError(st, ra_last_error(ctx))
    return st


def ra_get_allocation(ctx, prob, p, X):
    st = lib().ra_get_allocation(ctx, prob, p, X)
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return st


def ra_set_kernel_timing(ctx, enable):
    st = lib().ra_set_kernel_timing(ctx, 1 if enable else 0)
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return st


def ra_get_kernel_timing(ctx):
    """(milliseconds, launches) of the timed dual-kernel launches."""
    ms = ctypes.c_double()
    k = ctypes.c_int64()
    st = lib().ra_get_kernel_timing(ctx, ctypes.byref(ms), ctypes.byref(k))
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return ms.value, k.value


def ra_stream_read_ms(ctx, ptr, nbytes, reps=20):
    """Mean ms of one plain streaming read of nbytes at device address ptr."""
    ms = ctypes.c_double()
    st = lib().ra_stream_read_ms(ctx, ptr, nbytes, reps, ctypes.byref(ms))
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return ms.value


def ra_probe_first_vertex_ms(ctx, T_ptr, n, p, lanes_per_job, reps, j1_ptr):
    """Mean ms of one first-vertex scan pass over an n x 64 FP32 matrix with
    lanes_per_job lanes per job; the vertices go to the int16 device array
    at j1_ptr."""
    pa = (_d * 64)(*[float(v) for v in p])
    ms = ctypes.c_double()
    st = lib().ra_probe_first_vertex_ms(ctx, T_ptr, n, pa,
                                        lanes_per_job, reps, j1_ptr, ctypes.byref(ms))
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return ms.value


def ra_batch_solve(ctx, B, probs, opts, tol_each, p_inout, infos):
    """probs: ctypes array of problem handles; infos: ctypes array of
    ra_solve_info (or None)."""
    st = lib().ra_batch_solve(ctx, B, probs, ctypes.byref(opts) if opts is not None else None,
                              tol_each, p_inout, infos)
    if st not in (RA_OK, RA_ENOTCONV):
        raise RAError(st, ra_last_error(ctx))
    return st


def ra_batch_set_shape(ctx, tile_floats, rows=(0, 0, 0, 0), blocks_per_cu=0):
    """Fix the batched launch shape (tile_floats 0: back to the autotuner)."""
    arr = (_i32 * 4)(*[int(r) for r in rows])
    st = lib().ra_batch_set_shape(ctx, int(tile_floats), arr, int(blocks_per_cu))
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return st


def ra_batch_tuning(ctx):
    """The autotuner's JSON record of its last tuning on ctx ("" if none)."""
    n = ctypes.c_size_t()
    st = lib().ra_batch_tuning(ctx, None, 0, ctypes.byref(n))
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    buf = ctypes.create_string_buffer(n.value + 1)
    st = lib().ra_batch_tuning(ctx, buf, n.value + 1, ctypes.byref(n))
    if st != RA_OK:
        raise RAError(st, ra_last_error(ctx))
    return buf.value.decode()


def check(ctx, st, allow=(RA_OK,)):
    """Raise RAError unless st is in allow."""
    if st not in allow:
        raise RAError(st, ra_last_error(ctx) if ctx else "")
    return st
