"""The allocation-free evaluation ra_dual_eval_noalloc (C ABI) against the
evaluation it varies, ra_dual_eval, and against the oracle.

Three calls in a row on one GPU, each on a smaller problem than the one
before (the calls share the device's scratch array, which keeps the last
call's contents): m = 256 on the generic kernel with more blocks than the
scratch holds partials for (the launch is capped), m = 64 on the vectorised
kernel, and an FP64 problem.  g, grad and U(X~) must match ra_dual_eval and
the oracle to relative 1e-5 (FP32) / 1e-9 (FP64)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_relative, round_prices, to_device

pytestmark = pytest.mark.gpu


def _noalloc(ctx, prob, p, lower_bound=True):
    import paper_2104_00282_amd as ra
    L = ra._capi.lib()
    g = ctypes.c_double()
    grad = np.zeros(prob.m)
    lb = ctypes.c_double()
    pp = np.ascontiguousarray(p, dtype=np.float64)
    st = L.ra_dual_eval_noalloc(ctx.handle, prob.handle, pp.ctypes.data_as(ctypes.c_void_p),
                                ctypes.byref(g), grad.ctypes.data_as(ctypes.c_void_p),
                                ctypes.byref(lb) if lower_bound else None)
    assert st == ra.RA_OK, ra.ra_last_error(ctx.handle)
    return {"g": g.value, "grad": grad, "lower_bound": lb.value if lower_bound else None}


def test_noalloc_matches_dual_eval_on_shrinking_problems():
    import torch
    import paper_2104_00282_amd as ra
    assert torch.cuda.is_available()
    ctx = ra.Context(0)
    cases = [(300_000, 256, np.float32, 1e-5, 91), (50_003, 64, np.float32, 1e-5, 92),
             (2_049, 7, np.float64, 1e-9, 93)]
    for n, m, dt, tol, seed in cases:
        print("noalloc n=%d m=%d %s" % (n, m, np.dtype(dt).name), flush=True)
        I = synth.random_small(n, m, seed=seed, dtype=dt)
        T, w, c, kind = to_device(I, torch)
        prob = ra.Problem(ctx, T, w, c, kind, I.R, I.eps)
        p = round_prices(0.2 + np.random.default_rng(seed).random(m) * 3, dt)
        a = prob.dual_eval(p, lower_bound=True)
        b = _noalloc(ctx, prob, p)
        ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, ref.jobs)
        scale_g = abs(float(p @ I.R)) + np.abs(ref.jobs["v"]).sum()
        scale_r = np.maximum(I.R, np.abs(ref.r))
        for want_g, want_r, want_U in ((a["g"], a["r"], a["lower_bound"]), (ref.g, ref.r, U)):
            check_relative(b["g"], want_g, scale_g, tol, "g")
            assert np.all(np.abs((I.R - b["grad"]) - want_r) <= tol * scale_r)
            check_relative(b["lower_bound"], want_U, 2 * scale_g, tol, "U(X~)")
        # without the bound: one pass, the same g and grad
        c2 = _noalloc(ctx, prob, p, lower_bound=False)
        assert c2["g"] == b["g"] and np.array_equal(c2["grad"], b["grad"])
        prob.close()
    ctx.close()
