"""The price update on the device (ra_solve_opts.device_loop = 1): the same
projected L-BFGS iteration of Algorithm 2 as the host loop, run by a one-wave
kernel after each pass, with the passes replayed from a graph.

Its dot products are wave reductions, so iterates match the host loop's to
rounding: early iterates are compared closely, full solves by their
certificates, which the oracle re-evaluates in FP64 at the returned prices.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2104_00282_amd as ra
    c = ra.Context(0)
    yield c
    c.close()


def _problem(ctx, torch, I):
    import paper_2104_00282_amd as ra
    T, w, c, kind = to_device(I, torch)
    return ra.Problem(ctx, T, w, c, kind, I.R, I.eps)


def _certificate(I, p):
    d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
    U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, d.r, d.jobs)
    return d.g, U


def _agree(ih, sh, idv, sd):
    """The device loop ends like the host loop: same status, a certificate
    as good (to rounding), the same dual value within the gap reached."""
    assert sd == sh
    assert idv["rel_gap"] <= 1.5 * ih["rel_gap"] + 1e-9
    assert abs(idv["g"] - ih["g"]) <= 2 * max(ih["rel_gap"], 1e-9) * abs(ih["g"])
    assert idv["dual_evals"] <= 2 * ih["dual_evals"] + 10


@pytest.mark.parametrize("m,n,seed,log_frac", [(4, 20000, 501, 1.0), (16, 50000, 502, 0.5),
                                               (32, 30011, 503, 0.5), (64, 40000, 504, 0.7)])
def test_solve_matches_host_and_oracle(ctx, torch, m, n, seed, log_frac):
    print(f"device loop solve m={m} n={n} seed={seed}", flush=True)
    I = synth.random_small(n, m, seed=seed, dtype=np.float32, log_frac=log_frac)
    prob = _problem(ctx, torch, I)
    # FP32 instances with capped-linear jobs stop at their gap floor (stall)
    kw = dict(tol_rel=1e-6, max_iter=300, stall_evals=60)
    ph, ih, sh = prob.solve(**kw)
    pd, idv, sd = prob.solve(device_loop=True, **kw)
    print("host", ih, "\ndevice", idv, flush=True)
    _agree(ih, sh, idv, sd)
    assert idv["U_lb"] <= idv["g"] and idv["iters"] >= 1
    assert idv["fell_back"] <= idv["iters"]
    # the certificate holds at the returned prices (FP64 oracle)
    g, U = _certificate(I, pd)
    scale = abs(g) + abs(U)
    assert abs(idv["g"] - g) <= 1e-5 * scale
    assert abs(idv["U_lb"] - U) <= 1e-5 * scale


@pytest.mark.parametrize("budget", [1, 2, 3, 5, 8])
def test_early_iterates_match_host(ctx, torch, budget):
    """With the same pass budget both loops take the same steps; prices agree
    to a few FP32 ulps (the only difference is the order of the sums)."""
    I = synth.random_small(20000, 16, seed=505, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    ph, ih, _ = prob.solve(tol_rel=1e-9, max_iter=300, max_evals=budget)
    pd, idv, _ = prob.solve(tol_rel=1e-9, max_iter=300, max_evals=budget, device_loop=True)
    assert idv["dual_evals"] == ih["dual_evals"] <= budget
    assert idv["iters"] == ih["iters"] and idv["fell_back"] == ih["fell_back"]
    assert np.allclose(pd, ph, rtol=1e-6, atol=0)
    assert idv["g"] == pytest.approx(ih["g"], rel=1e-6)
    if np.isfinite(ih["rel_gap"]):
        assert idv["rel_gap"] == pytest.approx(ih["rel_gap"], rel=1e-4, abs=1e-9)
    else:
        assert not np.isfinite(idv["rel_gap"])


def test_iteration_budget_and_subgradient(ctx, torch):
    I = synth.random_small(20000, 8, seed=506, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    p, info, st = prob.solve(tol_rel=1e-12, max_iter=3, device_loop=True)
    ph, ih, _ = prob.solve(tol_rel=1e-12, max_iter=3)
    assert info["iters"] == ih["iters"] == 3
    assert info["dual_evals"] == ih["dual_evals"]
    assert np.allclose(p, ph, rtol=1e-5)
    ps, isg, _ = prob.solve(tol_rel=1e-9, max_iter=25, method=1, device_loop=True)
    pj, ihs, _ = prob.solve(tol_rel=1e-9, max_iter=25, method=1)
    assert isg["fell_back"] == isg["iters"] == ihs["iters"]
    assert np.allclose(ps, pj, rtol=1e-5)
    assert isg["rel_gap"] == pytest.approx(ihs["rel_gap"], rel=1e-3)


def test_warm_start_and_absolute_tolerance(ctx, torch):
    I = synth.random_small(30000, 16, seed=507, dtype=np.float32, log_frac=1.0)
    n = I.T.shape[0]
    prob = _problem(ctx, torch, I)
    p, info, st = prob.solve(tol_rel=1e-6, max_iter=300, stall_evals=60, device_loop=True)
    assert np.isfinite(info["rel_gap"])
    # restarted at its own answer with a tolerance it meets there, the loop
    # certifies the start in the second pass and stops; that pass's own point
    # is not taken into the iteration, so one evaluation is counted
    p2, info2, st2 = prob.solve(p0=p, tol_rel=1.01 * info["rel_gap"], max_iter=5,
                                device_loop=True)
    assert st2 == 0 and info2["iters"] == 0 and info2["dual_evals"] == 1
    assert np.array_equal(p2, p)
    pa, ia, sa = prob.solve(tol_rel=0.0, tol_abs=1e-3 * n, max_iter=300, paper_init=True,
                            device_loop=True)
    ph, ih, _ = prob.solve(tol_rel=0.0, tol_abs=1e-3 * n, max_iter=300, paper_init=True)
    assert sa == 0 and ia["converged"] == 1
    assert ia["g"] - ia["U_lb"] <= 1e-3 * n
    assert abs(ia["iters"] - ih["iters"]) <= max(3, ih["iters"] // 3)


def test_stall_stop(ctx, torch):
    I = synth.random_small(20000, 16, seed=508, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    p, info, st = prob.solve(tol_rel=0.0, max_iter=500, stall_evals=12, device_loop=True)
    ph, ih, sh = prob.solve(tol_rel=0.0, max_iter=500, stall_evals=12)
    assert st == sh == 5  # RA_ENOTCONV: tol_rel = 0 is never met
    assert info["dual_evals"] < 500
    assert np.isfinite(info["rel_gap"])
    assert info["rel_gap"] == pytest.approx(ih["rel_gap"], rel=0.5, abs=1e-6)


@pytest.mark.parametrize("budget", [10, 16, 24])
def test_stall_restarts_match_host(ctx, torch, budget):
    """Started at a solved problem's prices, the certified gap cannot improve,
    so with a window of 3 passes the loops stall every few passes: the first
    two stalls restart from the best certified point, the third stops.  The
    device loop takes the host loop's passes, with iterates equal to rounding,
    and both end at least as tight as without restarts."""
    I = synth.random_small(20000, 16, seed=509, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    p0, _, _ = prob.solve(tol_rel=0.0, max_iter=200, stall_evals=40)
    kw = dict(p0=p0, tol_rel=0.0, max_iter=300, max_evals=budget, stall_evals=3)
    ph, ih, sh = prob.solve(stall_restarts=2, **kw)
    pd, idv, sd = prob.solve(stall_restarts=2, device_loop=True, **kw)
    pn, inr, _ = prob.solve(**kw)
    assert sh == sd == 5  # RA_ENOTCONV: tol_rel = 0 is never met
    assert inr["dual_evals"] < ih["dual_evals"] <= budget
    assert idv["dual_evals"] == ih["dual_evals"] and idv["iters"] == ih["iters"]
    assert np.allclose(pd, ph, rtol=1e-6, atol=0)
    assert idv["rel_gap"] == pytest.approx(ih["rel_gap"], rel=1e-4, abs=1e-9)
    assert ih["rel_gap"] <= inr["rel_gap"] * (1 + 1e-12)


def test_demands_scalar_and_vector(ctx, torch):
    n, m = 40000, 16
    I = synth.random_small(n, m, seed=509, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    kw = dict(tol_rel=1e-6, max_iter=300, stall_evals=60)
    d = 0.5 + 2.5 * np.random.default_rng(510).random(n)
    prob.set_demands(torch.from_numpy(d.astype(np.float32)).cuda())
    ph, ih, sh = prob.solve(**kw)
    pd, idv, sd = prob.solve(device_loop=True, **kw)
    print("demands host", ih, "\ndevice", idv, flush=True)
    _agree(ih, sh, idv, sd)
    od = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, pd, d=d)
    assert idv["g"] == pytest.approx(od.g, rel=1e-5)
    prob.set_demands(None)
    D = 0.5 + 2.5 * np.random.default_rng(511).random((n, m))
    prob.set_demand_vectors(torch.from_numpy(D.astype(np.float32)).cuda())
    ph, ih, sh = prob.solve(**kw)
    pd, idv, sd = prob.solve(device_loop=True, **kw)
    print("demand vectors host", ih, "\ndevice", idv, flush=True)
    _agree(ih, sh, idv, sd)
    od = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, pd, d=D)
    assert idv["g"] == pytest.approx(od.g, rel=1e-5)
    # removing the demands drops the captured passes; the plain problem again
    prob.set_demand_vectors(None)
    pn, inn, sn = prob.solve(device_loop=True, **kw)
    g, U = _certificate(I, pn)
    assert inn["g"] == pytest.approx(g, rel=1e-5)
    assert np.isfinite(inn["rel_gap"]) and inn["rel_gap"] < 1e-3


def test_other_problems_run_the_host_loop(ctx, torch):
    """device_loop = 1 leaves the generic kernels (m outside the vectorised
    classes, FP64) and long L-BFGS memories to the host loop, unchanged."""
    for I, mem in ((synth.random_small(5000, 5, seed=512, dtype=np.float32), 10),
                   (synth.random_small(3000, 8, seed=513, dtype=np.float64), 10),
                   (synth.random_small(5000, 8, seed=514, dtype=np.float32), 40)):
        prob = _problem(ctx, torch, I)
        pa, ia, _ = prob.solve(tol_rel=1e-6, max_iter=60, lbfgs_mem=mem)
        pb, ib, _ = prob.solve(tol_rel=1e-6, max_iter=60, lbfgs_mem=mem, device_loop=True)
        assert np.array_equal(pa, pb)
        assert ia["g"] == ib["g"] and ia["dual_evals"] == ib["dual_evals"]


@pytest.mark.parametrize("mem", [1, 3, 32])
def test_memory_sizes_match_host(ctx, torch, mem):
    """The L-BFGS ring buffer at its smallest, an odd and its largest size
    on the device: the same passes and iterates as the host loop."""
    I = synth.random_small(20000, 32, seed=515 + mem, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    kw = dict(tol_rel=1e-9, max_iter=300, max_evals=40, lbfgs_mem=mem)
    ph, ih, _ = prob.solve(**kw)
    pd, idv, _ = prob.solve(device_loop=True, **kw)
    assert idv["dual_evals"] == ih["dual_evals"]
    assert idv["iters"] == ih["iters"] and idv["fell_back"] == ih["fell_back"]
    assert np.allclose(pd, ph, rtol=1e-5, atol=0)
    assert idv["rel_gap"] == pytest.approx(ih["rel_gap"], rel=1e-3)


def test_kernel_timing_keeps_the_host_loop(ctx, torch):
    """With per-kernel timing on, every pass is timed on the host side, so
    device_loop = 1 runs the host loop: the same result, and every pass of
    the solve shows up in the timing counters."""
    import paper_2104_00282_amd as ra
    I = synth.random_small(20000, 16, seed=520, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    pa, ia, _ = prob.solve(tol_rel=1e-5, max_iter=50)
    ra.ra_set_kernel_timing(ctx.handle, True)
    try:
        pb, ib, _ = prob.solve(tol_rel=1e-5, max_iter=50, device_loop=True)
        _, launches = ra.ra_get_kernel_timing(ctx.handle)
    finally:
        ra.ra_set_kernel_timing(ctx.handle, False)
    assert np.array_equal(pa, pb) and ia["dual_evals"] == ib["dual_evals"]
    assert launches >= ib["dual_evals"]


@pytest.mark.parametrize("n,m", [(1, 4), (65, 8), (1000, 64)])
def test_tiny_and_ragged_problems(ctx, torch, n, m):
    """A single job, one tile and a ragged second, a few tiles at m = 64:
    the device loop ends as the host loop does."""
    I = synth.random_small(n, m, seed=530 + n, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    kw = dict(tol_rel=1e-6, max_iter=100, stall_evals=40)
    ph, ih, sh = prob.solve(**kw)
    pd, idv, sd = prob.solve(device_loop=True, **kw)
    assert sd == sh
    assert idv["dual_evals"] == ih["dual_evals"] and idv["iters"] == ih["iters"]
    assert np.allclose(pd, ph, rtol=1e-5, atol=1e-12)
    if np.isfinite(ih["rel_gap"]):
        assert idv["rel_gap"] == pytest.approx(ih["rel_gap"], rel=1e-3, abs=1e-9)
