"""GPU tests of per-job demands (usage limit sum_i d_i x_i <= R; the paper's
extensions in §7) through the C ABI, against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_clear_allocations, round_prices, to_device

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


def _problem(ctx, torch, I, d):
    import paper_2104_00282_amd as ra
    T, w, c, kind = to_device(I, torch)
    pr = ra.Problem(ctx, T, w, c, kind, I.R, I.eps)
    if d is not None:
        pr.set_demands(torch.from_numpy(d.astype(I.T.dtype)).cuda())
    return pr


def _demands(n, seed):
    return 0.5 + 2.5 * np.random.default_rng(seed).random(n)


@pytest.mark.parametrize("m,dtype", [(4, np.float32), (16, np.float32), (5, np.float32),
                                     (4, np.float64)])
def test_dual_eval_with_demands(ctx, torch, m, dtype):
    """g, r = sum_i d_i x_i, U(X~) and the per-job allocation against the
    oracle evaluated with the same demands."""
    print("demands m=%d %s" % (m, np.dtype(dtype).name), flush=True)
    I = synth.random_small(64 * 4 * 5 + 37, m, seed=700 + m, dtype=dtype)
    d = _demands(I.n, 701 + m).astype(dtype).astype(np.float64)
    pr = _problem(ctx, torch, I, d)
    tol = 1e-5 if dtype == np.float32 else 1e-9
    for p in (np.ones(m), 0.3 + np.random.default_rng(m).random(m) * 2):
        p = round_prices(p, dtype)
        out = pr.dual_eval(p, lower_bound=True, support=True)
        ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=d)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, ref.jobs)
        scale = abs(float(p @ I.R)) + np.abs(ref.jobs["v"]).sum()
        assert abs(out["g"] - ref.g) <= tol * scale
        assert np.allclose(out["r"], ref.r, rtol=tol, atol=tol * np.abs(ref.r).max())
        assert abs(out["lower_bound"] - U) <= tol * (scale + abs(U))
        jp = out["j_pair"].cpu().numpy().astype(np.int64)
        xp = out["x_pair"].cpu().numpy().astype(np.float64)
        same = (jp[:, 1] == ref.jobs["jhi"]) & np.isclose(xp[:, 1], ref.jobs["xhi"], atol=1e-4)
        assert same.mean() >= 0.999
        check_clear_allocations(ref.jobs, jp, xp, 1e-4)
    pr.close()


def test_uniform_demand_is_a_rescaling(ctx, torch):
    """d = 2 with limits 2R at prices p/2 is the d = 1 problem at p."""
    I = synth.random_small(20000, 16, seed=710, dtype=np.float32)
    p = round_prices(0.3 + np.random.default_rng(711).random(16) * 2, np.float32)
    a = _problem(ctx, torch, I, None)
    ga = a.dual_eval(p)
    I2 = synth.random_small(20000, 16, seed=710, dtype=np.float32)
    I2.R = 2 * I2.R
    b = _problem(ctx, torch, I2, np.full(I2.n, 2.0))
    gb = b.dual_eval(p / 2)
    assert gb["g"] == pytest.approx(ga["g"], rel=1e-6)
    assert np.allclose(gb["r"], 2 * ga["r"], rtol=1e-6)
    a.close()
    b.close()


def test_solve_with_demands_certified_by_oracle(ctx, torch):
    I = synth.random_small(50000, 8, seed=720, dtype=np.float32)
    d = _demands(I.n, 721).astype(np.float32).astype(np.float64)
    pr = _problem(ctx, torch, I, d)
    p, info, _ = pr.solve(tol_rel=1e-4, max_iter=200)
    assert info["rel_gap"] <= 2e-4
    ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=d)
    U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, ref.jobs)
    scale = abs(ref.g) + abs(U)
    assert abs(info["g"] - ref.g) <= 1e-5 * scale
    assert abs(info["U_lb"] - U) <= 1e-5 * scale
    pr.close()


def test_batched_pass_with_demands(ctx, torch):
    import paper_2104_00282_amd as ra
    insts, ds, probs = [], [], []
    for k, (n, m) in enumerate([(1000, 4), (5003, 16), (777, 32), (20000, 8)]):
        I = synth.random_small(n, m, seed=730 + k, dtype=np.float32)
        d = _demands(n, 740 + k).astype(np.float32).astype(np.float64)
        insts.append(I)
        ds.append(d)
        probs.append(_problem(ctx, torch, I, d))
    rng = np.random.default_rng(750)
    p0 = [round_prices(0.2 + rng.random(I.m) * 2, np.float32) for I in insts]
    _, infos, _ = ra.batch_solve(probs, p0=p0, tol_rel=0.0, max_evals=2)
    for I, d, p, inf in zip(insts, ds, p0, infos):
        ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=d)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, ref.jobs)
        scale = abs(float(p @ I.R)) + np.abs(ref.jobs["v"]).sum()
        assert abs(inf["g"] - ref.g) <= 1e-5 * scale
        assert abs(inf["U_lb"] - U) <= 1e-5 * (scale + abs(U))
    for pr in probs:
        pr.close()


def test_batched_two_groups_with_demands(ctx, torch):
    """20 problems (two interleaved groups of rounds), every other one with
    demands: the kernel variant with demands runs every problem, those
    without at unit demands; g(p0) and U(X~(p0)) against the oracle."""
    import paper_2104_00282_amd as ra
    sizes = [(1000, 4), (5003, 16), (777, 32), (20000, 8), (64, 4), (3001, 8), (12000, 16),
             (900, 32), (1, 8), (40000, 4)] * 2
    insts, ds, probs = [], [], []
    for k, (n, m) in enumerate(sizes):
        I = synth.random_small(n, m, seed=760 + k, dtype=np.float32)
        d = _demands(n, 790 + k).astype(np.float32).astype(np.float64) if k % 2 == 0 else None
        insts.append(I)
        ds.append(d)
        probs.append(_problem(ctx, torch, I, d))
    rng = np.random.default_rng(751)
    p0 = [round_prices(0.2 + rng.random(I.m) * 2, np.float32) for I in insts]
    _, infos, _ = ra.batch_solve(probs, p0=p0, tol_rel=0.0, max_evals=2)
    for I, d, p, inf in zip(insts, ds, p0, infos):
        ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=d)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, ref.jobs)
        scale = abs(float(p @ I.R)) + np.abs(ref.jobs["v"]).sum()
        assert abs(inf["g"] - ref.g) <= 1e-5 * scale, (I.n, I.m, d is not None)
        assert abs(inf["U_lb"] - U) <= 1e-5 * (scale + abs(U)), (I.n, I.m, d is not None)
        assert inf["dual_evals"] == 2
    for pr in probs:
        pr.close()


def test_removing_and_rejecting_demands(ctx, torch):
    """Removing demands restores the results of a problem that never had
    them, bit for bit; invalid demands are rejected and leave none."""
    import paper_2104_00282_amd as ra
    I = synth.random_small(10000, 8, seed=760, dtype=np.float32)
    p = round_prices(0.5 + np.arange(8) * 0.1, np.float32)
    ref = _problem(ctx, torch, I, None).dual_eval(p, lower_bound=True)
    pr = _problem(ctx, torch, I, _demands(I.n, 761))
    assert pr.dual_eval(p)["g"] != ref["g"]
    pr.set_demands(None)
    out = pr.dual_eval(p, lower_bound=True)
    assert out["g"] == ref["g"] and out["lower_bound"] == ref["lower_bound"]
    bad = torch.from_numpy(np.where(np.arange(I.n) == 7, -1.0, 1.0).astype(np.float32)).cuda()
    with pytest.raises(ra.RAError):
        pr.set_demands(bad)
    assert pr.dual_eval(p)["g"] == ref["g"]
    pr.close()
