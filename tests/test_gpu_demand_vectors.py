"""GPU tests of per-job demand vectors (usage limit sum_i d_ij x_ij <= R_j,
job i priced at d_i * p; the paper's extensions in §7) through the C ABI,
against the oracle evaluated with the same demands."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import check_clear_allocations, check_first_vertex, round_prices, to_device

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


def _dvec(n, m, seed, dtype):
    """Demand vectors in [0.4, 2.9), rounded to the problem's element type."""
    D = 0.4 + 2.5 * np.random.default_rng(seed).random((n, m))
    return D.astype(dtype).astype(np.float64)


def _device_dvec(torch, D, dtype, aligned=True):
    """D on the device; aligned=False places it 4 bytes past a 16-byte
    boundary (the vectorised kernels then do not apply)."""
    flat = torch.from_numpy(np.ascontiguousarray(D.astype(dtype)).ravel()).cuda()
    if aligned:
        return flat.view(D.shape)
    buf = torch.empty(flat.numel() + 4, dtype=flat.dtype, device=flat.device)
    view = buf[1:1 + flat.numel()]
    view.copy_(flat)
    assert view.data_ptr() % 16 != 0
    return view.view(D.shape)


def _problem(ctx, torch, I, D=None, aligned=True):
    import paper_2104_00282_amd as ra
    T, w, c, kind = to_device(I, torch)
    pr = ra.Problem(ctx, T, w, c, kind, I.R, I.eps)
    if D is not None:
        pr.set_demand_vectors(_device_dvec(torch, D, I.T.dtype, aligned))
    return pr


def _check_eval(I, D, p, out, tol):
    ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=D)
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
    # j1 at the prices d_i * p: the kernel forms 1/(d_ij p_j) with the
    # hardware reciprocal (about 1 ulp), which no CPU code reproduces bit for
    # bit, so it is compared with the exact argmax wherever that is not a
    # near-tie, and nearly everywhere overall
    j1 = out["j1"].cpu().numpy().astype(np.int64)
    check_first_vertex(I.T.astype(np.float64) / D.astype(np.float64), p, j1, ref.jobs["j1"],
                       ref.jobs["margin1"], min_clear=0.99, tie_tol=1e-5)
    assert (j1 == ref.jobs["j1"]).mean() >= 0.999


@pytest.mark.parametrize("m,dtype,aligned", [(4, np.float32, True), (16, np.float32, True),
                                             (64, np.float32, True), (5, np.float32, True),
                                             (16, np.float32, False), (4, np.float64, True)])
def test_dual_eval_with_demand_vectors(ctx, torch, m, dtype, aligned):
    """g, r = sum_i d_ij x_ij, U(X~), the per-job support and j1 against the
    oracle, on several tiles and a ragged tail; vectorised (aligned FP32,
    m in the vector classes) and generic kernels."""
    print("demand vectors m=%d %s aligned=%d" % (m, np.dtype(dtype).name, aligned), flush=True)
    I = synth.random_small(64 * 4 * 5 + 37, m, seed=800 + m, dtype=dtype)
    D = _dvec(I.n, m, 801 + m, dtype)
    pr = _problem(ctx, torch, I, D, aligned)
    tol = 1e-5 if dtype == np.float32 else 1e-9
    for p in (np.ones(m), 0.3 + np.random.default_rng(m).random(m) * 2):
        p = round_prices(p, dtype)
        out = pr.dual_eval(p, lower_bound=True, support=True, j1=True)
        _check_eval(I, D, p, out, tol)
    pr.close()


def test_equal_columns_match_scalar_demands(ctx, torch):
    """Demand vectors whose entries all equal d_i give the results of the
    scalar demands d_i (different arithmetic: w_i / d_i packed against d_i p)."""
    I = synth.random_small(30000, 16, seed=810, dtype=np.float32)
    d = (0.5 + 2 * np.random.default_rng(811).random(I.n)).astype(np.float32).astype(np.float64)
    p = round_prices(0.3 + np.random.default_rng(812).random(16) * 2, np.float32)
    a = _problem(ctx, torch, I)
    a.set_demands(torch.from_numpy(d.astype(np.float32)).cuda())
    b = _problem(ctx, torch, I, np.repeat(d[:, None], 16, axis=1))
    ga = a.dual_eval(p, lower_bound=True)
    gb = b.dual_eval(p, lower_bound=True)
    assert gb["g"] == pytest.approx(ga["g"], rel=2e-6)
    assert np.allclose(gb["r"], ga["r"], rtol=2e-5, atol=1e-4 * np.abs(ga["r"]).max())
    assert gb["lower_bound"] == pytest.approx(ga["lower_bound"], rel=2e-5)
    a.close()
    b.close()


@pytest.mark.parametrize("m", [8, 6])
def test_solve_with_demand_vectors_certified_by_oracle(ctx, torch, m):
    """Price discovery with demand vectors (fused certificate): the reported
    g and U(X~) are the oracle's at the returned prices."""
    I = synth.random_small(50000, m, seed=820 + m, dtype=np.float32)
    D = _dvec(I.n, m, 821 + m, np.float32)
    pr = _problem(ctx, torch, I, D)
    p, info, _ = pr.solve(tol_rel=1e-4, max_iter=200)
    assert info["rel_gap"] <= 2e-4
    ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=D)
    U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, ref.jobs)
    scale = abs(ref.g) + abs(U)
    assert abs(info["g"] - ref.g) <= 1e-5 * scale
    assert abs(info["U_lb"] - U) <= 1e-5 * scale
    # the usage of the returned point respects R up to the certified gap
    assert np.all(ref.r <= I.R * 1.05)
    # the dense allocation: the oracle's, with each column scaled by
    # min(1, R_j / r_j), and within the limits in demanded units
    X = pr.allocation(p).cpu().numpy().astype(np.float64)
    s = np.where(ref.r > I.R, I.R / ref.r, 1.0)
    Xo = oracle.dense_allocation(I.n, m, ref.jobs) * s[None, :]
    assert np.all(X >= 0) and np.all(X.sum(1) <= 1 + 1e-5)
    assert np.all((D * X).sum(0) <= I.R * (1 + 1e-5))
    assert (np.abs(X - Xo).max(1) <= 1e-4).mean() >= 0.999
    pr.close()


@pytest.mark.parametrize("m,aligned", [(16, True), (7, True), (16, False)])
def test_init_prices_with_demand_vectors(ctx, torch, m, aligned):
    I = synth.random_small(20000, m, seed=830 + m, dtype=np.float32)
    D = _dvec(I.n, m, 831 + m, np.float32)
    pr = _problem(ctx, torch, I, D, aligned)
    p = pr.init_prices()
    ref = oracle.init_prices(I.T, I.w, I.c, I.kind, I.eps, I.R, d=D)
    assert np.allclose(p, ref, rtol=2e-5)
    pr.close()


def test_removing_and_rejecting_demand_vectors(ctx, torch):
    """Removing demand vectors restores the results of a problem that never
    had them, bit for bit; a non-positive entry is rejected and leaves the
    previous vectors in place; scalar demands and batched solves refuse a
    problem with demand vectors."""
    import paper_2104_00282_amd as ra
    I = synth.random_small(10000, 8, seed=840, dtype=np.float32)
    p = round_prices(0.5 + np.arange(8) * 0.1, np.float32)
    base = _problem(ctx, torch, I)
    ref = base.dual_eval(p, lower_bound=True)
    D = _dvec(I.n, 8, 841, np.float32)
    pr = _problem(ctx, torch, I, D)
    with_d = pr.dual_eval(p, lower_bound=True)
    assert with_d["g"] != ref["g"]
    bad = D.copy()
    bad[123, 5] = 0.0
    with pytest.raises(ra.RAError):
        pr.set_demand_vectors(torch.from_numpy(bad.astype(np.float32)).cuda())
    assert pr.dual_eval(p)["g"] == with_d["g"]
    with pytest.raises(ra.RAError):
        pr.set_demands(torch.ones(I.n, dtype=torch.float32, device="cuda"))
    with pytest.raises(ra.RAError):
        ra.batch_solve([pr], p0=[p], max_evals=2)
    pr.set_demand_vectors(None)
    out = pr.dual_eval(p, lower_bound=True)
    assert out["g"] == ref["g"] and out["lower_bound"] == ref["lower_bound"]
    base.close()
    pr.close()


def test_full_size_sampled_parity(ctx, torch):
    """The benchmark's demand-vector workload (n = 1e7, m = 64, FP32, the
    vectorised kernel): sampled jobs' supports against the oracle solved on
    those rows alone, and r equal to the sum of d_ij x_ij over the kernel's
    own per-job outputs (FP64 on the device)."""
    import paper_2104_00282_amd as ra
    I = synth.demand_vectors_device()
    pr = ra.Problem(ctx, I["T"], I["w"], I["c"], I["kind"], I["R"], I["eps"], validate=False)
    pr.set_demand_vectors(I["D"])
    p = round_prices(I["p"], np.float32)
    out = pr.dual_eval(p, support=True)
    jp = out["j_pair"].long()
    xp = out["x_pair"].double()
    Dd = I["D"]
    rows = torch.arange(I["n"], device="cuda")
    r = torch.zeros(64, dtype=torch.float64, device="cuda")
    for k in (0, 1):
        ok = jp[:, k] >= 0
        j = jp[ok, k]
        r.index_add_(0, j, Dd[rows[ok], j].double() * xp[ok, k])
    assert np.allclose(out["r"], r.cpu().numpy(), rtol=1e-5)
    idx = np.sort(np.random.default_rng(850).choice(I["n"], 3000, replace=False))
    ti = torch.from_numpy(idx).cuda()
    T = I["T"][ti].cpu().numpy()
    w = I["w"][ti].cpu().numpy()
    c = I["c"][ti].cpu().numpy()
    kind = I["kind"][ti].cpu().numpy()
    D = Dd[ti].cpu().numpy().astype(np.float64)
    ref = oracle.dual_eval(T, w, c, kind, I["eps"], I["R"], p, per_job=True, d=D)
    jps = jp[ti].cpu().numpy()
    xps = xp[ti].cpu().numpy()
    same = (jps[:, 1] == ref.jobs["jhi"]) & np.isclose(xps[:, 1], ref.jobs["xhi"], atol=1e-4)
    assert same.mean() >= 0.998
    pr.close()


@pytest.mark.parametrize("n,m", [(1, 1), (1, 4), (130, 4), (130, 5), (300, 16)])
def test_demand_vectors_edge_cases(ctx, torch, n, m):
    """A single job, a single resource, exact zero throughputs (20 %), free
    resources (p_j = 0) and alpha-fair jobs beside log and capped-linear ones,
    all with demand vectors: parity with the oracle.  Free resources make
    many allocations optimal (a capped job can fill its cap from any mix of
    them), so jobs whose allocation differs from the oracle's must be optimal
    at d_i * p, and r must be the d-weighted sum of the kernel's own
    allocations."""
    from gpu_util import dense_x, job_values
    print("demand vectors edge n=%d m=%d" % (n, m), flush=True)
    I = synth.random_small(n, m, seed=870 + n + m, dtype=np.float32, zero_frac=0.2)
    rng = np.random.default_rng(871 + n + m)
    af = rng.random(n) < 0.3
    I.kind = np.where(af, 2, I.kind).astype(np.uint8)
    I.c = np.where(af, rng.choice([0.0, 0.5, 2.0], n), I.c).astype(np.float32)
    D = _dvec(n, m, 872 + n + m, np.float32)
    pr = _problem(ctx, torch, I, D)
    p0 = 0.3 + rng.random(m) * 2
    pz = p0.copy()
    pz[rng.random(m) < 0.4] = 0.0
    for p in (p0, pz):
        p = round_prices(p, np.float32)
        out = pr.dual_eval(p, lower_bound=True, support=True, j1=True)
        ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=D)
        scale = abs(float(p @ I.R)) + np.abs(ref.jobs["v"]).sum() + 1.0
        assert abs(out["g"] - ref.g) <= 1e-5 * scale
        jp = out["j_pair"].cpu().numpy().astype(np.int64)
        xp = out["x_pair"].cpu().numpy().astype(np.float64)
        Xg = dense_x(n, m, jp[:, 0], jp[:, 1], xp[:, 0], xp[:, 1])
        J = ref.jobs
        Xo = dense_x(n, m, J["jlo"], J["jhi"], J["xlo"], J["xhi"])
        assert np.all(Xg >= 0) and np.all(Xg.sum(1) <= 1 + 1e-5)
        u, _ = job_values(I.T, np.zeros(m), I.kind, I.w.astype(np.float64),
                          I.c.astype(np.float64), I.eps, Xg)
        vg = u - (Xg * D) @ p
        assert np.all(vg >= J["v"] - 1e-5 * np.maximum(1.0, np.abs(J["v"])))
        rg = (Xg * D).sum(0)
        assert np.allclose(out["r"], rg, rtol=1e-5, atol=1e-5 * max(1.0, np.abs(rg).max()))
        if np.abs(Xg - Xo).max() <= 1e-5:
            assert np.allclose(out["r"], ref.r, rtol=1e-5,
                               atol=1e-5 * max(1.0, np.abs(ref.r).max()))
    pr.close()
