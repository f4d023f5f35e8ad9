"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here reaches its expected value by a route that does not use the
oracle's segment enumeration: values printed in the paper (tests/golden),
LP solves, scalar maximisation, grid search, closed forms (water-filling,
knapsack), and invariants of duality (§3).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import brute

LOG, CAPLIN = 0, 1


# ---------------------------------------------------------------- §4.1 -----

def test_worked_example_cost_curve(golden_dir):
    G = json.load(open(os.path.join(golden_dir, "worked_example.json")))
    a, p = G["a"], G["p"]
    for t, cv in zip(G["kinks_t"], G["kinks_cost"]):
        assert oracle.cost(a, p, t) == pytest.approx(cv, abs=1e-12)
    # affine between kinks, from the kink values alone
    for t in np.linspace(0, 5, 41):
        ks, cs = G["kinks_t"], G["kinks_cost"]
        assert oracle.cost(a, p, t) == pytest.approx(float(np.interp(t, ks, cs)), abs=1e-12)
    assert math.isinf(oracle.cost(a, p, 5.01))


def test_worked_example_supports(golden_dir):
    """For 0 <= t <= 2 only resource 2 is used, for 2 < t < 5 resources 2 and
    4, at t = 5 only resource 4; resources 1 and 3 never (1-based)."""
    G = json.load(open(os.path.join(golden_dir, "worked_example.json")))
    a, p = G["a"], G["p"]
    never = {j - 1 for j in G["never_used_1based"]}
    # sweep the optimum along the whole curve with log utilities of many weights
    for w in np.geomspace(0.05, 50, 60):
        J = oracle.subproblem(a, p, LOG, w, 0.0, 0.0)
        used = {j for j, x in ((J["jlo"], J["xlo"]), (J["jhi"], J["xhi"])) if j >= 0 and x > 0}
        assert not (used & never)
        if J["t"] < 2 - 1e-12:
            assert used == {1}
        elif 2 + 1e-12 < J["t"] < 5 - 1e-12:
            assert used == {1, 3}
    J = oracle.subproblem(a, p, LOG, 1e9, 0.0, 0.0)  # cheap enough: t = 5
    assert J["t"] == pytest.approx(5.0)
    assert J["jhi"] == 3 and J["xhi"] == pytest.approx(1.0)


def test_worked_example_net_utility(golden_dir):
    """u = log t: optimum at the vertex t = 2; u = 4 log t: t = 2.4 with
    x_2 = 13/15, x_4 = 2/15 (the paper's 't about 2.4')."""
    G = json.load(open(os.path.join(golden_dir, "worked_example.json")))
    a, p = G["a"], G["p"]
    J = oracle.subproblem(a, p, LOG, 1.0, 0.0, 0.0)
    assert J["t"] == pytest.approx(2.0, abs=1e-12)
    assert J["v"] == pytest.approx(math.log(2.0) - 1.0, abs=1e-12)
    J = oracle.subproblem(a, p, LOG, 4.0, 0.0, 0.0)
    assert J["t"] == pytest.approx(G["net_utility_optimum_t_approx"], abs=1e-12)
    assert (J["jlo"], J["jhi"]) == (1, 3)
    assert J["xlo"] == pytest.approx(13 / 15, abs=1e-12)
    assert J["xhi"] == pytest.approx(2 / 15, abs=1e-12)
    # independent route: golden section on u - c_LP
    t, v = brute.job_golden(a, p, LOG, 4.0, 0.0, 1e-12)
    assert t == pytest.approx(2.4, abs=1e-6)


def test_cost_matches_lp():
    rng = np.random.default_rng(11)
    for _ in range(40):
        m = int(rng.integers(1, 6))
        a = rng.random(m) * 3
        p = rng.random(m) * 2
        for t in rng.random(4) * a.max():
            assert oracle.cost(a, p, t) == pytest.approx(brute.cost_lp(a, p, t), abs=1e-9)


def test_cost_convex_increasing():
    rng = np.random.default_rng(12)
    for _ in range(20):
        m = int(rng.integers(2, 7))
        a = rng.random(m) + 0.05
        p = rng.random(m)
        ts = np.linspace(0, a.max(), 201)
        cs = np.array([oracle.cost(a, p, t) for t in ts])
        assert cs[0] == 0.0
        assert np.all(np.diff(cs) >= -1e-12)
        assert np.all(cs[:-2] + cs[2:] - 2 * cs[1:-1] >= -1e-9)


# ---------------------------------------------------------------- §4.2 -----

@pytest.mark.parametrize("kind", [LOG, CAPLIN])
def test_segment_argmax_vs_scalar(kind):
    rng = np.random.default_rng(13 + kind)
    for _ in range(200):
        g = rng.random() * 2
        d = g + rng.random() * 2 + 1e-3
        alpha = rng.random() * 3 + 1e-3
        w = 0.5 + 1.5 * rng.random()
        c = rng.random() * 4
        eps = 1e-3
        t = oracle.segment_argmax(kind, w, c, eps, alpha, g, d)
        v = brute.u(kind, w, c, eps, t) - alpha * t
        tn, vn = brute.segment_scalar(kind, w, c, eps, alpha, 0.0, g, d)
        assert v >= vn - 1e-9
        assert g - 1e-15 <= t <= d + 1e-15
        if kind == LOG:
            assert t == pytest.approx(tn, abs=1e-6)


def test_segment_target_priority_table_cases():
    """All four cases of the capped-linear maximiser, incl. w > alpha, c < gamma."""
    f = lambda w, c, al, g, d: oracle.segment_argmax(CAPLIN, w, c, 0.0, al, g, d)
    assert f(1.0, 1.5, 2.0, 1.0, 2.0) == 1.0  # w <= alpha -> gamma
    assert f(3.0, 1.5, 2.0, 1.0, 2.0) == 1.5  # target inside
    assert f(3.0, 2.5, 2.0, 1.0, 2.0) == 2.0  # target beyond delta
    assert f(3.0, 0.5, 2.0, 1.0, 2.0) == 1.0  # target below gamma (table gap)


def test_subproblem_vs_lp_golden():
    rng = np.random.default_rng(14)
    for it in range(30):
        m = int(rng.integers(1, 6))
        a = rng.random(m) * 2 + 0.01
        p = rng.random(m) * 2 + 0.01
        kind = it % 2
        w = 0.5 + 1.5 * rng.random()
        c = 0.5 + 1.5 * rng.random()
        J = oracle.subproblem(a, p, kind, w, c, 1e-3)
        t, v = brute.job_golden(a, p, kind, w, c, 1e-3)
        assert J["v"] == pytest.approx(v, abs=1e-7)
        if kind == LOG:
            assert J["t"] == pytest.approx(t, abs=1e-5)
        # the reported allocation realises t and v
        x = np.zeros(m)
        if J["jlo"] >= 0:
            x[J["jlo"]] += J["xlo"]
        if J["jhi"] >= 0:
            x[J["jhi"]] += J["xhi"]
        assert np.all(x >= -1e-15) and x.sum() <= 1 + 1e-12
        assert float(a @ x) == pytest.approx(J["t"], abs=1e-12)
        assert brute.u(kind, w, c, 1e-3, J["t"]) - float(p @ x) == pytest.approx(J["v"], abs=1e-12)


def test_subproblem_vs_simplex_grid():
    rng = np.random.default_rng(15)
    h = 2e-3
    for it in range(12):
        m = 1 + it % 3
        a = rng.random(m) * 2 + 0.05
        p = rng.random(m) * 2 + 0.05
        kind = it % 2
        w, c = 0.5 + 1.5 * rng.random(), 0.5 + 1.5 * rng.random()
        J = oracle.subproblem(a, p, kind, w, c, 1e-3)
        vg, _ = brute.job_grid(a, p, kind, w, c, 1e-3, h=h if m < 3 else 1e-2)
        L = (w * a.max() / 1e-3 if kind == LOG else w * a.max()) + p.max()
        assert J["v"] >= vg - 1e-12
        assert J["v"] <= vg + L * m * (h if m < 3 else 1e-2)


def test_subproblem_zero_row_and_zero_price():
    J = oracle.subproblem([0.0, 0.0], [1.0, 1.0], LOG, 2.0, 0.0, 1e-3)
    assert J["t"] == 0.0 and J["jhi"] == -1 and J["v"] == pytest.approx(2 * math.log(1e-3))
    J = oracle.subproblem([0.0, 0.0], [1.0, 1.0], CAPLIN, 2.0, 1.0, 1e-3)
    assert J["t"] == 0.0 and J["v"] == 0.0
    # a free resource: take all of the best free one
    J = oracle.subproblem([0.5, 2.0, 1.0], [0.0, 0.0, 3.0], LOG, 1.0, 0.0, 1e-3)
    assert J["t"] == pytest.approx(2.0) and J["jhi"] == 1 and J["v"] == pytest.approx(math.log(2.001))


# ------------------------------------------------------------ §3 duality ---

def _inst(n, m, seed, **kw):
    return synth.random_small(n, m, seed, **kw)


def test_weak_duality_random_prices():
    I = _inst(300, 4, 1)
    rng = np.random.default_rng(16)
    for _ in range(10):
        p = rng.random(4) * 3
        d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
        U, du = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, d.r, d.jobs)
        assert d.g >= U - 1e-9
        # the scaled allocation is feasible
        X = oracle.dense_allocation(I.n, I.m, d.jobs)
        s = np.where(d.r > I.R, I.R / np.maximum(d.r, 1e-300), 1.0)
        Xs = X * s[None, :]
        assert np.all(Xs.sum(0) <= I.R * (1 + 1e-12))
        assert np.all(Xs.sum(1) <= 1 + 1e-12)
        # better-conditioned form of the gap agrees
        assert d.g - U == pytest.approx(float(p @ (I.R - d.r)) + du, rel=1e-9, abs=1e-9)


def test_dual_convex_along_segments():
    I = _inst(200, 3, 2)
    rng = np.random.default_rng(17)
    for _ in range(10):
        p1, p2 = rng.random(3) * 3, rng.random(3) * 3
        g = lambda p: oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p).g
        for th in (0.25, 0.5, 0.75):
            assert g(th * p1 + (1 - th) * p2) <= th * g(p1) + (1 - th) * g(p2) + 1e-9


def test_danskin_gradient_finite_difference():
    """q = R - r is the gradient of g where g is differentiable (§3)."""
    I = _inst(60, 3, 3, log_frac=1.0)
    rng = np.random.default_rng(18)
    for _ in range(5):
        p = 0.5 + rng.random(3) * 2
        d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p)
        for j in range(3):
            h = 1e-6
            e = np.zeros(3)
            e[j] = h
            gp = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p + e).g
            gm = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p - e).g
            assert (gp - gm) / (2 * h) == pytest.approx(I.R[j] - d.r[j], rel=1e-6, abs=1e-6)


def test_upper_bound_max_throughput():
    """U* <= sum_i u_i(max_j a_ij) (§2.4) and g(p*) >= U*."""
    I = _inst(200, 4, 4)
    p, info = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R, tol_rel=1e-9, max_iter=200)
    ub = sum(brute.u(I.kind[i], I.w[i], I.c[i], I.eps, I.T[i].max()) for i in range(I.n))
    assert info["U"] <= ub + 1e-9
    assert info["g"] >= info["U"] - 1e-9


# ----------------------------------------------------- whole problem pins ---

def test_problem_grid_tiny():
    rng = np.random.default_rng(19)
    for it in range(3):
        n, m = 2, 2
        T = rng.random((n, m)) + 0.1
        kind = np.array([it % 2, (it + 1) % 2], np.uint8)
        w = 0.5 + 1.5 * rng.random(n)
        c = 0.5 + 1.5 * rng.random(n)
        R = np.array([0.6, 0.5])
        eps = 0.05
        h = 0.02
        Ug = brute.problem_grid(T, kind, w, c, eps, R, h=h)
        p, info = oracle.solve(T, w, c, kind, eps, R, tol_rel=1e-10, max_iter=400)
        Lip = float(np.max(w[:, None] * T) / eps) * 2
        # strong duality: the dual optimum equals U*; grid is within L*h below it
        assert Ug <= info["g"] + 1e-7
        assert info["g"] <= Ug + Lip * h * m


def test_waterfilling_single_resource():
    rng = np.random.default_rng(20)
    n = 2000
    a = 0.1 + 0.9 * rng.random(n)
    w = 0.5 + 1.5 * rng.random(n)
    R = 300.0
    ps, Us = brute.waterfill_m1(a, w, 1e-3, R)
    T = a[:, None]
    p, info = oracle.solve(T, w, np.zeros(n), np.zeros(n, np.uint8), 1e-3, np.array([R]),
                           tol_rel=1e-12, max_iter=300)
    assert p[0] == pytest.approx(ps, rel=1e-7)
    assert info["g"] == pytest.approx(Us, rel=1e-9)
    assert info["U"] == pytest.approx(Us, rel=1e-9)


def test_identical_jobs_knapsack():
    a = np.array([0.3, 0.9, 0.6])
    n = 500
    R = np.array([200.0, 100.0, 120.0])
    T = np.tile(a, (n, 1))
    w = np.ones(n)
    tau = brute.knapsack_identical(a, R, n)
    Ustar = n * math.log(tau + 1e-3)
    p, info = oracle.solve(T, w, np.zeros(n), np.zeros(n, np.uint8), 1e-3, R, tol_rel=1e-12,
                           max_iter=400)
    # the dual optimum is U* (strong duality); the scaled recovery can lose
    # whole jobs at the massive tie, so only the upper bound is tight here
    assert info["g"] == pytest.approx(Ustar, rel=1e-7)
    assert info["U"] <= Ustar + 1e-9


def test_linear_utility_lp():
    """Capped-linear with c >= max_j a_ij is linear utility: U* is an LP."""
    I = _inst(80, 3, 5)
    c = np.full(I.n, 10.0)
    kind = np.ones(I.n, np.uint8)
    Ulp = brute.lp_linear(I.T, I.w, I.R)
    p, info = oracle.solve(I.T, I.w, c, kind, I.eps, I.R, tol_rel=1e-10, max_iter=400)
    assert info["g"] == pytest.approx(Ulp, rel=1e-7)


def test_price_is_sensitivity_of_optimum():
    """p* = grad_R U*(R) (§3, eq. e-pstar-grad), by central differences of the
    dual optimum g(p*) = U* in R."""
    I = _inst(400, 3, 6, log_frac=1.0)
    p, info = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R, tol_rel=1e-12, max_iter=300)
    for j in range(3):
        h = 2.0
        e = np.zeros(3)
        e[j] = h
        _, ip = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R + e, p0=p, tol_rel=1e-12,
                             max_iter=300)
        _, im = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R - e, p0=p, tol_rel=1e-12,
                             max_iter=300)
        assert (ip["g"] - im["g"]) / (2 * h) == pytest.approx(p[j], rel=2e-2)


def test_kkt_at_convergence():
    I = _inst(20000, 4, 7, log_frac=1.0)
    p, info = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R, tol_rel=1e-6, max_iter=200)
    # the column-scaling recovery leaves a floor of order 1/n at ties
    assert info["rel_gap"] <= 5e-5
    d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
    X = oracle.dense_allocation(I.n, I.m, d.jobs)
    assert np.all((X > 0).sum(1) <= 2)
    s = np.where(d.r > I.R, I.R / d.r, 1.0)
    rt = (X * s).sum(0)
    assert np.all(rt <= I.R * (1 + 1e-12))
    # complementary slackness: priced resources are (nearly) used up
    gap = info["g"] - info["U"]
    assert np.all(p * (I.R - rt) <= gap + 1e-9)
    assert np.all(p >= 0)


def test_trace_example_gap_definition(golden_dir):
    """The printed gap is dual value per job minus utility per job (§6.1)."""
    G = json.load(open(os.path.join(golden_dir, "trace_example.json")))
    for L in G["lines"]:
        assert "%.2e" % (L["dual_value"] - L["utility"]) == L["gap_printed"]
    assert G["final_residual"] < G["tolerance_per_job"]


def test_generator_determinism():
    a = synth.mixed_16(n=70000, m=16)
    b = synth.mixed_16(n=70000, m=16)
    assert a.T.tobytes() == b.T.tobytes() and a.w.tobytes() == b.w.tobytes()
    rows = synth.roofline_rows(65530, 65600, n=200000, m=8)
    full = synth.roofline_64(n=200000, m=8)
    assert rows[0].tobytes() == full.T[65530:65600].tobytes()
    assert rows[1].tobytes() == full.kind[65530:65600].tobytes()


# ------------------------------------------------- §5 initialisation -----

def _init_instance(seed, n=40, m=3, R_scale=0.2):
    rng = np.random.default_rng(seed)
    T = 0.2 + rng.random((n, m))
    w = 0.5 + rng.random(n)
    kind = (rng.random(n) < 0.5).astype(np.uint8)
    R = R_scale * n / m * (0.5 + rng.random(m))
    return T, w, kind, R


def _phi(T, w, c, kind, eps, y):
    """sum_i u_i(a_i^T y), numpy."""
    t = T @ y
    return float(np.sum(np.where(kind == LOG, w * np.log(t + eps), w * np.minimum(t, c))))


def _caps_away_from_kinks(T, kind, y, rng):
    # capped jobs strictly below or above their cap at the uniform allocation,
    # so the finite differences below do not straddle a kink
    t = T @ y
    below = rng.random(len(t)) < 0.5
    return np.where(kind == LOG, 0.0, np.where(below, t * 2.0 + 0.5, t * 0.5))


def test_init_prices_gradient_of_utility_at_R():
    """p1 = grad_R sum_i u_i(a_i^T R / n) when 1^T R / n <= 1, by central
    differences (eq. e-initialization, the sensitivity reading of §5)."""
    T, w, kind, R = _init_instance(3)
    n, m = T.shape
    assert R.sum() / n <= 1
    c = _caps_away_from_kinks(T, kind, R / n, np.random.default_rng(4))
    p = oracle.init_prices(T, w, c, kind, 1e-3, R)
    for j in range(m):
        h = 1e-5 * R[j]
        e = np.zeros(m)
        e[j] = h
        fd = (_phi(T, w, c, kind, 1e-3, (R + e) / n) - _phi(T, w, c, kind, 1e-3, (R - e) / n)) / (2 * h)
        assert p[j] == pytest.approx(fd, rel=1e-7)


def test_init_prices_rescaled_share_when_limits_exceed_one_unit():
    """kappa = 1^T R / n > 1: every job gets x = R / (kappa n) (1^T x = 1), so
    p1 = (1/n) grad_y sum_i u_i(a_i^T y) at y = x, and scaling R up leaves it
    unchanged."""
    T, w, kind, R = _init_instance(5, R_scale=2.0)
    n, m = T.shape
    kappa = R.sum() / n
    assert kappa > 1
    x = R / (kappa * n)
    c = _caps_away_from_kinks(T, kind, x, np.random.default_rng(6))
    p = oracle.init_prices(T, w, c, kind, 1e-3, R)
    for j in range(m):
        h = 1e-6
        e = np.zeros(m)
        e[j] = h
        fd = (_phi(T, w, c, kind, 1e-3, x + e) - _phi(T, w, c, kind, 1e-3, x - e)) / (2 * h) / n
        assert p[j] == pytest.approx(fd, rel=1e-7)
    assert np.allclose(oracle.init_prices(T, w, c, kind, 1e-3, 3.0 * R), p, rtol=1e-13)
    # below kappa = 1 the share follows R itself: p1 changes when R is scaled
    Rs = R / (2 * kappa)
    assert not np.allclose(oracle.init_prices(T, w, c, kind, 1e-3, Rs),
                           oracle.init_prices(T, w, c, kind, 1e-3, 0.5 * Rs))


def test_init_prices_identical_jobs():
    """n copies of one job: p1 = u'(a^T x) a."""
    a = np.array([0.5, 2.0, 1.25])
    n = 7
    R = np.array([0.5, 1.0, 2.0])
    T = np.tile(a, (n, 1))
    x = R / n
    t = a @ x
    p = oracle.init_prices(T, np.full(n, 1.5), np.zeros(n), np.zeros(n, np.uint8), 1e-3, R)
    assert np.allclose(p, 1.5 / (t + 1e-3) * a, rtol=1e-14)
    # capped linear below its cap: slope w; at or above the cap: 0
    p = oracle.init_prices(T, np.full(n, 1.5), np.full(n, t + 1), np.ones(n, np.uint8), 1e-3, R)
    assert np.allclose(p, 1.5 * a, rtol=1e-14)
    p = oracle.init_prices(T, np.full(n, 1.5), np.full(n, t / 2), np.ones(n, np.uint8), 1e-3, R)
    assert np.all(p == 0)


# ---------------------------------------- §6.2 printed statistics -----

def _e1_stats(T, w, c, kind, X):
    used = X > 1e-9
    out = {"two": float(np.mean(used.sum(1) == 2)), "slack": float(np.mean(X.sum(1) < 1 - 1e-6))}
    if kind[0] == CAPLIN:
        reach = (T * X).sum(1) >= c * (1 - 1e-5)
        out.update(reach=float(reach.mean()), w2=float(reach[w == 2].mean()),
                   miss1=float(1 - reach[w == 1].mean()))
    return out


@pytest.mark.parametrize("kind", ["log", "target"])
def test_medium_example_printed_statistics(kind):
    """§6.2's medium-size example (n scaled to 2e5, R scaled with it), solved
    from the paper's start to its tolerance g - U <= 1e-3 n: the allocation's
    outcome shares match the ones the paper prints (log: about 17 % of jobs on
    two resources, 18 % with slack; target-priority: 50 % with slack, over 95 %
    reaching the target, virtually all high-priority jobs and all but about
    10 % of low-priority ones).  The target-priority share on two resources
    (printed 67 %) is not pinned: resource 1 is free at the optimum, so jobs
    have equally good allocations with one or two resources."""
    n = 200000
    I = synth.e1_instance(kind, n=n, dtype=np.float64)
    p0 = oracle.init_prices(I.T, I.w, I.c, I.kind, I.eps, I.R)
    p, info = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R, p0=p0, tol_rel=0.0,
                           tol_abs=1e-3 * n, max_iter=300)
    assert info["status"] == 0 and info["g"] - info["U"] <= 1e-3 * n
    d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
    s = _e1_stats(I.T, I.w, I.c, I.kind, oracle.dense_allocation(n, 4, d.jobs))
    if kind == "log":
        assert abs(s["two"] - 0.17) <= 0.02 and abs(s["slack"] - 0.18) <= 0.02
    else:
        assert abs(s["slack"] - 0.50) <= 0.02
        assert s["reach"] > 0.95 and s["w2"] >= 0.99
        assert 0.02 <= s["miss1"] <= 0.15


def test_free_resource_segment_follows_the_tables():
    """A free resource (p_j = 0) gives a zero-slope segment on the envelope:
    the log closed form takes its right end (w / alpha is infinite), and the
    target-priority table's w > alpha row stops at the target (eq.
    e-opt-t-target) -- both are optimal there, the table fixes the choice."""
    assert oracle.segment_argmax(CAPLIN, 1.5, 0.2, 0.0, 0.0, 0.0, 0.3) == 0.2
    assert oracle.segment_argmax(CAPLIN, 1.5, 0.5, 0.0, 0.0, 0.0, 0.3) == 0.3
    assert oracle.segment_argmax(LOG, 1.5, 0.0, 1e-3, 0.0, 0.0, 0.3) == 0.3
    J = oracle.subproblem([0.3, 0.9], [0.0, 2.0], CAPLIN, 1.0, 0.2, 0.0)
    assert J["t"] == pytest.approx(0.2) and J["xhi"] == pytest.approx(0.2 / 0.3)


# -------------------------------------------- alpha-fair utilities ----

AFAIR = 2


@pytest.mark.parametrize("a", [0.5, 2.0, 3.5])
def test_alpha_fair_segment_argmax_vs_scalar(a):
    """Alpha-fair maximiser on a segment ((u')^{-1} projected, §4.2's log
    rule generalised) against numerical maximisation of u(t) - alpha t."""
    rng = np.random.default_rng(int(17 * a))
    for _ in range(200):
        g = rng.random() * 2
        d = g + rng.random() * 2 + 1e-3
        alpha = rng.random() * 3 + 1e-3
        w = 0.5 + 1.5 * rng.random()
        t = oracle.segment_argmax(AFAIR, w, a, 1e-3, alpha, g, d)
        tn, vn = brute.segment_scalar(AFAIR, w, a, 1e-3, alpha, 0.0, g, d)
        assert brute.u(AFAIR, w, a, 1e-3, t) - alpha * t >= vn - 1e-9
        assert t == pytest.approx(tn, abs=1e-5)


def test_alpha_fair_linear_case_takes_an_end():
    """Exponent 0 is linear utility: the right end when w > alpha, else the left."""
    assert oracle.segment_argmax(AFAIR, 2.0, 0.0, 0.0, 1.5, 0.5, 1.0) == 1.0
    assert oracle.segment_argmax(AFAIR, 1.0, 0.0, 0.0, 1.5, 0.5, 1.0) == 0.5
    assert oracle.segment_argmax(AFAIR, 1.5, 0.0, 0.0, 1.5, 0.5, 1.0) == 0.5


@pytest.mark.parametrize("a", [0.0, 0.5, 2.0])
def test_alpha_fair_job_optimum_vs_lp_golden(a):
    rng = np.random.default_rng(int(23 + 10 * a))
    for _ in range(30):
        m = int(rng.integers(1, 6))
        A = rng.random(m) * 2 + 0.01
        p = rng.random(m) * 2 + 0.01
        w = 0.5 + 1.5 * rng.random()
        J = oracle.subproblem(A, p, AFAIR, w, a, 1e-3)
        t, v = brute.job_golden(A, p, AFAIR, w, a, 1e-3)
        assert J["v"] == pytest.approx(v, abs=1e-7)
        if a > 0:
            assert J["t"] == pytest.approx(t, abs=1e-5)


def test_alpha_fair_near_one_is_log():
    """The family's exponent 1 is the log utility: nearby exponents give
    nearly the log optimum (continuity in the exponent)."""
    rng = np.random.default_rng(29)
    for _ in range(20):
        A = rng.random(4) * 2 + 0.01
        p = rng.random(4) * 2 + 0.01
        Jl = oracle.subproblem(A, p, LOG, 1.3, 0.0, 1e-3)
        for a in (1.0 - 1e-7, 1.0 + 1e-7):
            Ja = oracle.subproblem(A, p, AFAIR, 1.3, a, 1e-3)
            assert Ja["t"] == pytest.approx(Jl["t"], abs=1e-5)
        assert oracle.subproblem(A, p, AFAIR, 1.3, 1.0, 1e-3)["t"] == pytest.approx(Jl["t"], abs=1e-12)


def test_alpha_fair_zero_is_the_linear_lp():
    """Exponent 0 (u = w (t + eps), eps = 0: linear utility) over a whole
    problem: the dual optimum equals the LP optimum."""
    I = _inst(80, 3, 7)
    kind = np.full(I.n, AFAIR, np.uint8)
    c = np.zeros(I.n)
    Ulp = brute.lp_linear(I.T, I.w, I.R)
    p, info = oracle.solve(I.T, I.w, c, kind, 0.0, I.R, tol_rel=1e-10, max_iter=400)
    assert info["g"] == pytest.approx(Ulp, rel=1e-7)


def test_alpha_fair_initial_prices_gradient():
    """eq. e-initialization with alpha-fair jobs: central differences of
    sum_i u_i(a_i^T R / n)."""
    rng = np.random.default_rng(31)
    n, m = 50, 3
    T = 0.2 + rng.random((n, m))
    w = 0.5 + rng.random(n)
    c = rng.choice([0.0, 0.5, 2.0], n)
    kind = np.full(n, AFAIR, np.uint8)
    R = 0.2 * n / m * (0.5 + rng.random(m))
    p = oracle.init_prices(T, w, c, kind, 1e-3, R)
    phi = lambda y: sum(brute.u(AFAIR, w[i], c[i], 1e-3, float(T[i] @ y)) for i in range(n))
    for j in range(m):
        h = 1e-5 * R[j]
        e = np.zeros(m)
        e[j] = h
        fd = (phi((R + e) / n) - phi((R - e) / n)) / (2 * h)
        assert p[j] == pytest.approx(fd, rel=1e-7)


# ------------------------------------ per-job demands (extensions) ----

def test_uniform_demand_is_a_rescaling():
    """Demand d_i = 2 for every job with limits 2R is the same primal problem
    as d = 1 with R: at prices p/2 the dual value, every job's allocation and
    (twice) the usage agree."""
    I = _inst(300, 4, 40)
    rng = np.random.default_rng(41)
    p = 0.2 + rng.random(4) * 2
    a = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
    b = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, 2 * I.R, p / 2, per_job=True,
                         d=np.full(I.n, 2.0))
    assert b.g == pytest.approx(a.g, rel=1e-12)
    assert np.allclose(b.r, 2 * a.r, rtol=1e-12)
    for k in ("jlo", "jhi"):
        assert np.array_equal(a.jobs[k], b.jobs[k])
    assert np.allclose(a.jobs["xhi"], b.jobs["xhi"], rtol=1e-12)


def test_demands_whole_problem_grid():
    """Two jobs with different demands: the dual optimum equals the best
    grid allocation with sum_i d_i x_i <= R (strong duality)."""
    rng = np.random.default_rng(42)
    for _ in range(3):
        n, m = 2, 2
        T = 0.3 + rng.random((n, m))
        w = 0.5 + rng.random(n)
        c = np.zeros(n)
        kind = np.zeros(n, np.uint8)
        d = np.array([1.0, 2.5])
        R = np.array([0.9, 0.8])
        eps, h = 0.05, 0.02
        Ug = brute.problem_grid(T, kind, w, c, eps, R, h=h, d=d)
        p, info = oracle.solve(T, w, c, kind, eps, R, tol_rel=1e-10, max_iter=400, d=d)
        Lip = float(np.max(w[:, None] * T) / eps) * 2
        assert Ug <= info["g"] + 1e-7
        assert info["g"] <= Ug + Lip * h * m


def test_demands_kkt_at_optimum():
    """With heterogeneous demands: at the solution, usage r = sum_i d_i x_i
    respects R up to the gap, and prices are zero on slack resources.  (Log
    jobs alone would not show the demands: x = w / (d p) makes d x
    independent of d; capped-linear jobs do.)"""
    I = _inst(2000, 3, 43)
    d = 0.5 + np.random.default_rng(44).random(I.n) * 2
    p, info = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R, tol_rel=1e-9, max_iter=400, d=d)
    assert info["rel_gap"] <= 1e-4  # the recovery's floor for n = 2000 with capped jobs
    r = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, d=d).r
    assert np.all(r <= I.R * (1 + 5e-3))
    assert np.all(p * np.abs(I.R - r) <= 5e-3 * np.abs(p @ I.R) + 1e-9)
    # a demand-blind usage would not balance: sum_i x_i differs from R
    r1 = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p).r
    assert np.max(np.abs(r1 - I.R) / I.R) > 0.01


# ------------------------------- per-job demand vectors (extensions) ----

def test_demand_vectors_with_equal_columns_are_scalar_demands():
    """A demand vector whose entries all equal d_i is the scalar demand d_i."""
    I = _inst(300, 4, 45)
    rng = np.random.default_rng(46)
    d = 0.5 + rng.random(I.n) * 2
    D = np.repeat(d[:, None], I.m, axis=1)
    p = 0.2 + rng.random(4) * 2
    a = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=d)
    b = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True, d=D)
    assert b.g == a.g and np.array_equal(a.r, b.r)
    for k in ("jlo", "jhi", "xlo", "xhi"):
        assert np.array_equal(a.jobs[k], b.jobs[k])


def test_demand_vectors_danskin_gradient():
    """With a demand vector per job, job i pays d_ij p_j per unit of x_ij, so
    dg/dp_j = R_j - sum_i d_ij x_ij: central differences of g in FP64 (log
    jobs, where g is differentiable) against R - r.  A usage that ignored the
    demands, or took them from the wrong column, fails this."""
    I = _inst(80, 4, 47, log_frac=1.0)
    rng = np.random.default_rng(48)
    D = 0.4 + rng.random((I.n, I.m)) * 2.5
    for _ in range(4):
        p = 0.5 + rng.random(4) * 2
        r = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, d=D).r
        r1 = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p).r
        assert np.max(np.abs(r - r1) / r1) > 0.05  # the demands matter here
        for j in range(4):
            h = 1e-6
            e = np.zeros(4)
            e[j] = h
            gp = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p + e, d=D).g
            gm = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p - e, d=D).g
            assert (gp - gm) / (2 * h) == pytest.approx(I.R[j] - r[j], rel=1e-6, abs=1e-6)


def test_demand_vectors_job_sees_scaled_prices():
    """Each job's optimum under a demand vector is its subproblem at the
    prices d_i * p (the only change the extension makes), checked by scalar
    maximisation of u(t) - c(t) on the LP cost curve at those prices."""
    rng = np.random.default_rng(49)
    for _ in range(20):
        m = 3
        T = 0.2 + rng.random((1, m))
        D = 0.3 + rng.random((1, m)) * 3
        w = np.array([0.5 + rng.random()])
        p = 0.2 + rng.random(m)
        R = np.ones(m)
        res = oracle.dual_eval(T, w, np.zeros(1), np.zeros(1, np.uint8), 1e-2, R, p,
                               per_job=True, d=D)
        pd = D[0] * p
        t_star, v_star = brute.job_golden(T[0], pd, LOG, w[0], 0.0, 1e-2)
        assert res.jobs["t"][0] == pytest.approx(t_star, abs=1e-5)
        assert res.jobs["v"][0] == pytest.approx(v_star, abs=1e-7)


def test_demand_vectors_strong_duality():
    """Three log jobs with demand vectors: the minimum of the oracle's dual
    function (found by a derivative-free search over p >= 0) equals the
    primal optimum with sum_i d_ij x_ij <= R_j for every j, found by a
    general nonlinear solver on the allocation itself (§3, strong duality).
    (Tiny instances put the dual optimum on a kink, which the price loop
    approaches slowly; the search here only needs function values.)"""
    from scipy.optimize import minimize
    rng = np.random.default_rng(50)
    for k in range(3):
        n, m = 3, 3
        T = 0.3 + rng.random((n, m))
        w = 0.5 + rng.random(n)
        D = 0.4 + rng.random((n, m)) * 2.5
        R = 0.4 + rng.random(m) * 0.6
        eps, z, kind = 0.05, np.zeros(n), np.zeros(n, np.uint8)
        Us = brute.problem_slsqp_log(T, w, eps, R, d=D, seed=k)
        assert abs(Us - brute.problem_slsqp_log(T, w, eps, R, seed=k)) > 1e-2
        g = lambda q: oracle.dual_eval(T, w, z, kind, eps, R, np.abs(q), d=D).g
        best = min(minimize(g, 0.5 + rng.random(m), method="Nelder-Mead",
                            options={"xatol": 1e-12, "fatol": 1e-14, "maxfev": 40000}).fun
                   for _ in range(2))
        assert best == pytest.approx(Us, abs=1e-8)


def test_demand_vectors_kkt_at_optimum():
    """Mixed jobs with demand vectors: at the solution the usage
    sum_i d_ij x_ij respects R up to the gap and prices vanish on slack
    resources; a demand-blind usage would not balance."""
    I = _inst(2000, 3, 51)
    D = 0.5 + np.random.default_rng(52).random((I.n, I.m)) * 2
    p, info = oracle.solve(I.T, I.w, I.c, I.kind, I.eps, I.R, tol_rel=1e-9, max_iter=400, d=D)
    # the recovery's floor: a capped job flipping at a tie moves r_j by up to
    # d_ij, so the floor is a few times that of unit demands
    assert info["rel_gap"] <= 5e-4
    r = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, d=D).r
    assert np.all(r <= I.R * (1 + 5e-3))
    assert np.all(p * np.abs(I.R - r) <= 5e-3 * np.abs(p @ I.R) + 1e-9)
    r1 = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p).r
    assert np.max(np.abs(r1 - I.R) / I.R) > 0.01


def test_demand_vectors_init_prices():
    """The data-dependent start with demands divides job i's term for
    resource j by d_ij: equal columns give the start of the weights w_i / d_i,
    and scaling column j of every demand vector by lam scales p_j by 1/lam
    and leaves the other prices unchanged."""
    I = _inst(500, 4, 53)
    rng = np.random.default_rng(54)
    d = 0.5 + rng.random(I.n) * 2
    D = np.repeat(d[:, None], I.m, axis=1)
    a = oracle.init_prices(I.T, I.w, I.c, I.kind, I.eps, I.R, d=D)
    b = oracle.init_prices(I.T, I.w / d, I.c, I.kind, I.eps, I.R)
    assert np.allclose(a, b, rtol=1e-12)
    D = 0.5 + rng.random((I.n, I.m)) * 2
    p0 = oracle.init_prices(I.T, I.w, I.c, I.kind, I.eps, I.R, d=D)
    D2 = D.copy()
    D2[:, 2] *= 4.0
    p1 = oracle.init_prices(I.T, I.w, I.c, I.kind, I.eps, I.R, d=D2)
    assert p1[2] == pytest.approx(p0[2] / 4, rel=1e-12)
    for j in (0, 1, 3):
        assert p1[j] == pytest.approx(p0[j], rel=1e-12)


# ------------------------------- first vertex in the element type -----

def test_first_vertex_matches_exact_argmax_off_ties():
    """The element-type decision equals the exact argmax of a_ij / p_j (numpy,
    FP64) wherever the best key beats the runner-up by more than 1e-6."""
    for dtype in (np.float32, np.float64):
        I = synth.random_small(4000, 16, seed=90, dtype=dtype, zero_frac=0.1)
        p = (0.2 + np.random.default_rng(91).random(16) * 2).astype(dtype).astype(np.float64)
        j1 = oracle.first_vertex(I.T, p)
        keys = I.T.astype(np.float64) / p[None, :]
        srt = np.sort(keys, axis=1)
        clear = (srt[:, -1] - srt[:, -2]) > 1e-6 * srt[:, -1]
        assert clear.mean() > 0.99
        assert np.array_equal(j1[clear], np.argmax(keys, axis=1)[clear])


def test_first_vertex_ties_zero_prices_and_zero_rows():
    for dtype in (np.float32, np.float64):
        T = np.array([[1.0, 2.0, 0.5],     # keys 1, 1, 0.25: equal keys -> lowest index
                      [0.5, 2.0, 1.0],     # two free resources: the first +inf key wins
                      [0.0, 0.0, 0.0],     # nothing to buy
                      [0.0, 3.0, 0.0]],    # zero entries never win
                     dtype=dtype)
        p = np.array([1.0, 2.0, 2.0])
        pz = np.array([0.0, 0.0, 3.0])
        assert list(oracle.first_vertex(T[[0, 2, 3]], p)) == [0, -1, 1]
        assert oracle.first_vertex(T[[1]], pz)[0] == 0
        assert oracle.first_vertex(np.array([[0.0, 2.0, 1.0]], dtype=dtype), pz)[0] == 1


def test_first_vertex_decided_in_single_precision():
    """Keys that differ below FP32 resolution tie in FP32 (lowest index) but
    not in FP64: the decision is taken in the data's own precision."""
    T64 = np.array([[1.0, 1.0 + 1e-9]])
    p = np.array([1.0, 1.0])
    assert oracle.first_vertex(T64, p)[0] == 1
    assert oracle.first_vertex(T64.astype(np.float32), p)[0] == 0


# ------------------------------- efficiency-per-price margin (j1) -----

def _keys64(T, p):
    """Efficiency per price a_ij / p_j in FP64: p_j = 0 gives +inf for
    a_ij > 0, and a_ij = 0 gives key 0 (never chosen), whatever p_j."""
    T = np.asarray(T, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = np.where(p[None, :] > 0, T / np.where(p > 0, p, 1.0)[None, :], np.inf)
    return np.where(T > 0, k, 0.0)


def _margin_numpy(T, p):
    """(j1, margin) from the sorted keys of each row: j1 = first index of the
    largest key (-1 when every key is 0), margin = (k1 - k2) / k1 with k2 the
    largest key among the other entries; 0 for equal keys, 1 when only the
    best key is infinite."""
    K = _keys64(T, p)
    j1 = np.argmax(K, axis=1)
    k1 = K[np.arange(len(K)), j1]
    K2 = K.copy()
    K2[np.arange(len(K)), j1] = -1.0
    k2 = K2.max(axis=1) if K.shape[1] > 1 else np.zeros(len(K))
    k2 = np.maximum(k2, 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        mg = np.where(np.isinf(k1), np.where(np.isinf(k2), 0.0, 1.0), (k1 - k2) / k1)
    mg = np.where(k1 > 0, mg, 0.0)
    return np.where(k1 > 0, j1, -1), mg


@pytest.mark.parametrize("m", [1, 2, 5, 16, 64])
def test_margin1_matches_keys_computed_independently(m):
    """The oracle's first vertex and its margin equal a numpy computation of
    the sorted keys, on rows with zero entries, zero prices and exact ties."""
    I = synth.random_small(3000, m, seed=2000 + m, dtype=np.float64, zero_frac=0.2)
    rng = np.random.default_rng(2100 + m)
    I.T[::29] = 0.0                                  # rows with nothing to buy
    if m > 1:
        I.T[5::31, m - 1] = I.T[5::31, 0]            # equal keys under equal prices
    p = 0.2 + rng.random(m) * 2
    if m > 1:
        p[m - 1] = p[0]
    for pp in (p, np.where(np.arange(m) % 4 == 1, 0.0, p)):
        ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, pp, per_job=True)
        j1, mg = _margin_numpy(I.T, pp)
        assert np.array_equal(ref.jobs["j1"], j1)
        np.testing.assert_allclose(ref.jobs["margin1"], mg, rtol=1e-12, atol=0)


def test_margin1_special_cases():
    p = np.array([1.0, 2.0, 0.5])
    cases = [
        ([1.0, 2.0, 0.5], 0.0),        # keys 1, 1, 1: exact three-way tie
        ([2.0, 1.0, 0.25], 0.75),      # keys 2, 0.5, 0.5
        ([0.0, 0.0, 0.0], 0.0),        # nothing to buy: j1 = -1
        ([0.0, 0.0, 0.3], 1.0),        # a single positive key
    ]
    for row, want in cases:
        J = oracle.subproblem(np.array(row), p, LOG, 1.0, 0.0, 1e-3)
        assert J["margin1"] == pytest.approx(want, abs=1e-15), (row, J)
    pz = np.array([0.0, 0.0, 1.0])
    assert oracle.subproblem(np.array([1.0, 2.0, 5.0]), pz, LOG, 1.0, 0.0, 1e-3)["margin1"] == 0.0
    J = oracle.subproblem(np.array([1.0, 0.0, 5.0]), pz, LOG, 1.0, 0.0, 1e-3)
    assert J["j1"] == 0 and J["margin1"] == 1.0    # one free resource beats every finite key
    J = oracle.subproblem(np.array([0.0, 0.0, 5.0]), pz, LOG, 1.0, 0.0, 1e-3)
    assert J["j1"] == 2 and J["margin1"] == pytest.approx(1.0)  # a = 0 never wins at p = 0


def test_margin1_is_the_relative_price_change_that_moves_the_argmax():
    """margin1 = mu means: raising the winner's price by a factor below
    1 / (1 - mu) keeps it the best efficiency per price, and raising it by
    more hands the first vertex to another resource (a numpy argmax decides,
    not the oracle)."""
    rng = np.random.default_rng(2200)
    T = 0.1 + rng.random((400, 6))
    p = 0.2 + rng.random(6)
    ref = oracle.dual_eval(T, np.ones(400), np.zeros(400), np.zeros(400, np.uint8), 1e-3,
                           np.ones(6), p, per_job=True)
    checked = 0
    for i in range(400):
        j1, mu = int(ref.jobs["j1"][i]), float(ref.jobs["margin1"][i])
        if not 1e-4 < mu < 0.99:
            continue
        for f, stays in ((1.0 - 1e-3, True), (1.0 + 1e-3, False)):
            q = p.copy()
            q[j1] *= f / (1.0 - mu)
            assert (int(np.argmax(T[i] / q)) == j1) == stays, (i, mu, f)
        checked += 1
    assert checked > 300


def _u(kind, w, c, eps, t):
    return w * math.log(t + eps) if kind == LOG else w * min(t, c)


def _numeric_candidates(a, p, kind, w, c, eps):
    """Every candidate allocation of one job with its net utility: the origin
    and, for each pair of ends (origin or resource k, resource l) with
    a_k < a_l, the best point of that segment found by a bounded scalar
    search over t (the allocation then follows from eq. e-xixj).  Returns a
    list of (value, {resource: share})."""
    from scipy.optimize import minimize_scalar
    m = len(a)
    out = [(_u(kind, w, c, eps, 0.0), {})]
    ends = [(-1, 0.0, 0.0)] + [(k, a[k], p[k]) for k in range(m)]
    for k, ak, pk in ends:
        for l in range(m):
            al, pl = a[l], p[l]
            if not ak < al:
                continue

            def neg(t):
                xl = (t - ak) / (al - ak)
                xk = (al - t) / (al - ak)
                return -(_u(kind, w, c, eps, t) - pk * xk - pl * xl)

            res = minimize_scalar(neg, bounds=(ak, al), method="bounded",
                                  options={"xatol": 1e-13})
            best_t, best_f = res.x, res.fun
            for t in (ak, al):  # the bounded search may stop just inside an end
                if neg(t) < best_f:
                    best_t, best_f = t, neg(t)
            xl = (best_t - ak) / (al - ak)
            xk = (al - best_t) / (al - ak)
            x = {}
            if k >= 0 and xk > 0:
                x[k] = xk
            if xl > 0:
                x[l] = x.get(l, 0.0) + xl
            out.append((-best_f, x))
    return out


def _margin_numeric(a, p, kind, w, c, eps, best_x, same_tol=1e-6):
    cands = _numeric_candidates(a, p, kind, w, c, eps)
    v1 = max(v for v, _ in cands)
    keys = set(best_x)
    diff = [v for v, x in cands
            if any(abs(x.get(j, 0.0) - best_x.get(j, 0.0)) > same_tol for j in keys | set(x))]
    if not diff:
        return math.inf
    return (v1 - max(diff)) / max(1.0, abs(v1))


@pytest.mark.parametrize("kind", [LOG, CAPLIN])
def test_marginx_against_a_numeric_search_of_every_candidate(kind):
    """The allocation margin (how far a job's optimum is from a tie with a
    different allocation) against candidates found by a bounded scalar search
    on every segment, on random jobs with up to four resources."""
    rng = np.random.default_rng(2300 + kind)
    checked = 0
    for trial in range(150):
        m = int(rng.integers(1, 5))
        a = np.round(0.1 + 2 * rng.random(m), 3)
        p = np.round(0.1 + rng.random(m), 3)
        w, c = 0.5 + rng.random(), 0.2 + 2 * rng.random()
        J = oracle.subproblem(a, p, kind, w, c, 1e-3)
        best_x = {}
        if J["jlo"] >= 0 and J["xlo"] > 0:
            best_x[J["jlo"]] = J["xlo"]
        if J["jhi"] >= 0 and J["xhi"] > 0:
            best_x[J["jhi"]] = best_x.get(J["jhi"], 0.0) + J["xhi"]
        want = _margin_numeric(a, p, kind, w, c, 1e-3, best_x)
        if math.isinf(want):
            assert math.isinf(J["marginx"]), (a, p, w, c, J)
        else:
            assert J["marginx"] == pytest.approx(want, abs=2e-6), (a, p, w, c, J, want)
            checked += 1
    assert checked > 100


def test_marginx_special_cases():
    # equal efficiencies a_j / p_j: the log optimum t = 0.5 can be bought on
    # resource 0 alone (x = 0.5) or on resource 1 alone (x = 0.25) at the
    # same cost: a tie between allocations
    J = oracle.subproblem(np.array([1.0, 2.0]), np.array([1.0, 2.0]), LOG, 0.501, 0.0, 1e-3)
    assert J["marginx"] == pytest.approx(0.0, abs=1e-12)
    # nothing to buy: the origin is the only allocation
    J = oracle.subproblem(np.array([0.0, 0.0]), np.array([1.0, 1.0]), LOG, 1.0, 0.0, 1e-3)
    assert math.isinf(J["marginx"])
    # one resource, interior log optimum: the other candidate is the origin,
    # so the margin is (v* - w log eps) / max(1, |v*|), v* from a 1-D search
    from scipy.optimize import minimize_scalar
    a, pr, w, eps = 2.0, 0.7, 1.3, 1e-3
    res = minimize_scalar(lambda x: -(w * math.log(a * x + eps) - pr * x), bounds=(0.0, 1.0),
                          method="bounded", options={"xatol": 1e-13})
    vstar = -res.fun
    J = oracle.subproblem(np.array([a]), np.array([pr]), LOG, w, 0.0, eps)
    assert J["marginx"] == pytest.approx((vstar - w * math.log(eps)) / max(1.0, abs(vstar)),
                                         abs=1e-7)
