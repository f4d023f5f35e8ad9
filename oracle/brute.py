"""Independent tiny-case routes that pin the C oracle (test infrastructure).

None of these follow the oracle's segment enumeration; each reaches the same
quantity another way:

* ``cost_lp``        -- c(t) as the LP of §4 solved by HiGHS (scipy);
* ``segment_scalar`` -- bounded scalar maximisation of u(t) - alpha t on a
                        segment (scipy ``minimize_scalar``);
* ``job_golden``     -- max_t u(t) - c_LP(t) by golden-section search (u - c is
                        concave, §4);
* ``job_grid``       -- brute force over a grid of the simplex x >= 0,
                        1^T x <= 1 (m <= 3);
* ``problem_grid``   -- brute force over allocations of a whole problem
                        (n <= 3, m <= 2);
* ``waterfill_m1``   -- the single-resource problem, solved by bisection on
                        the price (textbook water-filling);
* ``knapsack_identical`` -- identical jobs: the optimum gives every job the
                        same x, a fractional knapsack over x <= R/n, 1^T x <= 1;
* ``lp_linear``      -- linear utility: the whole problem as one LP (HiGHS).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy.optimize import linprog, minimize_scalar

LOG = 0
CAPLIN = 1
AFAIR = 2


def u(kind, w, c, eps, t):
    if kind == LOG or (kind == AFAIR and c == 1.0):
        return w * math.log(t + eps)
    if kind == AFAIR:
        return w * (t + eps) ** (1.0 - c) / (1.0 - c)
    return w * min(t, c)


def cost_lp(a, p, t):
    """min p^T x  s.t.  a^T x = t, 1^T x <= 1, x >= 0   (+inf if infeasible)."""
    a = np.asarray(a, float)
    p = np.asarray(p, float)
    m = len(a)
    res = linprog(p, A_ub=np.ones((1, m)), b_ub=[1.0], A_eq=a[None, :], b_eq=[t],
                  bounds=[(0, None)] * m, method="highs",
                  options={"primal_feasibility_tolerance": 1e-10,
                           "dual_feasibility_tolerance": 1e-10})
    if res.status != 0:
        return math.inf
    return float(res.fun)


def segment_scalar(kind, w, c, eps, alpha, beta, gamma, delta):
    """argmax and max of u(t) - (alpha t + beta) on [gamma, delta], numerically."""
    f = lambda t: -(u(kind, w, c, eps, t) - (alpha * t + beta))
    if delta - gamma < 1e-15:
        return gamma, -f(gamma)
    res = minimize_scalar(f, bounds=(gamma, delta), method="bounded",
                          options={"xatol": 1e-12})
    cands = [gamma, delta, float(res.x)]
    if kind == CAPLIN and gamma <= c <= delta:
        cands.append(c)
    best = max(cands, key=lambda t: -f(t))
    return best, -f(best)


def job_golden(a, p, kind, w, c, eps, iters=200):
    """max over t in [0, max a] of u(t) - c_LP(t) by golden-section search."""
    lo, hi = 0.0, float(np.max(a))
    phi = (math.sqrt(5) - 1) / 2
    F = lambda t: u(kind, w, c, eps, t) - cost_lp(a, p, t)
    x1 = hi - phi * (hi - lo)
    x2 = lo + phi * (hi - lo)
    f1, f2 = F(x1), F(x2)
    for _ in range(iters):
        if hi - lo < 1e-12:
            break
        if f1 < f2:
            lo, x1, f1 = x1, x2, f2
            x2 = lo + phi * (hi - lo)
            f2 = F(x2)
        else:
            hi, x2, f2 = x2, x1, f1
            x1 = hi - phi * (hi - lo)
            f1 = F(x1)
    cands = [0.0, float(np.max(a)), 0.5 * (lo + hi)]
    best = max(cands, key=F)
    return best, F(best)


def simplex_grid(m, h):
    """All x in h*Z^m with x >= 0, sum x <= 1."""
    k = int(round(1 / h))
    for idx in itertools.product(range(k + 1), repeat=m):
        if sum(idx) <= k:
            yield np.array(idx, float) * h


def job_grid(a, p, kind, w, c, eps, h=1e-3):
    best = -math.inf
    bx = None
    a = np.asarray(a, float)
    p = np.asarray(p, float)
    for x in simplex_grid(len(a), h):
        v = u(kind, w, c, eps, float(a @ x)) - float(p @ x)
        if v > best:
            best, bx = v, x
    return best, bx


def problem_grid(T, kind, w, c, eps, R, h=0.01, d=None):
    """max sum_i u_i(a_i^T x_i) over grid allocations with sum_i d_i * x_i <= R
    (d = 1 by default; n scalar demands, or n x m demand vectors)."""
    n, m = T.shape
    dd = np.ones((n, 1)) if d is None else np.asarray(d, float)
    if dd.ndim == 1:
        dd = dd[:, None]
    pts = list(simplex_grid(m, h))
    best = -math.inf
    for combo in itertools.product(range(len(pts)), repeat=n):
        X = np.array([pts[k] for k in combo])
        if np.any((dd * X).sum(0) > np.asarray(R) + 1e-12):
            continue
        val = sum(u(kind[i], w[i], c[i], eps, float(T[i] @ X[i])) for i in range(n))
        best = max(best, val)
    return best


def waterfill_m1(a, w, eps, R, iters=200):
    """m = 1, log utility: x_i(p) = clip(w_i/p - eps/a_i, 0, 1); find p with
    sum_i x_i(p) = R by bisection (0 when sum_i x_i(0+) <= R)."""
    a = np.asarray(a, float)
    w = np.asarray(w, float)
    x = lambda p: np.clip(w / p - eps / a, 0.0, 1.0)
    if np.sum(np.ones_like(a)) <= R:
        return 0.0, float(np.sum(w * np.log(a + eps)))
    lo, hi = 1e-12, 1e12
    for _ in range(iters):
        mid = math.sqrt(lo * hi)
        if np.sum(x(mid)) > R:
            lo = mid
        else:
            hi = mid
    p = math.sqrt(lo * hi)
    xs = x(p)
    return p, float(np.sum(w * np.log(a * xs + eps)))


def knapsack_identical(a, R, n):
    """Identical jobs: the largest common throughput tau = max a^T xbar subject
    to 0 <= xbar <= R/n, 1^T xbar <= 1 (greedy by a_j)."""
    a = np.asarray(a, float)
    cap = np.asarray(R, float) / n
    left = 1.0
    tau = 0.0
    for j in np.argsort(-a):
        take = min(cap[j], left)
        tau += a[j] * take
        left -= take
        if left <= 0:
            break
    return tau


def lp_linear(T, w, R):
    """Linear utility u_i(t) = w_i t: max sum_i w_i a_i^T x_i as an LP."""
    n, m = T.shape
    cobj = -(w[:, None] * T).ravel()
    A = []
    b = []
    for i in range(n):  # 1^T x_i <= 1
        row = np.zeros(n * m)
        row[i * m:(i + 1) * m] = 1
        A.append(row)
        b.append(1.0)
    for j in range(m):  # sum_i x_ij <= R_j
        row = np.zeros(n * m)
        row[j::m] = 1
        A.append(row)
        b.append(R[j])
    res = linprog(cobj, A_ub=np.array(A), b_ub=np.array(b), bounds=[(0, None)] * (n * m),
                  method="highs")
    assert res.status == 0
    return -float(res.fun)


def problem_slsqp_log(T, w, eps, R, d=None, starts=4, seed=0):
    """Log utilities: max sum_i w_i log(a_i^T x_i + eps) subject to x >= 0,
    1^T x_i <= 1 and sum_i d_i * x_i <= R (scalar or vector demands), by
    scipy's SLSQP from a few feasible starts (a smooth concave program, so
    every start reaches the same optimum up to the solver's tolerance)."""
    from scipy.optimize import minimize
    n, m = T.shape
    dd = np.ones((n, m)) if d is None else np.broadcast_to(
        np.asarray(d, float).reshape(n, -1), (n, m))
    R = np.asarray(R, float)
    f = lambda z: -float(np.sum(w * np.log((T * z.reshape(n, m)).sum(1) + eps)))
    def grad(z):
        X = z.reshape(n, m)
        t = (T * X).sum(1) + eps
        return -(w[:, None] * T / t[:, None]).ravel()
    cons = [{"type": "ineq", "fun": lambda z: 1.0 - z.reshape(n, m).sum(1)},
            {"type": "ineq", "fun": lambda z: R - (dd * z.reshape(n, m)).sum(0)}]
    rng = np.random.default_rng(seed)
    best = -math.inf
    for _ in range(starts):
        x0 = rng.random((n, m))
        x0 /= x0.sum(1, keepdims=True)
        x0 *= min(1.0, float(np.min(R / (dd * x0).sum(0)))) * 0.5
        res = minimize(f, x0.ravel(), jac=grad, bounds=[(0.0, 1.0)] * (n * m),
                       constraints=cons, method="SLSQP",
                       options={"ftol": 1e-14, "maxiter": 2000})
        X = res.x.reshape(n, m)
        if np.all(X >= -1e-9) and np.all(X.sum(1) <= 1 + 1e-7) and \
                np.all((dd * X).sum(0) <= R + 1e-7):
            best = max(best, -res.fun)
    return best
