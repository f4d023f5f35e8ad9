/*
 * FP64 CPU oracle for the price-discovery method of "Allocation of Fungible
 * Resources via a Fast, Scalable Price Discovery Method" (Agrawal, Boyd,
 * Narayanan, Kazhamiaka, Zaharia).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test-suite, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or constant with the HIP library.
 *
 * It is deliberately slow and plain:
 *   - per job, the subproblem (paper §3, eq. e-subprob; restated in §4 as
 *     eq. e-subproblem) is solved by enumerating every basic feasible
 *     solution with at most two nonzeros of (x, s) (§4.1): the m single
 *     resource segments from the origin (a_0, p_0) = (0, 0) and every pair of
 *     resources with a_k < a_l.  On each segment the cost is the affine
 *     function of eq. e-optcostij and the allocation is eq. e-xixj; the
 *     throughput maximising u(t) minus that cost on the segment is taken from
 *     eq. e-opt-t-log (log utility) or eq. e-opt-t-target (capped-linear
 *     utility).  The job optimum is the best segment: c(t) is the pointwise
 *     minimum of the segment costs, so maximising u - c equals maximising
 *     u - cost over every segment separately (§4.1, §4.2).  Cost is O(m^2)
 *     per job, the complexity stated in §4.2.
 *   - the dual function and its subgradient are eq. e-subprob summed with
 *     p^T R, and q = R - r (§3, eq. e-g-subgrad);
 *   - the feasible allocation scales every over-used column of X down to its
 *     limit, and its utility is the lower bound of the duality gap (§5);
 *   - the outer loop is Algorithm 2 (§5) with a projected L-BFGS price
 *     update (§5, "More efficient price updates") and a projected
 *     subgradient fallback (§5, "Standard subgradient price update").
 *
 * Utilities (§2.2): kind 0 = log, u(t) = w*log(t + eps); kind 1 = capped
 * linear, u(t) = w*min(t, c), which is the target-priority utility
 * w*min(t - c, 0) plus the constant w*c (same maximisers); kind 2 =
 * alpha-fair with exponent c (the family that holds the linear, log and
 * power utilities of §2.2), u(t) = w*(t + eps)^(1 - c)/(1 - c) for c != 1
 * (c = 0: linear, 0 < c < 1: power t^q with q = 1 - c, c > 1: -t^q with
 * q < 0 up to the factor 1/|1 - c|) and w*log(t + eps) for c = 1.
 *
 * Readings taken where the paper is silent:
 *   - equal efficiencies a_k = a_l give a zero-width segment and are skipped
 *     (that basic solution is the endpoint of a single-resource segment);
 *   - the target-priority table has no row for w > alpha with c < gamma: the
 *     utility is flat on the whole segment, so the cheapest point gamma wins;
 *   - a segment with alpha < 0 (never on the lower envelope for p >= 0) is
 *     maximised at delta for both utilities (increasing objective); a
 *     segment with alpha = 0 (a free resource, on the envelope) follows the
 *     closed forms: delta for log (w/alpha is infinite), and the
 *     target-priority table's w > alpha row, clip(c, gamma, delta), for the
 *     capped-linear utility;
 *   - ties between segments keep the first one in enumeration order
 *     (origin point, then single-resource segments, then pairs);
 *   - the L-BFGS details (projection, line search, memory) are not in the
 *     paper; see orc_solve.
 *
 * All sums over jobs are taken per fixed chunk of rows and then combined in
 * chunk order, so results do not depend on the number of OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LOG 0
#define ORC_CAPLIN 1
#define ORC_AFAIR 2
#define ORC_CHUNK 4096

/* ------------------------------------------------------------ utilities -- */

/* u_i(t) of §2.2 for the kinds used here. */
double orc_utility(int kind, double w, double c, double eps, double t)
{
    if (kind == ORC_LOG || (kind == ORC_AFAIR && c == 1.0))
        return w * log(t + eps);
    if (kind == ORC_AFAIR)
        return w * pow(t + eps, 1.0 - c) / (1.0 - c);
    return w * (t < c ? t : c);
}

/* Maximiser of u(t) - (alpha t + beta) over [gamma, delta] (§4.2).
 * Log: t = projection of (u')^{-1}(alpha) = w/alpha - eps onto the interval
 * (eq. e-opt-t-log).  Capped-linear: eq. e-opt-t-target with t_des = c.
 * Alpha-fair with exponent c > 0: the same projection of (u')^{-1}(alpha) =
 * (w/alpha)^(1/c) - eps (u' = w (t + eps)^(-c) is decreasing); c = 0
 * (linear): the right end if w > alpha, else the left end. */
double orc_segment_argmax(int kind, double w, double c, double eps, double alpha, double gamma,
                          double delta)
{
    if (alpha < 0.0)
        return delta;
    if (kind == ORC_LOG) {
        double t = w / alpha - eps;
        if (t < gamma) t = gamma;
        if (t > delta) t = delta;
        return t;
    }
    if (kind == ORC_AFAIR) {
        if (c == 0.0) return w > alpha ? delta : gamma;
        double t = pow(w / alpha, 1.0 / c) - eps;
        if (t < gamma) t = gamma;
        if (t > delta) t = delta;
        return t;
    }
    /* target-priority table */
    if (w <= alpha) return gamma;
    if (c >= gamma && c <= delta) return c;
    if (delta <= c) return delta;
    return gamma; /* w > alpha, c < gamma: utility flat on the segment */
}

/* c(t): the LP optimal value of §4 (cheapest way to reach throughput t with
 * x >= 0, 1^T x <= 1), as the pointwise minimum over the basic feasible
 * segments that contain t (§4.1).  +inf outside [0, max_j a_j]. */
double orc_cost(int m, const double *a, const double *p, double t)
{
    double best = (t == 0.0) ? 0.0 : INFINITY;
    for (int k = -1; k < m; ++k) {
        double ak = (k < 0) ? 0.0 : a[k];
        double pk = (k < 0) ? 0.0 : p[k];
        for (int l = 0; l < m; ++l) {
            double al = a[l], pl = p[l];
            if (!(ak < al)) continue;
            if (t < ak || t > al) continue;
            double xk = (al - t) / (al - ak); /* eq. e-xixj */
            double xl = (t - ak) / (al - ak);
            double cost = pk * xk + pl * xl;  /* eq. e-optcostij */
            if (cost < best) best = cost;
        }
    }
    return best;
}

/* Result of one job subproblem. jlo = -1 means the origin end (slack). */
typedef struct {
    double t, v;       /* optimal throughput and net utility u(t) - p^T x  */
    int32_t jlo, jhi;  /* support (resource indices), -1 = none            */
    double xlo, xhi;   /* allocation on jlo / jhi                           */
    int32_t j1;        /* argmax_j a_j/p_j (first lower-envelope vertex)   */
    double margin1;    /* (k(1) - k(2)) / k(1) over keys k_j = a_j / p_j   */
    double marginx;    /* (v(1) - v(2)) / max(1, |v(1)|), v(2) the best net
                          utility of a candidate whose allocation differs
                          from the optimum's (+inf if none): how far the job
                          is from a tie between allocations                  */
} orc_job;

/* A candidate allocation: shares x[s] on resources j[s] (j = -1: unused). */
typedef struct {
    int32_t j[2];
    double x[2];
} orc_alloc;

static double alloc_share(const orc_alloc *A, int j)
{
    double s = 0.0;
    for (int k = 0; k < 2; ++k)
        if (A->j[k] == j) s += A->x[k];
    return s;
}

/* Two allocations differ when some resource's share differs by more than
 * 1e-9 (shares lie in [0, 1]). */
static int alloc_differs(const orc_alloc *A, const orc_alloc *B)
{
    for (int k = 0; k < 2; ++k) {
        if (A->j[k] >= 0 && fabs(A->x[k] - alloc_share(B, A->j[k])) > 1e-9) return 1;
        if (B->j[k] >= 0 && fabs(B->x[k] - alloc_share(A, B->j[k])) > 1e-9) return 1;
    }
    return 0;
}

/* Algorithm 1 (§4.2) by enumeration of every basic feasible segment. */
void orc_subproblem(int m, const double *a, const double *p, int kind, double w, double c,
                    double eps, orc_job *out)
{
    /* origin point: x = 0, t = 0 */
    double best_v = orc_utility(kind, w, c, eps, 0.0);
    double best_t = 0.0, bxlo = 0.0, bxhi = 0.0;
    int bjlo = -1, bjhi = -1;
    /* the best allocation so far, and the best value among the candidates
     * whose allocation differs from it (a candidate with the same
     * allocation has the same value, so the second value only needs the
     * old best when a different candidate takes over) */
    orc_alloc best_x = {{-1, -1}, {0.0, 0.0}};
    double second_v = -INFINITY;

    for (int k = -1; k < m; ++k) {
        double ak = (k < 0) ? 0.0 : a[k];
        double pk = (k < 0) ? 0.0 : p[k];
        for (int l = 0; l < m; ++l) {
            double al = a[l], pl = p[l];
            if (!(ak < al)) continue;
            double alpha = (pl - pk) / (al - ak);
            double t = orc_segment_argmax(kind, w, c, eps, alpha, ak, al);
            double xk = (al - t) / (al - ak); /* eq. e-xixj */
            double xl = (t - ak) / (al - ak);
            double cost = pk * xk + pl * xl;  /* eq. e-optcostij */
            double v = orc_utility(kind, w, c, eps, t) - cost;
            orc_alloc cx = {{k >= 0 && xk != 0.0 ? k : -1, xl != 0.0 ? l : -1},
                            {k >= 0 ? xk : 0.0, xl}};
            const int differs = alloc_differs(&cx, &best_x);
            if (v > best_v) {
                if (differs && best_v > second_v) second_v = best_v;
                best_v = v;
                best_t = t;
                bjlo = k;
                bjhi = l;
                bxlo = (k < 0) ? 0.0 : xk;
                bxhi = xl;
                best_x = cx;
            } else if (differs && v > second_v) {
                second_v = v;
            }
        }
    }
    out->marginx = (second_v == -INFINITY)
                       ? INFINITY
                       : (best_v - second_v) / (fabs(best_v) > 1.0 ? fabs(best_v) : 1.0);
    out->t = best_t;
    out->v = best_v;
    out->jlo = bjlo;
    out->jhi = bjhi;
    out->xlo = bxlo;
    out->xhi = bxhi;

    /* best efficiency per price: key_j = a_j / p_j (p_j = 0 -> +inf when
     * a_j > 0; a_j = 0 -> 0, never chosen); ties -> lowest j */
    double keys[512];
    int j1 = -1;
    double k1 = 0.0;
    for (int j = 0; j < m; ++j) {
        keys[j] = (a[j] > 0.0) ? (p[j] > 0.0 ? a[j] / p[j] : INFINITY) : 0.0;
        if (keys[j] > k1) {
            k1 = keys[j];
            j1 = j;
        }
    }
    double k2 = 0.0;
    for (int j = 0; j < m; ++j)
        if (j != j1 && keys[j] > k2) k2 = keys[j];
    out->j1 = j1;
    if (j1 < 0)
        out->margin1 = 0.0;
    else if (isinf(k1))
        out->margin1 = isinf(k2) ? 0.0 : 1.0;
    else
        out->margin1 = (k1 - k2) / k1;
}

static inline double tval(const void *T, int tdt, int64_t idx)
{
    return tdt == 0 ? (double)((const float *)T)[idx] : ((const double *)T)[idx];
}

static inline double pval(const void *v, int tdt, int64_t idx)
{
    return tdt == 0 ? (double)((const float *)v)[idx] : ((const double *)v)[idx];
}

/* ------------------------------------------------------- dual function -- */

/* g(p) = p^T R + sum_i max_x (u_i(a_i^T x) - p^T x)   (§3, eq. e-subprob)
 * r = sum_i x_i, so the subgradient is q = R - r      (§3, eq. e-g-subgrad)
 * T is n x m row-major, float32 (tdt = 0) or float64 (tdt = 1); w, c have
 * T's type; kind is one byte per job.  Per-job outputs may be NULL.
 * Returns 0, or -1 on an allocation failure. */
/* With per-job demands (NULL = all 1; §7, "Extensions and variations"):
 * the usage limit becomes sum_i d_i * x_i <= R, job i sees the prices
 * d_i * p (elementwise), and r = sum_i d_i * x_i.  dcols = 1: one scalar
 * demand per job (d has n entries); dcols = m: a demand vector per job (d is
 * n x m, row-major). */
static inline double demand(const double *d, int dcols, int64_t i, int j)
{
    if (!d) return 1.0;
    return dcols == 1 ? d[i] : d[i * dcols + j];
}

int orc_dual_eval_m(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                    const uint8_t *kind, double eps, const double *R, const double *p, double *g,
                    double *r, double *sumv_out, int32_t *jlo, int32_t *jhi, double *xlo,
                    double *xhi, double *tout, double *vout, int32_t *j1, double *margin1,
                    double *marginx, const double *d, int dcols);

int orc_dual_eval_d(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                    const uint8_t *kind, double eps, const double *R, const double *p, double *g,
                    double *r, double *sumv_out, int32_t *jlo, int32_t *jhi, double *xlo,
                    double *xhi, double *tout, double *vout, int32_t *j1, double *margin1,
                    const double *d, int dcols)
{
    return orc_dual_eval_m(n, m, tdt, T, w, c, kind, eps, R, p, g, r, sumv_out, jlo, jhi, xlo,
                           xhi, tout, vout, j1, margin1, NULL, d, dcols);
}

/* orc_dual_eval_d, also returning each job's allocation margin (marginx). */
int orc_dual_eval_m(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                    const uint8_t *kind, double eps, const double *R, const double *p, double *g,
                    double *r, double *sumv_out, int32_t *jlo, int32_t *jhi, double *xlo,
                    double *xhi, double *tout, double *vout, int32_t *j1, double *margin1,
                    double *marginx, const double *d, int dcols)
{
    int64_t nchunks = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double *part = (double *)calloc((size_t)(nchunks > 0 ? nchunks : 1) * (size_t)(m + 1),
                                    sizeof(double));
    if (!part) return -1;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        double a[512], pd[512];
        double *acc = part + ch * (m + 1);
        int64_t lo = ch * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        for (int64_t i = lo; i < hi; ++i) {
            for (int j = 0; j < m; ++j) a[j] = tval(T, tdt, i * m + j);
            for (int j = 0; j < m; ++j) pd[j] = demand(d, dcols, i, j) * p[j];
            orc_job J;
            orc_subproblem(m, a, pd, kind[i], pval(w, tdt, i), pval(c, tdt, i), eps, &J);
            if (J.jlo >= 0) acc[J.jlo] += demand(d, dcols, i, J.jlo) * J.xlo;
            if (J.jhi >= 0) acc[J.jhi] += demand(d, dcols, i, J.jhi) * J.xhi;
            acc[m] += J.v;
            if (jlo) jlo[i] = J.jlo;
            if (jhi) jhi[i] = J.jhi;
            if (xlo) xlo[i] = J.xlo;
            if (xhi) xhi[i] = J.xhi;
            if (tout) tout[i] = J.t;
            if (vout) vout[i] = J.v;
            if (j1) j1[i] = J.j1;
            if (margin1) margin1[i] = J.margin1;
            if (marginx) marginx[i] = J.marginx;
        }
    }
    double sv = 0.0;
    for (int j = 0; j < m; ++j) r[j] = 0.0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        for (int j = 0; j < m; ++j) r[j] += part[ch * (m + 1) + j];
        sv += part[ch * (m + 1) + m];
    }
    free(part);
    double pr = 0.0;
    for (int j = 0; j < m; ++j) pr += p[j] * R[j];
    *g = pr + sv;
    if (sumv_out) *sumv_out = sv;
    return 0;
}

int orc_dual_eval(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                  const uint8_t *kind, double eps, const double *R, const double *p, double *g,
                  double *r, double *sumv_out, int32_t *jlo, int32_t *jhi, double *xlo,
                  double *xhi, double *tout, double *vout, int32_t *j1, double *margin1)
{
    return orc_dual_eval_d(n, m, tdt, T, w, c, kind, eps, R, p, g, r, sumv_out, jlo, jhi, xlo,
                           xhi, tout, vout, j1, margin1, NULL, 0);
}

/* Feasible allocation and its utility (§5): column j of X is scaled by
 * s_j = min(1, R_j / r_j) (s_j = 1 when r_j = 0), and the lower bound is
 * U(X~) = sum_i u_i(a_i^T x~_i).  Also returns sum_i [u_i(t_i) - u_i(t~_i)]
 * (the utility lost by scaling) when du is not NULL. */
double orc_lower_bound(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                       const uint8_t *kind, double eps, const double *R, const double *r,
                       const int32_t *jlo, const int32_t *jhi, const double *xlo,
                       const double *xhi, double *du)
{
    double s[512];
    for (int j = 0; j < m; ++j) s[j] = (r[j] > R[j]) ? R[j] / r[j] : 1.0;
    int64_t nchunks = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double *part = (double *)calloc((size_t)(nchunks > 0 ? nchunks : 1) * 2, sizeof(double));
    if (!part) return NAN;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        int64_t lo = ch * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        for (int64_t i = lo; i < hi; ++i) {
            double t = 0.0, tt = 0.0;
            if (jlo[i] >= 0) {
                double aij = tval(T, tdt, i * m + jlo[i]);
                t += aij * xlo[i];
                tt += s[jlo[i]] * aij * xlo[i];
            }
            if (jhi[i] >= 0) {
                double aij = tval(T, tdt, i * m + jhi[i]);
                t += aij * xhi[i];
                tt += s[jhi[i]] * aij * xhi[i];
            }
            double wi = pval(w, tdt, i), ci = pval(c, tdt, i);
            double ut = orc_utility(kind[i], wi, ci, eps, tt);
            part[2 * ch] += ut;
            part[2 * ch + 1] += orc_utility(kind[i], wi, ci, eps, t) - ut;
        }
    }
    double U = 0.0, d = 0.0;
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        U += part[2 * ch];
        d += part[2 * ch + 1];
    }
    free(part);
    if (du) *du = d;
    return U;
}

/* ------------------------------------------------------------ outer loop -- */

typedef struct {
    double tol_rel;   /* stop when (g - U)/max(|g|, |U|) <= tol_rel          */
    int32_t max_iter; /* price updates                                        */
    int32_t mem;      /* L-BFGS memory (the paper uses 10)                     */
    int32_t method;   /* 0 = L-BFGS, 1 = projected subgradient only            */
    int32_t verbose;
    double tol_abs;   /* > 0: also stop when g - U <= tol_abs (Algorithm 2's
                         test "g - U(X~) <= epsilon"; the paper suggests
                         epsilon = 1e-3 n)                                   */
} orc_solve_opts;

/* The stopping test of Algorithm 2 on a certified point. */
static int orc_met(double g, double U, double rel, const orc_solve_opts *o)
{
    return rel <= o->tol_rel || (o->tol_abs > 0.0 && g - U <= o->tol_abs);
}

typedef struct {
    int32_t iters, evals, status; /* status 0 = converged, 1 = max_iter        */
    double g, U, rel_gap;
} orc_solve_info;

/* Everything one evaluation of Algorithm 2 step 1 produces. */
typedef struct {
    double g, U, rel, f;
    double grad[512]; /* gradient of f = g/n, i.e. (R - r)/n */
} orc_eval;

static int orc_eval_at(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                       const uint8_t *kind, double eps, const double *R, const double *p,
                       int32_t *jlo, int32_t *jhi, double *xlo, double *xhi, const double *d,
                       int dcols, orc_eval *E)
{
    double r[512];
    if (orc_dual_eval_d(n, m, tdt, T, w, c, kind, eps, R, p, &E->g, r, NULL, jlo, jhi, xlo, xhi,
                        NULL, NULL, NULL, NULL, d, dcols))
        return -1;
    E->U = orc_lower_bound(n, m, tdt, T, w, c, kind, eps, R, r, jlo, jhi, xlo, xhi, NULL);
    double den = fabs(E->g) > fabs(E->U) ? fabs(E->g) : fabs(E->U);
    E->rel = (E->g - E->U) / (den > 0 ? den : 1.0);
    E->f = E->g / (double)n;
    for (int j = 0; j < m; ++j) E->grad[j] = (R[j] - r[j]) / (double)n;
    return 0;
}

static double dot(int m, const double *x, const double *y)
{
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += x[j] * y[j];
    return s;
}

static double amax(int m, const double *x)
{
    double s = 0.0;
    for (int j = 0; j < m; ++j) s = fabs(x[j]) > s ? fabs(x[j]) : s;
    return s;
}

/* Algorithm 2 (§5): evaluate the dual at p^k, recover a feasible allocation,
 * stop on the relative duality gap, else update the prices.
 *
 * Price update: projected L-BFGS on f(p) = g(p)/n over p >= 0.  Direction
 * d = -H grad f from the two-loop recursion over the last `mem` pairs with
 * H0 = (s^T y / y^T y) I, with components that would push a zero price
 * negative removed; trial p+ = max(p + lambda d, 0), lambda = 1 (first
 * iteration and after a reset: lambda = 0.1 |p|_inf / |grad|_inf), accepted
 * on the Armijo test f(p+) <= f(p) + 1e-4 grad^T (p+ - p), halving lambda up
 * to 20 times.  A pair is stored only if s^T y > 1e-12 |s| |y|.  When the
 * line search fails, one projected subgradient step
 * p+ = max(p - alpha_k q, 0) with alpha_k = a0 / sqrt(k) is taken and the
 * memory is cleared (the fallback of §5).  method = 1 uses only that step.
 * Every evaluated point is tested against the tolerance; p_inout receives
 * the iterate with the smallest relative gap (the certificate reported). */
int orc_solve_d(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                const uint8_t *kind, double eps, const double *R, const orc_solve_opts *opt,
                double *p_inout, orc_solve_info *info, const double *dem, int dcols)
{
    if (m > 512 || n < 1) return -2;
    int M = opt->mem > 0 ? opt->mem : 10;
    if (M > 64) M = 64;
    int32_t *jlo = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *jhi = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    double *xlo = (double *)malloc(sizeof(double) * (size_t)n);
    double *xhi = (double *)malloc(sizeof(double) * (size_t)n);
    double *S = (double *)calloc((size_t)M * (size_t)m, sizeof(double));
    double *Y = (double *)calloc((size_t)M * (size_t)m, sizeof(double));
    double *rho = (double *)calloc((size_t)M, sizeof(double));
    orc_eval *E = (orc_eval *)malloc(sizeof(orc_eval));
    orc_eval *E2 = (orc_eval *)malloc(sizeof(orc_eval));
    int rc = 0;
    if (!jlo || !jhi || !xlo || !xhi || !S || !Y || !rho || !E || !E2) {
        rc = -1;
        goto done;
    }
    double p[512], pn[512], d[512], q[512], al[64];
    for (int j = 0; j < m; ++j) p[j] = p_inout[j] > 0 ? p_inout[j] : 0.0;
    int evals = 0, iters = 0, npairs = 0, head = 0, sg_k = 0;
    if (orc_eval_at(n, m, tdt, T, w, c, kind, eps, R, p, jlo, jhi, xlo, xhi, dem, dcols, E)) {
        rc = -1;
        goto done;
    }
    ++evals;
    int status = 1;
    double best_rel = E->rel, best_g = E->g, best_U = E->U, pbest[512];
    memcpy(pbest, p, sizeof(double) * m);
    for (; iters < opt->max_iter; ++iters) {
        if (E->rel < best_rel) {
            best_rel = E->rel;
            best_g = E->g;
            best_U = E->U;
            memcpy(pbest, p, sizeof(double) * m);
        }
        if (orc_met(E->g, E->U, E->rel, opt)) {
            status = 0;
            break;
        }
        int took = 0;
        if (opt->method == 0) {
            /* two-loop recursion */
            for (int j = 0; j < m; ++j) q[j] = E->grad[j];
            for (int h = 0; h < npairs; ++h) {
                int s = (head - 1 - h + M) % M;
                al[h] = rho[s] * dot(m, S + s * m, q);
                for (int j = 0; j < m; ++j) q[j] -= al[h] * Y[s * m + j];
            }
            double gam = 1.0;
            if (npairs > 0) {
                int s = (head - 1 + M) % M;
                gam = dot(m, S + s * m, Y + s * m) / dot(m, Y + s * m, Y + s * m);
            }
            for (int j = 0; j < m; ++j) q[j] *= gam;
            for (int h = npairs - 1; h >= 0; --h) {
                int s = (head - 1 - h + M) % M;
                double be = rho[s] * dot(m, Y + s * m, q);
                for (int j = 0; j < m; ++j) q[j] += S[s * m + j] * (al[h] - be);
            }
            for (int j = 0; j < m; ++j) {
                d[j] = -q[j];
                if (p[j] <= 0.0 && d[j] < 0.0) d[j] = 0.0;
            }
            if (dot(m, d, E->grad) >= 0.0) { /* not a descent direction: reset */
                npairs = 0;
                for (int j = 0; j < m; ++j) {
                    d[j] = -E->grad[j];
                    if (p[j] <= 0.0 && d[j] < 0.0) d[j] = 0.0;
                }
            }
            double dn = amax(m, d);
            if (dn == 0.0) break; /* stationary on the free coordinates */
            double lam = 1.0;
            if (npairs == 0) {
                double pi = amax(m, p);
                lam = 0.1 * (pi > 0 ? pi : 1.0) / dn;
            }
            for (int ls = 0; ls < 20; ++ls) {
                for (int j = 0; j < m; ++j) {
                    pn[j] = p[j] + lam * d[j];
                    if (pn[j] < 0.0) pn[j] = 0.0;
                    q[j] = pn[j] - p[j];
                }
                if (orc_eval_at(n, m, tdt, T, w, c, kind, eps, R, pn, jlo, jhi, xlo, xhi, dem, dcols, E2)) {
                    rc = -1;
                    goto done;
                }
                ++evals;
                if (orc_met(E2->g, E2->U, E2->rel, opt) ||
                    E2->f <= E->f + 1e-4 * dot(m, E->grad, q)) {
                    took = 1;
                    break;
                }
                lam *= 0.5;
            }
            if (took) {
                double yv[512];
                for (int j = 0; j < m; ++j) yv[j] = E2->grad[j] - E->grad[j];
                double sy = dot(m, q, yv);
                double ns = sqrt(dot(m, q, q)), ny = sqrt(dot(m, yv, yv));
                if (sy > 1e-12 * ns * ny) {
                    memcpy(S + head * m, q, sizeof(double) * m);
                    memcpy(Y + head * m, yv, sizeof(double) * m);
                    rho[head] = 1.0 / sy;
                    head = (head + 1) % M;
                    if (npairs < M) ++npairs;
                }
            } else {
                npairs = 0;
            }
        }
        if (!took) { /* projected subgradient step */
            ++sg_k;
            double gi = amax(m, E->grad), pi = amax(m, p);
            double a0 = (gi > 0) ? 0.1 * (pi > 0 ? pi : 1.0) / gi : 0.0;
            double step = a0 / sqrt((double)sg_k);
            for (int j = 0; j < m; ++j) {
                pn[j] = p[j] - step * E->grad[j];
                if (pn[j] < 0.0) pn[j] = 0.0;
            }
            if (orc_eval_at(n, m, tdt, T, w, c, kind, eps, R, pn, jlo, jhi, xlo, xhi, dem, dcols, E2)) {
                rc = -1;
                goto done;
            }
            ++evals;
        }
        memcpy(p, pn, sizeof(double) * m);
        orc_eval *tmp = E;
        E = E2;
        E2 = tmp;
    }
    if (E->rel < best_rel) {
        best_rel = E->rel;
        best_g = E->g;
        best_U = E->U;
        memcpy(pbest, p, sizeof(double) * m);
    }
    if (orc_met(best_g, best_U, best_rel, opt)) status = 0;
    for (int j = 0; j < m; ++j) p_inout[j] = pbest[j];
    info->iters = iters;
    info->evals = evals;
    info->status = status;
    info->g = best_g;
    info->U = best_U;
    info->rel_gap = best_rel;
done:
    free(jlo);
    free(jhi);
    free(xlo);
    free(xhi);
    free(S);
    free(Y);
    free(rho);
    free(E);
    free(E2);
    return rc;
}

int orc_solve(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
              const uint8_t *kind, double eps, const double *R, const orc_solve_opts *opt,
              double *p_inout, orc_solve_info *info)
{
    return orc_solve_d(n, m, tdt, T, w, c, kind, eps, R, opt, p_inout, info, NULL, 0);
}

/* ------------------------------------------------- initial prices -- */

/* Data-dependent starting prices (§5, "Initialization", eq. e-initialization):
 * every job gets the same share x = R/n of the limits, or R/(kappa n) when
 * kappa = 1^T R / n exceeds 1 (so that 1^T x = 1), and
 *   p1 = (1/n) sum_i u_i'(a_i^T x) a_i,
 * the gradient of U at R under that uniform allocation.  Derivatives:
 * log, w/(t + eps); alpha-fair, w (t + eps)^(-c); capped linear, w below
 * the cap and 0 at or above it (the right derivative, one supergradient at
 * the kink).
 * With per-job demands (d, dcols as in orc_dual_eval_d) each job's term is
 * u_i'(a_i^T x) a_ij / d_ij: what the job would pay per unit of resource j it
 * demands (the paper states no start for demands; this is the formula's
 * reading per unit of demand, and equals dividing w_i by a scalar d_i).
 * Sums run per fixed chunk of rows, then in chunk order.
 * Returns 0, or -1 on an allocation failure. */
int orc_init_prices_d(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                      const uint8_t *kind, double eps, const double *R, double *p,
                      const double *d, int dcols)
{
    double x[512];
    double kappa = 0.0;
    for (int j = 0; j < m; ++j) kappa += R[j] / (double)n;
    const double scale = kappa > 1.0 ? 1.0 / (kappa * (double)n) : 1.0 / (double)n;
    for (int j = 0; j < m; ++j) x[j] = R[j] * scale;
    int64_t nchunks = (n + ORC_CHUNK - 1) / ORC_CHUNK;
    double *part = (double *)calloc((size_t)(nchunks > 0 ? nchunks : 1) * (size_t)m,
                                    sizeof(double));
    if (!part) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ch = 0; ch < nchunks; ++ch) {
        double *acc = part + ch * m;
        int64_t lo = ch * ORC_CHUNK, hi = lo + ORC_CHUNK < n ? lo + ORC_CHUNK : n;
        for (int64_t i = lo; i < hi; ++i) {
            double t = 0.0;
            for (int j = 0; j < m; ++j) t += tval(T, tdt, i * m + j) * x[j];
            const double wi = pval(w, tdt, i);
            double du;
            if (kind[i] == ORC_LOG)
                du = wi / (t + eps);
            else if (kind[i] == ORC_AFAIR)
                du = wi * pow(t + eps, -pval(c, tdt, i));
            else
                du = t < pval(c, tdt, i) ? wi : 0.0;
            for (int j = 0; j < m; ++j)
                acc[j] += du * tval(T, tdt, i * m + j) / demand(d, dcols, i, j);
        }
    }
    for (int j = 0; j < m; ++j) p[j] = 0.0;
    for (int64_t ch = 0; ch < nchunks; ++ch)
        for (int j = 0; j < m; ++j) p[j] += part[ch * m + j];
    for (int j = 0; j < m; ++j) p[j] /= (double)n;
    free(part);
    return 0;
}

int orc_init_prices(int64_t n, int m, int tdt, const void *T, const void *w, const void *c,
                    const uint8_t *kind, double eps, const double *R, double *p)
{
    return orc_init_prices_d(n, m, tdt, T, w, c, kind, eps, R, p, NULL, 0);
}

/* First lower-envelope vertex of every job (§4.1: the segment from the origin
 * with the least cost per unit of throughput) decided in the element type of
 * T: the key a_ij * (1/p_j) is formed with 1/p_j rounded to that type
 * (+inf for p_j = 0) and the product rounded to it, and the largest key wins
 * with the lowest index on equal keys (a key of 0 or NaN, from a_ij = 0,
 * never wins; -1 when no key is positive).  This is the decision a
 * single-precision implementation takes for FP32 data: it equals the exact
 * argmax of a_ij / p_j except on near-ties. */
void orc_first_vertex(int64_t n, int m, int tdt, const void *T, const double *p, int32_t *j1)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int best_j = -1;
        if (tdt == 0) {
            const float *a = (const float *)T + i * m;
            float best = 0.0f;
            for (int j = 0; j < m; ++j) {
                const float pf = (float)p[j];
                const float ip = pf > 0.0f ? 1.0f / pf : INFINITY;
                const float key = a[j] * ip;
                if (key > best) {
                    best = key;
                    best_j = j;
                }
            }
        } else {
            const double *a = (const double *)T + i * m;
            double best = 0.0;
            for (int j = 0; j < m; ++j) {
                const double ip = p[j] > 0.0 ? 1.0 / p[j] : INFINITY;
                const double key = a[j] * ip;
                if (key > best) {
                    best = key;
                    best_j = j;
                }
            }
        }
        j1[i] = best_j;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
