/*
 * Drives every entry point of the FP64 oracle (oracle/oracle.c, compiled into
 * this file) on small seeded instances, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: each call's outputs must be finite, and the
 * sanitizers report any out-of-bounds access, use of freed memory, overflow or
 * other undefined behaviour.  Prints "ok" and exits 0 when all is well.
 */
#include "../oracle/oracle.c"

#include <stdio.h>
#include <stdlib.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static double urand(void)
{
    /* xorshift64*: uniform in [0, 1) */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (double)((rng_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int finite_all(const double *x, int64_t k)
{
    for (int64_t i = 0; i < k; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

/* One instance: n jobs, m resources, FP64 (tdt 1) or FP32 (tdt 0) data, a
 * third each log, capped-linear and alpha-fair jobs, some zero entries, one
 * zero row, and (with_demands) per-job demand vectors. */
static int run(int64_t n, int m, int tdt, int with_demands)
{
    const size_t es = tdt ? sizeof(double) : sizeof(float);
    void *T = malloc((size_t)n * m * es), *w = malloc((size_t)n * es), *c = malloc((size_t)n * es);
    uint8_t *kind = (uint8_t *)malloc((size_t)n);
    double *R = (double *)malloc(sizeof(double) * m), *p = (double *)malloc(sizeof(double) * m);
    double *r = (double *)malloc(sizeof(double) * m), *d = NULL;
    int32_t *jlo = (int32_t *)malloc(sizeof(int32_t) * n), *jhi = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *j1 = (int32_t *)malloc(sizeof(int32_t) * n), *j1b = (int32_t *)malloc(sizeof(int32_t) * n);
    double *xlo = (double *)malloc(sizeof(double) * n), *xhi = (double *)malloc(sizeof(double) * n);
    double *t = (double *)malloc(sizeof(double) * n), *v = (double *)malloc(sizeof(double) * n);
    double *mg = (double *)malloc(sizeof(double) * n);
    int ok = 1;
    for (int64_t i = 0; i < n; ++i) {
        for (int j = 0; j < m; ++j) {
            double a = urand() < 0.1 || i == 3 ? 0.0 : 0.1 + urand();
            if (tdt) ((double *)T)[i * m + j] = a;
            else ((float *)T)[i * m + j] = (float)a;
        }
        kind[i] = (uint8_t)(i % 3);
        double wi = 0.5 + 1.5 * urand();
        double ci = kind[i] == 2 ? 3.0 * urand() : 0.5 + 1.5 * urand();
        if (tdt) {
            ((double *)w)[i] = wi;
            ((double *)c)[i] = ci;
        } else {
            ((float *)w)[i] = (float)wi;
            ((float *)c)[i] = (float)ci;
        }
    }
    for (int j = 0; j < m; ++j) {
        R[j] = 0.3 * (double)n / m;
        p[j] = j == 0 ? 0.0 : 0.2 + urand(); /* one free resource */
    }
    if (with_demands) {
        d = (double *)malloc(sizeof(double) * (size_t)n * m);
        for (int64_t k = 0; k < n * m; ++k) d[k] = 0.5 + 1.5 * urand();
    }
    double g = 0.0, sv = 0.0;
    if (orc_dual_eval_d(n, m, tdt, T, w, c, kind, 1e-3, R, p, &g, r, &sv, jlo, jhi, xlo, xhi, t,
                        v, j1, mg, d, d ? m : 0) != 0)
        ok = 0;
    ok = ok && isfinite(g) && finite_all(r, m) && finite_all(xlo, n) && finite_all(xhi, n) &&
         finite_all(t, n) && finite_all(v, n);
    double du = 0.0;
    double U = orc_lower_bound(n, m, tdt, T, w, c, kind, 1e-3, R, r, jlo, jhi, xlo, xhi, &du);
    ok = ok && isfinite(U) && isfinite(du);
    orc_first_vertex(n, m, tdt, T, p, j1b);
    double p0[512];
    if (orc_init_prices_d(n, m, tdt, T, w, c, kind, 1e-3, R, p0, d, d ? m : 0) != 0) ok = 0;
    ok = ok && finite_all(p0, m);
    orc_solve_opts o = {1e-6, 8, 5, 0, 0, 0.0};
    orc_solve_info info;
    for (int j = 0; j < m; ++j) p0[j] = 1.0;
    orc_solve_d(n, m, tdt, T, w, c, kind, 1e-3, R, &o, p0, &info, d, d ? m : 0);
    ok = ok && finite_all(p0, m) && isfinite(info.g);
    o.method = 1;
    for (int j = 0; j < m; ++j) p0[j] = 1.0;
    orc_solve(n, m, tdt, T, w, c, kind, 1e-3, R, &o, p0, &info);
    ok = ok && finite_all(p0, m) && isfinite(info.g);
    free(T); free(w); free(c); free(kind); free(R); free(p); free(r); free(d);
    free(jlo); free(jhi); free(j1); free(j1b); free(xlo); free(xhi); free(t); free(v); free(mg);
    if (!ok) fprintf(stderr, "non-finite output: n=%lld m=%d tdt=%d demands=%d\n", (long long)n, m,
                     tdt, with_demands);
    return ok;
}

int main(void)
{
    int ok = 1;
    ok &= run(1, 1, 1, 0);
    ok &= run(257, 3, 1, 0);
    ok &= run(3001, 7, 0, 0);
    ok &= run(500, 16, 0, 1);
    ok &= run(300, 64, 1, 0);
    ok &= run(40, 256, 0, 0);
    if (!ok) return 1;
    printf("ok\n");
    return 0;
}
