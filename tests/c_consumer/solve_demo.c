/*
 * A plain C consumer of the library's C ABI (no Python, no torch): reads a
 * problem from a binary file, evaluates the dual at p = 1 with every per-job
 * output, solves to a relative gap of 1e-4 and materialises the allocation,
 * and writes the results to a second binary file.
 *
 * Input:  int64 n, int32 m, float32 T[n*m], float32 w[n], float32 c[n],
 *         uint8 kind[n], float64 R[m], float64 eps
 * Output: float64 g, float64 grad[m], float64 lower_bound,
 *         int16 j_pair[2n], float32 x_pair[2n], int16 j1[n],
 *         float64 p[m], int32 iters, int32 dual_evals, float64 g_solve,
 *         float64 U_lb, float64 rel_gap, float32 X[n*m]
 * Exit status 0 on success; otherwise the failing call is printed.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "resalloc.h"

#define HIP_OK(call)                                                        \
    do {                                                                    \
        hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                             \
            fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));      \
            return 2;                                                       \
        }                                                                   \
    } while (0)

#define RA_OK_(ctx, call)                                                   \
    do {                                                                    \
        ra_status s_ = (call);                                              \
        if (s_ != RA_OK && s_ != RA_ENOTCONV) {                             \
            fprintf(stderr, "%s: %s (%s)\n", #call, ra_status_string(s_),   \
                    ra_last_error(ctx));                                    \
            return 3;                                                       \
        }                                                                   \
    } while (0)

static int read_all(FILE *f, void *p, size_t bytes)
{
    return fread(p, 1, bytes, f) == bytes ? 0 : -1;
}

int main(int argc, char **argv)
{
    if (argc != 3) {
        fprintf(stderr, "usage: %s input output\n", argv[0]);
        return 1;
    }
    FILE *in = fopen(argv[1], "rb");
    if (!in) return 1;
    int64_t n;
    int32_t m;
    if (read_all(in, &n, 8) || read_all(in, &m, 4) || n < 1 || m < 1 || m > RA_MAX_RESOURCES)
        return 1;
    const size_t nm = (size_t)n * (size_t)m;
    float *T = malloc(nm * 4), *w = malloc(n * 4), *c = malloc(n * 4), *X = malloc(nm * 4);
    float *xp = malloc(2 * n * 4);
    unsigned char *kind = malloc(n);
    short *jp = malloc(2 * n * 2), *j1 = malloc(n * 2);
    double *R = malloc(m * 8), *grad = malloc(m * 8), *p = malloc(m * 8), eps;
    if (!T || !w || !c || !X || !xp || !kind || !jp || !j1 || !R || !grad || !p) return 1;
    if (read_all(in, T, nm * 4) || read_all(in, w, n * 4) || read_all(in, c, n * 4) ||
        read_all(in, kind, n) || read_all(in, R, m * 8) || read_all(in, &eps, 8))
        return 1;
    fclose(in);

    void *dT, *dw, *dc, *dkind, *djp, *dxp, *dj1, *dX;
    HIP_OK(hipMalloc(&dT, nm * 4));
    HIP_OK(hipMalloc(&dw, n * 4));
    HIP_OK(hipMalloc(&dc, n * 4));
    HIP_OK(hipMalloc(&dkind, n));
    HIP_OK(hipMalloc(&djp, 2 * n * 2));
    HIP_OK(hipMalloc(&dxp, 2 * n * 4));
    HIP_OK(hipMalloc(&dj1, n * 2));
    HIP_OK(hipMalloc(&dX, nm * 4));
    HIP_OK(hipMemcpy(dT, T, nm * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dw, w, n * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dc, c, n * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(dkind, kind, n, hipMemcpyHostToDevice));

    ra_ctx *ctx = NULL;
    ra_status st = ra_create(&ctx, 0, NULL);
    if (st != RA_OK) {
        fprintf(stderr, "ra_create: %s\n", ra_status_string(st));
        return 3;
    }
    ra_problem *prob = NULL;
    RA_OK_(ctx, ra_problem_create(ctx, &prob, n, m, RA_F32, dT, dw, dc, dkind, R, eps, 1));

    for (int j = 0; j < m; ++j) p[j] = 1.0;
    double g = 0.0, lb = 0.0;
    RA_OK_(ctx, ra_dual_eval(ctx, prob, p, &g, grad, &lb, (int16_t *)djp, dxp, (int16_t *)dj1));
    HIP_OK(hipMemcpy(jp, djp, 2 * n * 2, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(xp, dxp, 2 * n * 4, hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(j1, dj1, n * 2, hipMemcpyDeviceToHost));

    ra_solve_opts o;
    ra_solve_opts_default(&o);
    o.tol_rel = 1e-4;
    ra_solve_info info;
    RA_OK_(ctx, ra_solve(ctx, prob, &o, p, &info));
    RA_OK_(ctx, ra_get_allocation(ctx, prob, p, dX));
    HIP_OK(hipMemcpy(X, dX, nm * 4, hipMemcpyDeviceToHost));

    FILE *out = fopen(argv[2], "wb");
    if (!out) return 1;
    fwrite(&g, 8, 1, out);
    fwrite(grad, 8, m, out);
    fwrite(&lb, 8, 1, out);
    fwrite(jp, 2, 2 * n, out);
    fwrite(xp, 4, 2 * n, out);
    fwrite(j1, 2, n, out);
    fwrite(p, 8, m, out);
    fwrite(&info.iters, 4, 1, out);
    fwrite(&info.dual_evals, 4, 1, out);
    fwrite(&info.g, 8, 1, out);
    fwrite(&info.U_lb, 8, 1, out);
    fwrite(&info.rel_gap, 8, 1, out);
    fwrite(X, 4, nm, out);
    fclose(out);

    RA_OK_(ctx, ra_problem_destroy(prob));
    RA_OK_(ctx, ra_destroy(ctx));
    hipFree(dT);
    hipFree(dw);
    hipFree(dc);
    hipFree(dkind);
    hipFree(djp);
    hipFree(dxp);
    hipFree(dj1);
    hipFree(dX);
    free(T); free(w); free(c); free(X); free(xp); free(kind); free(jp); free(j1);
    free(R); free(grad); free(p);
    return 0;
}
