/*
 * resalloc.h -- C ABI of the MI355X (gfx950) price-discovery library.
 *
 * The library solves the fungible resource allocation problem of Agrawal,
 * Boyd, Narayanan, Kazhamiaka and Zaharia, "Allocation of Fungible Resources
 * via a Fast, Scalable Price Discovery Method" (§2.4, eq. e-res-alloc):
 *
 *     maximise   sum_i u_i(t_i)
 *     subject to x_i >= 0,  1^T x_i <= 1,  t_i = a_i^T x_i,   i = 1..n
 *                sum_i x_i <= R
 *
 * by price discovery (§5, Algorithm 2): for prices p >= 0 it evaluates the
 * dual function g(p) = p^T R + sum_i max_x (u_i(a_i^T x) - p^T x) (§3,
 * eq. e-subprob) and its subgradient q = R - r, r = sum_i x_i (§3,
 * eq. e-g-subgrad), recovers a feasible allocation by scaling over-used
 * columns (§5), and updates p with projected L-BFGS (§5).
 *
 * Conventions for every call:
 *   - every function returns ra_status; nothing aborts or throws;
 *   - "device" pointers are HIP device memory on the context's device (for
 *     example torch tensor data pointers); "host" pointers are ordinary
 *     host memory;
 *   - inputs are BORROWED: the caller keeps them alive and unchanged until
 *     the object that uses them is destroyed; outputs are caller-allocated;
 *     scratch space is owned by the context or the problem;
 *   - calls are ordered on the context's stream and are synchronous: results
 *     are valid when the call returns;
 *   - one context per host thread; a context is not thread-safe;
 *   - on error, outputs are left untouched and ra_last_error(ctx) describes
 *     the failure; RA_EINVAL is returned before any device work is queued.
 *
 * Utility functions (§2.2), one per job:
 *   RA_UTIL_LOG     u(t) = w * log(t + eps)                    (w > 0)
 *   RA_UTIL_CAPLIN  u(t) = w * min(t, c)   (capped linear; the target-priority
 *                   utility w*min(t - c, 0) of §2.2 shifted by w*c; c >= 0)
 *   RA_UTIL_ALPHA_FAIR  u(t) = w * (t + eps)^(1 - a) / (1 - a) with exponent
 *                   a = c >= 0 (the alpha-fair family of §2.2: a = 0 linear,
 *                   0 < a < 1 power t^q, a > 1 -t^q with q < 0 up to a positive
 *                   factor; a = 1 is taken as RA_UTIL_LOG). With a > 1 and
 *                   eps = 0 every optimum must have t > 0.
 */
#ifndef RESALLOC_H
#define RESALLOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RA_OK = 0,
    RA_EINVAL = 1,       /* invalid argument (checked before any device work)   */
    RA_ENOMEM = 2,       /* device or pinned host allocation failed             */
    RA_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed          */
    RA_ENUMERIC = 4,     /* non-finite dual value or gradient                   */
    RA_ENOTCONV = 5,     /* solver stopped at max_iter above the tolerance      */
    RA_EUNSUPPORTED = 6  /* valid request the library does not implement       */
} ra_status;

typedef enum { RA_F32 = 0, RA_F64 = 1 } ra_dtype;

typedef enum { RA_UTIL_LOG = 0, RA_UTIL_CAPLIN = 1, RA_UTIL_ALPHA_FAIR = 2 } ra_util_kind;

typedef struct ra_ctx ra_ctx;         /* device, stream, scratch, pinned staging   */
typedef struct ra_problem ra_problem; /* borrowed T + packed per-job utilities      */
typedef struct ra_mlp ra_mlp;         /* warm-start network and its training state */

/* Largest number of resources a problem may have. */
#define RA_MAX_RESOURCES 256

/* Create a context on HIP device `device_ordinal`. `hip_stream` is a
 * hipStream_t to order work on, or NULL for a context-owned stream (default
 * priority). Errors: RA_EINVAL (bad ordinal, out NULL), RA_EDEVICE, RA_ENOMEM. */
ra_status ra_create(ra_ctx **out, int device_ordinal, void *hip_stream);

/* Destroy a context (waits for its stream). NULL is accepted. Problems
 * created on it stay usable until they are destroyed; the context's stream
 * and memory are released with the last of them. */
ra_status ra_destroy(ra_ctx *ctx);

/* Static string naming a status code. */
const char *ra_status_string(ra_status s);

/* Human-readable detail of the last failure on `ctx` ("" if none). */
const char *ra_last_error(const ra_ctx *ctx);

/* Describe a problem instance (§2.4, eq. e-res-alloc).
 *   n, m      jobs and resources: n >= 1, 1 <= m <= RA_MAX_RESOURCES
 *   dt        element type of T, w and c (RA_F32 or RA_F64)
 *   T         device, n x m row-major efficiency matrix; row i is the job's
 *             efficiency vector a_i of §2.1 (entries >= 0, finite)
 *   w, c      device, n values each: utility weight (> 0) and, for capped
 *             linear jobs, the cap c (>= 0), for alpha-fair jobs the exponent
 *             (>= 0); ignored for log jobs
 *   kind      device, n bytes of ra_util_kind, or NULL for all RA_UTIL_LOG
 *   R         host, m resource limits R_j (> 0, finite); copied
 *   eps       log offset (>= 0; eps = 0 requires every optimum t_i > 0)
 *   validate  1: check T, w, c and kind on the device (one pass) and return
 *             RA_EINVAL on a bad value; 0: trust the caller
 * T stays borrowed. w, c and kind are read once, here, into a problem-owned
 * packed copy (8 bytes per job in FP32, 16 in FP64). */
ra_status ra_problem_create(ra_ctx *ctx, ra_problem **out, int64_t n, int32_t m, ra_dtype dt,
                            const void *T, const void *w, const void *c, const uint8_t *kind,
                            const double *R, double eps, int validate);

/* Release a problem and its packed copy. NULL is accepted. */
ra_status ra_problem_destroy(ra_problem *prob);

/* One evaluation of the dual function at prices p (§3, eq. e-subprob and
 * eq. e-g-subgrad; per job, Algorithm 1 of §4.2).
 *   p            host, m prices (>= 0, finite); the kernel evaluates at p
 *                rounded to the problem's element type
 *   g            host, 1: g(p) = p^T R + sum_i v_i (v_i = the job's net utility)
 *   grad         host, m: q = R - r (a subgradient; the gradient where g is
 *                differentiable)
 *   lower_bound  host, 1 or NULL: utility U(X~) of the feasible allocation
 *                obtained by scaling each over-used column j of X by R_j/r_j
 *                (§5); g(p) - U(X~) is the duality gap
 *   j_pair       device, n x 2 int16 or NULL: the job's support (j_lo, j_hi),
 *                -1 where unused; j_lo = -1 means the slack end of §4.1
 *   x_pair       device, n x 2 of dt or NULL: the allocation on (j_lo, j_hi)
 *                (eq. e-xixj); written only together with j_pair
 *   j1           device, n int16 or NULL: argmax_j a_ij / p_j, the first
 *                vertex of the job's cost curve, decided in the element type
 *                with the key a_ij * (1/p_j) (1/p_j rounded to dt, +inf for
 *                p_j = 0); lowest j on equal finite keys; among free
 *                resources (p_j = 0, infinite keys) the largest a_ij, then
 *                the lowest j; -1 when no key is positive (an all-zero row).  With demand vectors the prices
 *                are d_ij p_j and the FP32 kernels form the reciprocal with
 *                the hardware approximation (about 1 ulp)
 * Errors: RA_EINVAL, RA_EDEVICE, RA_ENUMERIC (non-finite g or grad). */
ra_status ra_dual_eval(ra_ctx *ctx, const ra_problem *prob, const double *p, double *g,
                       double *grad, double *lower_bound, int16_t *j_pair, void *x_pair,
                       int16_t *j1);

/* ra_dual_eval for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments and results as ra_dual_eval without the per-job outputs:
 *   p            host, m prices (>= 0, finite)
 *   g, grad      host, 1 and m: g(p) and R - r
 *   lower_bound  host, 1 or NULL: U(X~), here from a second pass over T that
 *                solves every job again at p and scales it by the column
 *                scales of r(p), instead of a per-job workspace
 * No device memory is allocated: the dual kernel's block partials and their
 * column sums live in a static device array of 2 MiB + 2 KiB that each GPU
 * the library runs on holds until the process ends; a launch uses at most
 * 2^18 / (m + 3) blocks so that its partials fit (the kernels stride over
 * the jobs), so every problem the library accepts fits.  Calls on one GPU
 * share that array: calls that overlap on one GPU (other threads, other
 * contexts) race and must be serialised by the caller.  Synchronous on the
 * context stream.
 * Errors: RA_EINVAL, RA_EDEVICE, RA_ENUMERIC, as ra_dual_eval. */
ra_status ra_dual_eval_noalloc(ra_ctx *ctx, const ra_problem *prob, const double *p, double *g,
                               double *grad, double *lower_bound);

/* Options of the price-discovery loop (§5, Algorithm 2). */
typedef struct {
    double tol_rel;          /* stop when (g - U(X~)) / max(|g|, |U(X~)|) <= tol_rel */
    int32_t max_iter;        /* price updates (Algorithm 2, K^max)                   */
    int32_t lbfgs_mem;       /* L-BFGS memory (the paper's default is 10)            */
    int32_t method;          /* 0 = projected L-BFGS, 1 = projected subgradient     */
    int32_t init;            /* 0 = p = 1, 1 = use p_inout as given,
                                2 = the paper's data-dependent prices (ra_init_prices;
                                one extra pass, included in the reported time)      */
    int32_t use_graph;       /* 1 = replay one captured HIP graph per evaluation
                                for the generic kernels; the vectorised FP32
                                kernels take the prices as a kernel argument and
                                are always launched directly                      */
    int32_t verbose;         /* 1 = one line per iteration on stderr                */
    int32_t max_evals;       /* > 0: stop after at most this many passes over T      */
    int32_t stall_evals;     /* > 0: stop when the best certified relative gap has
                                not improved by 0.1% within this many passes       */
    double init_step;        /* > 0: a step taken with an empty L-BFGS memory moves
                                the largest price by this fraction of max_j p_j;
                                0 = the default (0.1, or 0.005 from a learned start);
                                must be finite, 0 <= init_step <= 10               */
    double tol_abs;          /* > 0: also stop when g - U(X~) <= tol_abs (Algorithm 2's
                                absolute test; the paper suggests 1e-3 n)          */
    int32_t device_loop;     /* 1: run the price update itself on the device: after
                                each pass, the kernel that sums its columns also
                                takes the L-BFGS step (one wave, FP64) and writes
                                the next prices, and the host replays graphs of 6
                                passes until the loop publishes its outcome in
                                pinned memory.  Applies to problems on the
                                vectorised kernels (FP32 T, m in {4, 8, 16, 32,
                                64}, T and any demand vectors 16-byte aligned)
                                with lbfgs_mem <= 32, verbose = 0 and timing off;
                                otherwise the host loop runs.  Same iteration as
                                the host loop; its dot products are summed in
                                another order, so iterates agree to rounding.
                                Spare passes of the last replay (no-ops) may
                                still be queued on the context's stream when the
                                call returns.  ra_batch_solve and
                                ra_solve_learned ignore it.  0 or 1              */
    int32_t stall_restarts;  /* >= 0, with stall_evals > 0: the first this many
                                stalls restart the update from the best certified
                                point with an empty L-BFGS memory and the first
                                step of init_step (a new approach to the optimum,
                                which can certify a tighter gap) instead of
                                stopping; the next stall stops                    */
    int32_t warm_stall_restarts; /* ra_solve_learned only (others ignore it):
                                -1 = off; >= 0: the warm run restarts on its first
                                this many stalls, and if it stalls once more
                                without meeting the tolerance, a cold solve from
                                p = 1 with stall_restarts follows (another path
                                to the optimum, another chance of a tight
                                certificate); the result is the better certified
                                point of the two runs, and max_evals bounds
                                their passes together                            */
    int32_t warm_stall_evals; /* ra_solve_learned only: > 0: the warm run's stall
                                window instead of stall_evals (a short one ends a
                                warm path that stalls sooner, for the cold solve
                                that follows with warm_stall_restarts >= 0);
                                0 = stall_evals                                  */
} ra_solve_opts;

/* Outcome of a solve. */
typedef struct {
    int32_t iters;           /* price updates taken                                  */
    int32_t dual_evals;      /* points evaluated and taken into the iteration (line-
                                search trials included); a last pass whose only
                                use was to certify the previous point is not
                                counted                                           */
    int32_t fell_back;       /* projected-subgradient steps taken                     */
    int32_t converged;       /* 1 if rel_gap <= tol_rel                               */
    double g;                /* dual value at the returned prices (upper bound)      */
    double U_lb;             /* U(X~) at the returned prices (lower bound)           */
    double rel_gap;          /* (g - U_lb) / max(|g|, |U_lb|)                         */
    double seconds;          /* wall time of the call                                */
    int32_t restarted;       /* a learned warm start was followed by a solve from
                                p = 1: 1 = abandoned after fallback_window
                                certificates, 2 = it stalled (warm_stall_restarts);
                                0 otherwise                                       */
    int32_t warm_evals;      /* passes of the warm run when restarted != 0           */
} ra_solve_info;

/* Defaults: tol_rel = 1e-6, max_iter = 500, lbfgs_mem = 10, method = 0,
 * init = 0, use_graph = 1, verbose = 0, max_evals = 0 (no limit),
 * stall_evals = 0 (off), init_step = 0 (default step), tol_abs = 0 (off),
 * device_loop = 0, stall_restarts = 0, warm_stall_restarts = -1 (off),
 * warm_stall_evals = 0 (stall_evals). */
void ra_solve_opts_default(ra_solve_opts *opts);

/* Per-job demands (§7, "Extensions and variations"): the usage limit becomes
 * sum_i d_i x_i <= R, so job i sees the prices d_i p and adds d_i x_i to the
 * usage r (g, the gradient R - r, the certificate and the batched solver all
 * follow).  x_i stays the job's time fractions (ra_get_allocation, support
 * outputs).  d: device, n values of the problem's dtype, each > 0 and finite,
 * copied; NULL removes the demands (all 1).  Implemented by packing w_i / d_i
 * as the job's weight (every utility here is linear in w), so the warm-start
 * features and the data-dependent start see w_i / d_i.  Invalidates the
 * problem's captured evaluation graph.  On a bad value returns RA_EINVAL and
 * leaves the problem without demands.  RA_EINVAL also when the problem has
 * demand vectors (the two kinds exclude each other).
 * Errors: RA_EINVAL, RA_EDEVICE. */
ra_status ra_problem_set_demands(ra_ctx *ctx, ra_problem *prob, const void *d);

/* Per-job demand vectors (§7, "Extensions and variations": jobs that demand
 * different amounts of different resources): job i uses d_ij units of
 * resource j per unit of time on it, so the usage limit becomes
 * sum_i d_ij x_ij <= R_j, job i's subproblem (eq. e-subproblem) is solved at
 * the prices d_i * p (elementwise), and r_j = sum_i d_ij x_ij (g, the gradient
 * R - r, the certificate's column scaling and the data-dependent start, whose
 * job terms become u_i' a_ij / d_ij, all follow).  x stays the jobs' time
 * fractions.  D: device, n x m of the problem's dtype, row-major like T
 * (16-byte aligned for the vectorised FP32 kernels, else the generic kernel
 * runs), each entry > 0 and finite (checked in one pass); BORROWED: the
 * caller keeps it alive and unchanged until it is removed (D = NULL) or the
 * problem is destroyed.  Each evaluation then reads n m more values.  Not
 * with scalar demands (RA_EINVAL), nor in ra_batch_solve (RA_EUNSUPPORTED);
 * the learned start's features do not see D.  Invalidates the problem's
 * captured evaluation graph.  On a bad value returns RA_EINVAL and leaves the
 * previous demand vectors in place.  Errors: RA_EINVAL, RA_EDEVICE. */
ra_status ra_problem_set_demand_vectors(ra_ctx *ctx, ra_problem *prob, const void *D);

/* The paper's data-dependent starting prices (§5, "Initialization", eq.
 * e-initialization): every job gets the uniform share x = R/n of the limits
 * (R/(kappa n) when kappa = 1^T R / n > 1, so that 1^T x = 1), and
 * p_out = (1/n) sum_i u_i'(a_i^T x) a_i, the sensitivity of the total
 * utility to R under that allocation.  u' is w/(t + eps) for log jobs, and w
 * below the cap, 0 at or above it, for capped-linear jobs (one supergradient
 * at the kink).  One pass over T; x is rounded to the problem dtype.
 * p_out: host, m doubles.  Blocks until the prices are on the host.
 * Errors: RA_EINVAL, RA_EDEVICE, RA_ENUMERIC (non-finite result). */
ra_status ra_init_prices(ra_ctx *ctx, const ra_problem *prob, double *p_out);

/* Price discovery (§5, Algorithm 2). Every pass over T evaluates g and its
 * gradient at the new prices and, in the same pass, the lower bound U(X~) of
 * the previously evaluated prices, so a point's certificate (its duality
 * gap) is known one pass after the point itself; a final pass certifies the
 * last point when the evaluation budget allows.
 * p_inout: host, m doubles; read when opts->init == 1, and on return holds
 * the certified prices with the smallest relative gap (the reported
 * certificate; U_lb is NaN and rel_gap +inf if no point could be certified
 * within max_evals). info: host, may be NULL.
 * Returns RA_OK when the tolerance was met, RA_ENOTCONV when max_iter ended
 * the loop (p_inout and info are still filled), or an error. */
ra_status ra_solve(ra_ctx *ctx, const ra_problem *prob, const ra_solve_opts *opts,
                   double *p_inout, ra_solve_info *info);

/* Dense feasible allocation X~ at prices p (§5): device, n x m of the
 * problem's element type, row-major. X~ = X diag(min(1, R_j / r_j)) with X
 * the subproblem solutions at p (at most two nonzeros per row, §4.1). */
ra_status ra_get_allocation(ra_ctx *ctx, const ra_problem *prob, const double *p, void *X);

/* Batched price discovery: B problems of one context solved together.
 * Each problem runs its own price loop (as ra_solve, same options); every
 * round evaluates all problems still running in one persistent kernel launch
 * (problems laid end to end in tiles of consecutive jobs, each wavefront
 * streaming a contiguous share of the tiles, the shares balanced by the
 * measured cost per job of each m class).  Below 16 problems each round
 * covers all of them and is replayed from one captured HIP graph; from 16 on,
 * the problems form two groups of about equal work whose rounds alternate on
 * the context's stream, so that the host steps one group's price loops while
 * the other group's round runs (use_graph is then ignored).  The launch shape (the tile height of each m class, the
 * tile budget the kernel is compiled for, blocks per compute unit) is chosen
 * by an autotuner that times candidate rounds at the first prices of a new
 * batch signature (number of problems, MiB of T, m classes, kernel variant);
 * its choice is cached in the context, and in the text file named by the
 * environment variable RESALLOC_TUNE_CACHE when it is set, and
 * ra_batch_tuning returns the times of its candidates.  ra_batch_set_shape
 * fixes a shape instead.  Results do not depend on the shape beyond the
 * order of floating-point sums.
 *   B         number of problems (>= 1)
 *   probs     host, B problem handles created on ctx; each FP32 with m in
 *             {4, 8, 16, 32} and T 16-byte aligned, else RA_EUNSUPPORTED
 *   opts      shared options (init = 1 reads p_inout); NULL = defaults
 *   tol_each  host, B per-problem tolerances replacing opts->tol_rel, or NULL
 *   p_inout   host, sum of the problems' m doubles, problem b's prices at
 *             offset m_0 + ... + m_{b-1}; on return each problem's certified
 *             prices with the smallest relative gap
 *   infos     host, B results, or NULL (seconds = wall time of the batch)
 * Returns RA_OK when every problem met its tolerance, RA_ENOTCONV otherwise
 * (outputs filled), or an error. */
ra_status ra_batch_solve(ra_ctx *ctx, int32_t B, ra_problem *const *probs,
                         const ra_solve_opts *opts, const double *tol_each, double *p_inout,
                         ra_solve_info *infos);

/* Fix the launch shape of later ra_batch_solve calls on ctx (callers that
 * want the same shape, and so the same summation order, in every process):
 *   tile_floats    1024, 2048 or 4096: floats of T a wavefront holds per
 *                  tile (the register budget of the kernel variant); 0
 *                  returns to the autotuner (rows and blocks_per_cu ignored)
 *   rows           host, 4 tile heights for m = 4, 8, 16, 32: each 0 (no
 *                  problems of that class allowed) or a multiple of 64, at
 *                  most 512, with rows[c] * m <= tile_floats
 *   blocks_per_cu  0 (as many as fit) .. 8
 * A batch with a class whose height is 0 fails with RA_EINVAL.  Errors:
 * RA_EINVAL. */
ra_status ra_batch_set_shape(ra_ctx *ctx, int32_t tile_floats, const int32_t *rows,
                             int32_t blocks_per_cu);

/* The autotuner's record of its last tuning on ctx, as JSON text:
 * {"signature": ..., "candidates": [{"tile_floats", "m" (0 = the whole
 * batch), "rows", "bpc", "ms"}, ...], "chosen": {"tile_floats", "rows",
 * "bpc", "ms", "cost_ns_per_job"}}; "" before any tuning.  *len (if len is
 * not NULL) gets its length without the terminating zero; with buf not NULL
 * the text and a zero are copied to buf, which needs cap >= *len + 1 bytes
 * (else RA_EINVAL, nothing copied). */
ra_status ra_batch_tuning(const ra_ctx *ctx, char *buf, size_t cap, size_t *len);

/* ---- Learned warm start (not in the paper; the paper's own starting point
 * is p = 1 or a data-dependent heuristic, §5 "Initialization"). ----------
 * A multilayer perceptron maps per-problem features to log-prices:
 *   in_dim -> hidden (ReLU) -> hidden (ReLU) -> out_dim, FP32,
 * inputs standardised and outputs de-standardised with stored means and
 * standard deviations.  Parameters are one flat FP32 array in the order
 * W1 (hidden x in_dim, row-major), b1, W2 (hidden x hidden), b2,
 * W3 (out_dim x hidden), b3.  Training minimises the mean squared error of
 * the standardised outputs with Adam (beta1 0.9, beta2 0.999, eps 1e-8). */

/* Feature vector of a problem (FP32 problems with m <= 64), 8 m + 16 floats
 * written to feat (device): for resource j, at 8 j .. 8 j + 7: the 10/50/90 %
 * nearest-rank quantiles of column j of T over the log jobs, the same over
 * the capped-linear jobs (0 where a kind has no job), R_j / n, and the log of
 * the column mean; then 8-bin histograms of w on [0.5, 2] (bins of width
 * 0.1875, values outside clamped to the end bins) for the log jobs and for
 * the capped-linear jobs, as fractions of the sample.  All statistics are
 * taken over the rows floor(k n / S), k < S, S = min(n, 8192). */
ra_status ra_features(ra_ctx *ctx, const ra_problem *prob, float *feat);

/* Create a network (weights He-normal from `seed`, zero biases, identity
 * standardisation). Errors: RA_EINVAL for non-positive sizes. */
ra_status ra_mlp_create(ra_ctx *ctx, int32_t in_dim, int32_t hidden, int32_t out_dim,
                        uint64_t seed, ra_mlp **out);
ra_status ra_mlp_destroy(ra_mlp *mlp);
/* Number of parameters (host output). */
ra_status ra_mlp_num_params(const ra_mlp *mlp, int64_t *count);
/* Copy the flat parameter array to / from host memory (num_params floats). */
ra_status ra_mlp_get_params(ra_mlp *mlp, float *host);
ra_status ra_mlp_set_params(ra_mlp *mlp, const float *host);
/* Standardisation (host arrays): x_mean, x_std (in_dim), y_mean, y_std (out_dim);
 * standard deviations must be > 0. */
ra_status ra_mlp_set_normalization(ra_mlp *mlp, const float *x_mean, const float *x_std,
                                   const float *y_mean, const float *y_std);
/* Forward pass for `batch` feature rows X (device, batch x in_dim) into Y
 * (device, batch x out_dim, de-standardised log-prices). */
ra_status ra_mlp_forward(ra_ctx *ctx, ra_mlp *mlp, int32_t batch, const float *X, float *Y);
/* Loss and gradients at targets Ty (device, batch x out_dim, raw log-prices)
 * without changing the parameters; grad_host (num_params floats) may be NULL. */
ra_status ra_mlp_gradients(ra_ctx *ctx, ra_mlp *mlp, int32_t batch, const float *X,
                           const float *Ty, float *grad_host, double *loss);
/* One Adam step of learning rate lr on one minibatch; loss before the step. */
ra_status ra_mlp_train_step(ra_ctx *ctx, ra_mlp *mlp, int32_t batch, const float *X,
                            const float *Ty, float lr, double *loss);
/* Save / load the network (dimensions, standardisation, parameters) to a file. */
ra_status ra_mlp_save(const ra_mlp *mlp, const char *path);
ra_status ra_mlp_load(ra_ctx *ctx, const char *path, ra_mlp **out);

/* Price discovery from a learned starting point: features, network forward,
 * p0 = exp(predicted log-prices), then the loop of ra_solve, with its
 * empty-memory steps sized by opts->init_step (default 0.005: a prediction is
 * expected within a few percent).  If after `fallback_window` certificates
 * the certified relative gap has not fallen below that of the starting
 * point (or any value is non-finite), the warm
 * run is abandoned and the solve restarts from p = 1 (info->restarted = 1,
 * info->warm_evals = passes spent before the restart, included in
 * dual_evals and seconds).  With opts->warm_stall_restarts >= 0, a warm run
 * that stalls short of the tolerance is followed by a solve from p = 1 in the
 * same way (info->restarted = 2).  The network's out_dim must equal the
 * problem's m. */
ra_status ra_solve_learned(ra_ctx *ctx, const ra_problem *prob, ra_mlp *mlp,
                           const ra_solve_opts *opts, int32_t fallback_window, double *p_out,
                           ra_solve_info *info);

/* The starting prices ra_solve_learned would use: p_out[j] = exp(y_j), y the
 * network's de-standardised output on the problem's features (ra_features).
 * p_out: host, m doubles.  Same requirements as ra_solve_learned; blocks
 * until the prices are on the host (the network's forward writes them to
 * pinned host memory the network owns and raises a flag there, so calls
 * with one network must not overlap; ra_solve_learned uses the same path).
 * Errors: RA_EINVAL, RA_EUNSUPPORTED, RA_EDEVICE. */
ra_status ra_predict_prices(ra_ctx *ctx, const ra_problem *prob, ra_mlp *mlp, double *p_out);

/* Measurement aid: the mean time (ms) of one plain streaming read of `bytes`
 * bytes at buf (device, 16-byte aligned, bytes a multiple of 16), over `reps`
 * reads after 3 untimed ones, timed with HIP events on the context's stream.
 * Gives the attainable read bandwidth that the dual kernel's HBM roofline
 * fraction can be compared with.  Errors: RA_EINVAL, RA_EDEVICE. */
ra_status ra_stream_read_ms(ra_ctx *ctx, const void *buf, int64_t bytes, int32_t reps, double *ms);

/* Measurement aid for the mapping of the first-vertex scan (§4.1: the first
 * envelope vertex of job i is argmax_j a_ij / p_j) onto a wavefront: over
 * the rows of an n x 64 FP32 matrix T (device, row-major, 16-byte aligned,
 * n a positive multiple of 64), staged through LDS in 64-row tiles as the
 * dual kernel stages them, each job's vertex is found by lanes_per_job
 * lanes (1, 2, 4, 8 or 16) that scan contiguous parts of its row and join
 * them with a shuffle argmax (lower index on equal keys).  p: host, 64
 * prices > 0 (the keys use their FP32 reciprocals).  j1: device, n int16,
 * receives the vertices.  ms: mean time of one pass over `reps` passes after
 * 3 untimed ones, HIP events on the context's stream.
 * Errors: RA_EINVAL, RA_EDEVICE. */
ra_status ra_probe_first_vertex_ms(ra_ctx *ctx, const float *T, int64_t n, const double *p,
                                   int32_t lanes_per_job, int32_t reps, int16_t *j1,
                                   double *ms);

/* Kernel timing on the context's stream (for benchmarks and profiling).
 * enable = 1 brackets every launch of the dual kernel with a pair of HIP
 * events on the context's stream and accumulates the elapsed times; while it
 * is on, evaluations launch kernels directly instead of replaying a graph.
 * enable = 0 stops timing; the totals are kept until the next enable = 1. */
ra_status ra_set_kernel_timing(ra_ctx *ctx, int enable);

/* Totals of the timed dual-kernel launches: milliseconds and launch count
 * (host outputs, either may be NULL). */
ra_status ra_get_kernel_timing(const ra_ctx *ctx, double *ms_total, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* RESALLOC_H */
