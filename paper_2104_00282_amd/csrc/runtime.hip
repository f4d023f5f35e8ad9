// Host runtime of the C ABI declared in include/resalloc.h.
//
// A context owns a device, a stream and error text.  A problem borrows T,
// owns a packed copy of the per-job utility parameters, its block-partial
// scratch, a device price block with a pinned host twin, a pinned result
// buffer and (lazily) the per-job support scratch and a captured HIP graph of
// one full evaluation.
//
// One evaluation (Algorithm 2 step 1, §5) is: copy prices in, dual kernel
// (per-job subproblems and block partials), column reduction (r and the sum
// of net utilities), lower-bound kernel (feasible allocation by column
// scaling) and its reduction, copy results out.  The price update (step 3)
// is a projected L-BFGS on the host over m doubles.
#include "ra_kernels.h"
#include "resalloc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

struct ra_ctx {
    int dev = 0;
    int cus = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    int live_problems = 0;  // problems created on this context and not destroyed
    bool closed = false;    // ra_destroy called; freed when the last problem goes
    bool timing = false;    // bracket dual-kernel launches with events
    bool timed_pending = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};

struct ra_problem {
    ra_ctx* ctx = nullptr;
    int64_t n = 0;
    int m = 0;
    int dt = 0;  // 0 = FP32, 1 = FP64
    const void* T = nullptr;
    bool vec_ok = false;
    void* prm = nullptr;
    std::vector<double> R;
    double* Rdev = nullptr;
    double eps = 0.0;
    int grid = 1;
    int lgrid = 1;
    double* partial = nullptr;
    double* partial2 = nullptr;
    double* dout = nullptr;     // r[0..m), sum v, sum u(t~), sum u(t) - u(t~)
    void* pblock = nullptr;
    void* h_pblock = nullptr;
    double* h_out = nullptr;
    int16_t* jpair_ws = nullptr;
    void* tpair_ws = nullptr;
    void* xpair_ws = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace {

ra_status fail(ra_ctx* ctx, ra_status st, const char* fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define RA_HIP(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((ctx), e_ == hipErrorOutOfMemory ? RA_ENOMEM : RA_EDEVICE, "%s: %s", \
                        #call, hipGetErrorString(e_));                                      \
    } while (0)

size_t elt(int dt) { return dt == 0 ? 4 : 8; }
size_t price_block_bytes(int dt)
{
    return dt == 0 ? sizeof(ra::PriceBlock<float>) : sizeof(ra::PriceBlock<double>);
}

// Fill the pinned price block from host prices; returns p^T R with the
// rounded prices (the point the kernel actually evaluates).  The block asks
// for no lower bound of a previous point (see fill_prev).
double fill_prices(ra_problem* P, const double* p, std::vector<double>* prounded)
{
    double pR = 0.0;
    if (P->dt == 0) {
        auto* b = static_cast<ra::PriceBlock<float>*>(P->h_pblock);
        for (int j = 0; j < P->m; ++j) {
            const float pf = (float)p[j];
            b->p[j] = pf;
            b->invp[j] = pf > 0.f ? 1.0f / pf : INFINITY;
            pR += (double)pf * P->R[j];
            if (prounded) (*prounded)[j] = (double)pf;
        }
        b->has_prev = 0;
    } else {
        auto* b = static_cast<ra::PriceBlock<double>*>(P->h_pblock);
        for (int j = 0; j < P->m; ++j) {
            b->p[j] = p[j];
            b->invp[j] = p[j] > 0.0 ? 1.0 / p[j] : INFINITY;
            pR += p[j] * P->R[j];
            if (prounded) (*prounded)[j] = p[j];
        }
        b->has_prev = 0;
    }
    return pR;
}

// Ask the next pass for the lower bound of a previously evaluated point:
// its (already rounded) prices q and the column scales of its usage r (§5).
template <typename F>
void fill_prev_t(ra_problem* P, const std::vector<double>& q, const std::vector<double>& r)
{
    auto* b = static_cast<ra::PriceBlock<F>*>(P->h_pblock);
    for (int j = 0; j < P->m; ++j) {
        const F qf = (F)q[j];
        b->q[j] = qf;
        b->invq[j] = qf > F(0) ? F(1) / qf : F(INFINITY);
        const bool over = r[j] > P->R[j];
        b->s[j] = over ? (F)(P->R[j] / r[j]) : F(1);
        b->sc[j] = over ? (F)((r[j] - P->R[j]) / r[j]) : F(0);
    }
    b->has_prev = 1;
}

void fill_prev(ra_problem* P, const std::vector<double>& q, const std::vector<double>& r)
{
    if (P->dt == 0)
        fill_prev_t<float>(P, q, r);
    else
        fill_prev_t<double>(P, q, r);
}

ra_status ensure_support_ws(ra_problem* P)
{
    ra_ctx* ctx = P->ctx;
    if (!P->jpair_ws) RA_HIP(ctx, hipMalloc(&P->jpair_ws, (size_t)P->n * 4));
    if (!P->tpair_ws) RA_HIP(ctx, hipMalloc(&P->tpair_ws, (size_t)P->n * 2 * elt(P->dt)));
    return RA_OK;
}

// Queue one evaluation on the context stream (no synchronisation).
ra_status enqueue_eval(ra_problem* P, bool lb, int16_t* jpair_user, void* xpair_user,
                       int16_t* j1_user)
{
    ra_ctx* ctx = P->ctx;
    hipStream_t st = ctx->stream;
    RA_HIP(ctx, hipMemcpyAsync(P->pblock, P->h_pblock, price_block_bytes(P->dt),
                               hipMemcpyHostToDevice, st));
    int16_t* jp = jpair_user ? jpair_user : (lb ? P->jpair_ws : nullptr);
    void* tp = lb ? P->tpair_ws : nullptr;
    if (ctx->timing) RA_HIP(ctx, hipEventRecord(ctx->ev0, st));
    RA_HIP(ctx, ra::launch_dual(P->dt, P->m, P->vec_ok, P->grid, st, P->T, P->prm, P->n,
                                P->pblock, P->eps, P->partial, jp, jpair_user ? xpair_user : nullptr,
                                tp, j1_user));
    if (ctx->timing) {
        RA_HIP(ctx, hipEventRecord(ctx->ev1, st));
        ctx->timed_pending = true;
    }
    RA_HIP(ctx, ra::launch_reduce_cols(st, P->partial, P->grid, ra::partial_cols(P->m), P->dout));
    if (lb) {
        RA_HIP(ctx, ra::launch_lower(P->dt, P->lgrid, st, jp, tp, P->prm, P->n, P->m, P->Rdev,
                                     P->dout, P->eps, P->partial2));
        RA_HIP(ctx, ra::launch_reduce_cols(st, P->partial2, P->lgrid, 2, P->dout + P->m + 1));
    }
    RA_HIP(ctx, hipMemcpyAsync(P->h_out, P->dout, sizeof(double) * (P->m + 3),
                               hipMemcpyDeviceToHost, st));
    return RA_OK;
}

// Add the last timed launch to the totals (after the stream has synchronised).
ra_status collect_timing(ra_ctx* ctx)
{
    if (!ctx->timed_pending) return RA_OK;
    float ms = 0.f;
    RA_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->timed_ms += ms;
    ctx->timed_launches += 1;
    ctx->timed_pending = false;
    return RA_OK;
}

struct Eval {
    double g = 0, f = 0;
    std::vector<double> grad;  // gradient of f = g / n
    std::vector<double> p;     // the (rounded) prices evaluated
    std::vector<double> r;     // usage r(p)
    double pR = 0;
    // certificate (§5): lower bound U(X~) of the column-scaled allocation,
    // gap = g - U(X~) and the relative gap; valid when certified
    bool certified = false;
    double U = 0, gap = 0, rel = INFINITY;
};

// Dual value, gradient and usage of the last pass from the pinned buffer.
void read_dual(const ra_problem* P, double pR, Eval& E)
{
    const int m = P->m;
    const double* o = P->h_out;
    E.pR = pR;
    E.g = pR + o[m];
    E.f = E.g / (double)P->n;
    E.grad.resize(m);
    E.r.assign(o, o + m);
    for (int j = 0; j < m; ++j) E.grad[j] = (P->R[j] - o[j]) / (double)P->n;
    E.certified = false;
}

// Certificate of E from the scaled-utility sums su (sum of u(t~)) and sdu
// (sum of u(t) - u(t~)) of its own allocation:
// gap = g - U(X~) = p^T (R - r) + sum_i [u(t_i) - u(t~_i)].
void certify(const ra_problem* P, double su, double sdu, Eval& E)
{
    (void)su;
    double pq = 0.0;
    for (int j = 0; j < P->m; ++j) pq += E.p[j] * (P->R[j] - E.r[j]);
    E.gap = pq + sdu;
    E.U = E.g - E.gap;
    const double den = std::max(std::fabs(E.g), std::fabs(E.U));
    E.rel = E.gap / (den > 0 ? den : 1.0);
    E.certified = true;
}

ra_status capture_graph(ra_problem* P)
{
    ra_ctx* ctx = P->ctx;
    if (P->gexec) return RA_OK;
    RA_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    ra_status st = enqueue_eval(P, false, nullptr, nullptr, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (st != RA_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(ctx, RA_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(ctx, RA_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    P->graph = g;
    return RA_OK;
}

// One pass at p: dual value, gradient and usage at p, and -- when prev is
// given -- the certificate of prev, computed in the same pass over T.
ra_status evaluate(ra_problem* P, const double* p, Eval* prev, bool use_graph, Eval& E)
{
    ra_ctx* ctx = P->ctx;
    E.p.resize(P->m);
    const double pR = fill_prices(P, p, &E.p);
    if (prev) fill_prev(P, prev->p, prev->r);
    if (use_graph && !ctx->timing) {
        ra_status st = capture_graph(P);
        if (st != RA_OK) return st;
        RA_HIP(ctx, hipGraphLaunch(P->gexec, ctx->stream));
    } else {
        ra_status st = enqueue_eval(P, false, nullptr, nullptr, nullptr);
        if (st != RA_OK) return st;
    }
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (collect_timing(ctx) != RA_OK) return RA_EDEVICE;
    read_dual(P, pR, E);
    if (!std::isfinite(E.g)) return fail(ctx, RA_ENUMERIC, "non-finite dual value");
    for (double q : E.grad)
        if (!std::isfinite(q)) return fail(ctx, RA_ENUMERIC, "non-finite gradient");
    if (prev) {
        certify(P, P->h_out[P->m + 1], P->h_out[P->m + 2], *prev);
        if (!std::isfinite(prev->gap)) return fail(ctx, RA_ENUMERIC, "non-finite duality gap");
    }
    return RA_OK;
}

double dotv(const std::vector<double>& a, const std::vector<double>& b)
{
    double s = 0.0;
    for (size_t j = 0; j < a.size(); ++j) s += a[j] * b[j];
    return s;
}

double inf_norm(const std::vector<double>& a)
{
    double s = 0.0;
    for (double v : a) s = std::max(s, std::fabs(v));
    return s;
}

}  // namespace

extern "C" {

const char* ra_status_string(ra_status s)
{
    switch (s) {
    case RA_OK: return "ok";
    case RA_EINVAL: return "invalid argument";
    case RA_ENOMEM: return "out of memory";
    case RA_EDEVICE: return "device error";
    case RA_ENUMERIC: return "non-finite result";
    case RA_ENOTCONV: return "not converged";
    case RA_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* ra_last_error(const ra_ctx* ctx) { return ctx ? ctx->err.c_str() : ""; }

ra_status ra_create(ra_ctx** out, int device_ordinal, void* hip_stream)
{
    if (!out) return RA_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) return RA_EDEVICE;
    if (device_ordinal < 0 || device_ordinal >= count) return RA_EINVAL;
    ra_ctx* c = new (std::nothrow) ra_ctx();
    if (!c) return RA_ENOMEM;
    c->dev = device_ordinal;
    if (hipSetDevice(c->dev) != hipSuccess) {
        delete c;
        return RA_EDEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->dev) != hipSuccess) {
        delete c;
        return RA_EDEVICE;
    }
    c->cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return RA_EDEVICE;
        }
        c->own_stream = true;
    }
    *out = c;
    return RA_OK;
}

static void free_ctx(ra_ctx* ctx)
{
    (void)hipSetDevice(ctx->dev);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

ra_status ra_destroy(ra_ctx* ctx)
{
    if (!ctx || ctx->closed) return RA_OK;
    ctx->closed = true;
    // problems keep using the context's stream: free it with the last one
    if (ctx->live_problems == 0) free_ctx(ctx);
    return RA_OK;
}

ra_status ra_problem_destroy(ra_problem* P)
{
    if (!P) return RA_OK;
    if (P->ctx) {
        (void)hipSetDevice(P->ctx->dev);
        (void)hipStreamSynchronize(P->ctx->stream);
    }
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    (void)hipFree(P->prm);
    (void)hipFree(P->Rdev);
    (void)hipFree(P->partial);
    (void)hipFree(P->partial2);
    (void)hipFree(P->dout);
    (void)hipFree(P->pblock);
    (void)hipFree(P->jpair_ws);
    (void)hipFree(P->tpair_ws);
    (void)hipFree(P->xpair_ws);
    if (P->h_pblock) (void)hipHostFree(P->h_pblock);
    if (P->h_out) (void)hipHostFree(P->h_out);
    ra_ctx* ctx = P->ctx;
    delete P;
    if (ctx && --ctx->live_problems == 0 && ctx->closed) free_ctx(ctx);
    return RA_OK;
}

ra_status ra_problem_create(ra_ctx* ctx, ra_problem** out, int64_t n, int32_t m, ra_dtype dt,
                            const void* T, const void* w, const void* c, const uint8_t* kind,
                            const double* R, double eps, int validate)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!out) return fail(ctx, RA_EINVAL, "out is NULL");
    if (n < 1) return fail(ctx, RA_EINVAL, "n = %lld must be >= 1", (long long)n);
    if (m < 1 || m > RA_MAX_RESOURCES)
        return fail(ctx, RA_EINVAL, "m = %d must be in [1, %d]", m, RA_MAX_RESOURCES);
    if (dt != RA_F32 && dt != RA_F64) return fail(ctx, RA_EINVAL, "unknown dtype %d", (int)dt);
    if (!T || !w || !R) return fail(ctx, RA_EINVAL, "T, w and R are required");
    if (kind && !c) return fail(ctx, RA_EINVAL, "c is required when kind is given");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(ctx, RA_EINVAL, "eps must be >= 0");
    if (n > (int64_t)1 << 40) return fail(ctx, RA_EINVAL, "n too large");
    for (int j = 0; j < m; ++j)
        if (!(R[j] > 0.0) || !std::isfinite(R[j]))
            return fail(ctx, RA_EINVAL, "R[%d] = %g must be positive and finite", j, R[j]);

    RA_HIP(ctx, hipSetDevice(ctx->dev));
    ra_problem* P = new (std::nothrow) ra_problem();
    if (!P) return fail(ctx, RA_ENOMEM, "host allocation failed");
    P->ctx = ctx;
    ++ctx->live_problems;
    P->n = n;
    P->m = m;
    P->dt = (int)dt;
    P->T = T;
    P->R.assign(R, R + m);
    P->eps = eps;
    P->vec_ok = (dt == RA_F32) && (reinterpret_cast<uintptr_t>(T) % 16 == 0);
    P->grid = ra::dual_grid(ctx->cus, m, P->dt, n, P->vec_ok);
    P->lgrid = ra::lower_grid(ctx->cus, n);

    auto cleanup = [&](ra_status st) {
        ra_problem_destroy(P);
        return st;
    };
    hipError_t e = hipSuccess;
#define RA_ALLOC(call)                                                                      \
    do {                                                                                    \
        e = (call);                                                                         \
        if (e != hipSuccess)                                                                \
            return cleanup(fail(ctx, e == hipErrorOutOfMemory ? RA_ENOMEM : RA_EDEVICE,     \
                                "%s: %s", #call, hipGetErrorString(e)));                    \
    } while (0)
    RA_ALLOC(hipMalloc(&P->prm, (size_t)n * 2 * elt(P->dt)));
    RA_ALLOC(hipMalloc(&P->Rdev, sizeof(double) * m));
    RA_ALLOC(hipMalloc(&P->partial, sizeof(double) * (size_t)P->grid * ra::partial_cols(m)));
    RA_ALLOC(hipMalloc(&P->partial2, sizeof(double) * (size_t)P->lgrid * 2));
    RA_ALLOC(hipMalloc(&P->dout, sizeof(double) * (m + 3)));
    RA_ALLOC(hipMalloc(&P->pblock, price_block_bytes(P->dt)));
    RA_ALLOC(hipHostMalloc(&P->h_pblock, price_block_bytes(P->dt), hipHostMallocDefault));
    RA_ALLOC(hipHostMalloc((void**)&P->h_out, sizeof(double) * (m + 3), hipHostMallocDefault));
    std::memset(P->h_pblock, 0, price_block_bytes(P->dt));
    RA_ALLOC(hipMemcpyAsync(P->Rdev, R, sizeof(double) * m, hipMemcpyHostToDevice, ctx->stream));

    int* dbad = nullptr;
    RA_ALLOC(hipMalloc(&dbad, sizeof(int)));
    int zero = 0, bad = 0;
    e = hipMemcpyAsync(dbad, &zero, sizeof(int), hipMemcpyHostToDevice, ctx->stream);
    if (e == hipSuccess) e = ra::launch_pack(P->dt, ctx->stream, w, c, kind, n, P->prm, dbad);
    if (e == hipSuccess && validate)
        e = ra::launch_validate_T(P->dt, ctx->stream, T, n * (int64_t)m, dbad);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(dbad);
    if (e != hipSuccess)
        return cleanup(fail(ctx, RA_EDEVICE, "packing inputs: %s", hipGetErrorString(e)));
    if (validate && bad) {
        return cleanup(fail(ctx, RA_EINVAL, "invalid input:%s%s%s%s",
                            (bad & 1) ? " w <= 0 or non-finite;" : "",
                            (bad & 2) ? " capped-linear c < 0 or non-finite;" : "",
                            (bad & 4) ? " unknown utility kind;" : "",
                            (bad & 8) ? " T negative or non-finite;" : ""));
    }
#undef RA_ALLOC
    *out = P;
    return RA_OK;
}

ra_status ra_dual_eval(ra_ctx* ctx, const ra_problem* prob, const double* p, double* g,
                       double* grad, double* lower_bound, int16_t* j_pair, void* x_pair,
                       int16_t* j1)
{
    if (!ctx) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!p || !g || !grad) return fail(ctx, RA_EINVAL, "p, g and grad are required");
    if (x_pair && !j_pair) return fail(ctx, RA_EINVAL, "x_pair needs j_pair");
    ra_problem* P = const_cast<ra_problem*>(prob);
    for (int j = 0; j < P->m; ++j)
        if (!(p[j] >= 0.0) || !std::isfinite(p[j]))
            return fail(ctx, RA_EINVAL, "p[%d] = %g must be >= 0 and finite", j, p[j]);
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    const bool lb = lower_bound != nullptr;
    if (lb && ensure_support_ws(P) != RA_OK) return RA_ENOMEM;
    Eval E;
    E.p.resize(P->m);
    const double pR = fill_prices(P, p, &E.p);
    ra_status st = enqueue_eval(P, lb, j_pair, x_pair, j1);
    if (st != RA_OK) return st;
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (collect_timing(ctx) != RA_OK) return RA_EDEVICE;
    read_dual(P, pR, E);
    if (!std::isfinite(E.g)) return fail(ctx, RA_ENUMERIC, "non-finite dual value");
    for (int j = 0; j < P->m; ++j)
        if (!std::isfinite(P->h_out[j])) return fail(ctx, RA_ENUMERIC, "non-finite usage");
    if (lb) {
        certify(P, P->h_out[P->m + 1], P->h_out[P->m + 2], E);
        if (!std::isfinite(E.U)) return fail(ctx, RA_ENUMERIC, "non-finite lower bound");
        *lower_bound = E.U;
    }
    *g = E.g;
    for (int j = 0; j < P->m; ++j) grad[j] = P->R[j] - P->h_out[j];
    return RA_OK;
}

void ra_solve_opts_default(ra_solve_opts* o)
{
    if (!o) return;
    o->tol_rel = 1e-6;
    o->max_iter = 500;
    o->lbfgs_mem = 10;
    o->method = 0;
    o->init = 0;
    o->use_graph = 1;
    o->verbose = 0;
    o->max_evals = 0;
}

ra_status ra_solve(ra_ctx* ctx, const ra_problem* prob, const ra_solve_opts* opts,
                   double* p_inout, ra_solve_info* info)
{
    if (!ctx) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!p_inout) return fail(ctx, RA_EINVAL, "p_inout is required");
    ra_solve_opts o;
    ra_solve_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.tol_rel >= 0.0) || o.max_iter < 0 || o.max_evals < 0 || o.lbfgs_mem < 1 ||
        o.lbfgs_mem > 64 ||
        (o.method != 0 && o.method != 1) || (o.init != 0 && o.init != 1))
        return fail(ctx, RA_EINVAL, "invalid solve options");
    ra_problem* P = const_cast<ra_problem*>(prob);
    const int m = P->m;
    std::vector<double> p(m, 1.0);
    if (o.init == 1) {
        for (int j = 0; j < m; ++j) {
            if (!std::isfinite(p_inout[j]) || p_inout[j] < 0.0)
                return fail(ctx, RA_EINVAL, "p_inout[%d] = %g must be >= 0 and finite", j, p_inout[j]);
            p[j] = p_inout[j];
        }
    }
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    const auto t0 = std::chrono::steady_clock::now();
    // the NULL stream cannot be captured
    const bool graph = o.use_graph && ctx->stream != nullptr;

    // cur: current iterate; trial: line-search point; pend: the last point
    // evaluated, whose certificate arrives with the next pass; best: the
    // certified point with the smallest relative gap
    Eval cur, trial, pend, best;
    int evals = 0, iters = 0, fallbacks = 0, sg_steps = 0;
    bool have_pend = false, done = false;
    auto budget_left = [&]() { return o.max_evals == 0 || evals < o.max_evals; };

    // One pass over T at x: evaluates x and certifies the pending point.
    auto pass = [&](const std::vector<double>& x, Eval& out) -> ra_status {
        ra_status s = evaluate(P, x.data(), have_pend ? &pend : nullptr, graph, out);
        if (s != RA_OK) return s;
        if (have_pend) {
            if (o.verbose)
                fprintf(stderr, "iteration %02d | utility=%.6f | dual_value=%.6f | gap=%.2e\n",
                        evals - 1, pend.U / (double)P->n, pend.g / (double)P->n,
                        pend.gap / (double)P->n);
            if (!best.certified || pend.rel < best.rel) best = pend;
            if (pend.rel <= o.tol_rel) done = true;
        }
        ++evals;
        pend = out;
        have_pend = true;
        return RA_OK;
    };

    ra_status st = pass(p, cur);
    if (st != RA_OK) return st;

    // L-BFGS memory: ring of (s, y, 1/s^T y)
    const int M = o.lbfgs_mem;
    std::vector<std::vector<double>> S(M, std::vector<double>(m)), Y(M, std::vector<double>(m));
    std::vector<double> rho(M), alpha(M), d(m), q(m), pn(m), step(m), yv(m);
    int npairs = 0, head = 0;
    bool out_of_budget = false;

    for (; iters < o.max_iter && !done; ++iters) {
        if (!budget_left()) break;
        bool took = false;
        if (o.method == 0) {
            // two-loop recursion: q = H grad
            q = cur.grad;
            for (int h = 0; h < npairs; ++h) {
                const int s = (head - 1 - h + M) % M;
                alpha[h] = rho[s] * dotv(S[s], q);
                for (int j = 0; j < m; ++j) q[j] -= alpha[h] * Y[s][j];
            }
            if (npairs > 0) {
                const int s = (head - 1 + M) % M;
                const double gam = dotv(S[s], Y[s]) / dotv(Y[s], Y[s]);
                for (int j = 0; j < m; ++j) q[j] *= gam;
            }
            for (int h = npairs - 1; h >= 0; --h) {
                const int s = (head - 1 - h + M) % M;
                const double b = rho[s] * dotv(Y[s], q);
                for (int j = 0; j < m; ++j) q[j] += S[s][j] * (alpha[h] - b);
            }
            // keep prices at zero that the direction would push negative
            for (int j = 0; j < m; ++j) d[j] = (cur.p[j] <= 0.0 && q[j] > 0.0) ? 0.0 : -q[j];
            if (dotv(d, cur.grad) >= 0.0) {
                npairs = 0;
                for (int j = 0; j < m; ++j)
                    d[j] = (cur.p[j] <= 0.0 && cur.grad[j] > 0.0) ? 0.0 : -cur.grad[j];
            }
            const double dn = inf_norm(d);
            if (dn == 0.0) break;
            double lam = 1.0;
            if (npairs == 0) {
                const double pi = inf_norm(cur.p);
                lam = 0.1 * (pi > 0.0 ? pi : 1.0) / dn;
            }
            for (int ls = 0; ls < 20; ++ls) {
                if (!budget_left()) {
                    out_of_budget = true;
                    break;
                }
                for (int j = 0; j < m; ++j) pn[j] = std::max(cur.p[j] + lam * d[j], 0.0);
                st = pass(pn, trial);
                if (st != RA_OK) return st;
                if (done) break;
                for (int j = 0; j < m; ++j) step[j] = trial.p[j] - cur.p[j];
                if (trial.f <= cur.f + 1e-4 * dotv(cur.grad, step)) {  // Armijo
                    took = true;
                    break;
                }
                lam *= 0.5;
            }
            if (done || out_of_budget) break;
            if (took) {
                for (int j = 0; j < m; ++j) yv[j] = trial.grad[j] - cur.grad[j];
                const double sy = dotv(step, yv);
                if (sy > 1e-12 * std::sqrt(dotv(step, step) * dotv(yv, yv))) {
                    S[head] = step;
                    Y[head] = yv;
                    rho[head] = 1.0 / sy;
                    head = (head + 1) % M;
                    npairs = std::min(npairs + 1, M);
                }
            } else {
                npairs = 0;
            }
        }
        if (!took) {
            // projected subgradient step p - a_k q with a_k = a0 / sqrt(k)
            if (!budget_left()) break;
            ++sg_steps;
            ++fallbacks;
            const double gi = inf_norm(cur.grad), pi = inf_norm(cur.p);
            const double a0 = gi > 0.0 ? 0.1 * (pi > 0.0 ? pi : 1.0) / gi : 0.0;
            const double ak = a0 / std::sqrt((double)sg_steps);
            for (int j = 0; j < m; ++j) pn[j] = std::max(cur.p[j] - ak * cur.grad[j], 0.0);
            st = pass(pn, trial);
            if (st != RA_OK) return st;
            if (done) break;
        }
        cur = trial;
    }
    // the last point evaluated still awaits its certificate
    if (!done && have_pend && budget_left()) {
        Eval tail;
        st = pass(pend.p, tail);
        if (st != RA_OK) return st;
    }
    const bool conv = best.certified && best.rel <= o.tol_rel;
    const Eval& ret = best.certified ? best : pend;
    if (o.verbose)
        fprintf(stderr, "%s in %03d iterations, with residual %g\n",
                conv ? "Converged" : "Stopped", iters, ret.gap / (double)P->n);
    for (int j = 0; j < m; ++j) p_inout[j] = ret.p[j];
    if (info) {
        info->iters = iters;
        info->dual_evals = evals;
        info->fell_back = fallbacks;
        info->converged = conv ? 1 : 0;
        info->g = ret.g;
        info->U_lb = ret.certified ? ret.U : NAN;
        info->rel_gap = ret.certified ? ret.rel : INFINITY;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return conv ? RA_OK : RA_ENOTCONV;
}

ra_status ra_get_allocation(ra_ctx* ctx, const ra_problem* prob, const double* p, void* X)
{
    if (!ctx) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!p || !X) return fail(ctx, RA_EINVAL, "p and X are required");
    ra_problem* P = const_cast<ra_problem*>(prob);
    for (int j = 0; j < P->m; ++j)
        if (!(p[j] >= 0.0) || !std::isfinite(p[j]))
            return fail(ctx, RA_EINVAL, "p[%d] = %g must be >= 0 and finite", j, p[j]);
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    if (ensure_support_ws(P) != RA_OK) return RA_ENOMEM;
    if (!P->xpair_ws) RA_HIP(ctx, hipMalloc(&P->xpair_ws, (size_t)P->n * 2 * elt(P->dt)));
    (void)fill_prices(P, p, nullptr);
    ra_status st = enqueue_eval(P, false, P->jpair_ws, P->xpair_ws, nullptr);
    if (st != RA_OK) return st;
    RA_HIP(ctx, ra::launch_materialize(P->dt, ctx->stream, P->jpair_ws, P->xpair_ws, P->n, P->m,
                                       P->Rdev, P->dout, X));
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return collect_timing(ctx);
}

ra_status ra_set_kernel_timing(ra_ctx* ctx, int enable)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    if (enable) {
        if (!ctx->ev0) RA_HIP(ctx, hipEventCreate(&ctx->ev0));
        if (!ctx->ev1) RA_HIP(ctx, hipEventCreate(&ctx->ev1));
        ctx->timed_ms = 0.0;
        ctx->timed_launches = 0;
        ctx->timed_pending = false;
    }
    ctx->timing = enable != 0;
    return RA_OK;
}

ra_status ra_get_kernel_timing(const ra_ctx* ctx, double* ms_total, int64_t* launches)
{
    if (!ctx) return RA_EINVAL;
    if (ms_total) *ms_total = ctx->timed_ms;
    if (launches) *launches = ctx->timed_launches;
    return RA_OK;
}

}  // extern "C"
