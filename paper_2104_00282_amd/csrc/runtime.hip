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
#include "price_loop.hpp"
#include "ra_internal.hpp"
#include "ra_kernels.h"
#include "resalloc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <map>
#include <memory>
#include <new>
#include <cstddef>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// Device scratch of the allocation-free evaluation (ra_dual_eval_noalloc):
// the dual kernel's block partials, then the column sums they reduce to.
// Each GPU the library runs on holds its own copy until the process ends.
constexpr int NOALLOC_PARTIAL = 1 << 18;                  // doubles (2 MiB)
constexpr int NOALLOC_OUT = RA_MAX_RESOURCES + 3;         // one row of column sums
static __device__ __align__(256) double scratch[NOALLOC_PARTIAL + NOALLOC_OUT];

namespace ra {

// Wait for the completion flag of a signalled pass.  The stream is queried
// now and then, so that a failed or finished stream without the flag ends
// the wait with an error instead of spinning.
ra_status wait_flag(ra_ctx* ctx, unsigned* flag)
{
    for (uint64_t k = 1;; ++k) {
        if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == 1u) return RA_OK;
        if ((k & 4095) == 0) {
            const hipError_t e = hipStreamQuery(ctx->stream);
            if (e == hipSuccess) {
                if (__atomic_load_n(flag, __ATOMIC_ACQUIRE) == 1u) return RA_OK;
                return fail(ctx, RA_EDEVICE, "evaluation finished without its completion flag");
            }
            if (e != hipErrorNotReady)
                return fail(ctx, RA_EDEVICE, "evaluation failed: %s", hipGetErrorString(e));
        }
        __builtin_ia32_pause();
    }
}

}  // namespace ra

namespace {

using ra::fail;
using ra::wait_flag;

// The device address of `scratch` on each device, found once per device
// with that device current (the host-side name of the array is not a device
// address).
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double* scratch_ptr[MAX_DEVICES] = {};

hipError_t scratch_address(int dev, double** out)
{
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* a = nullptr;
        const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = static_cast<double*>(a);
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

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
void fill_prev_t(ra_problem* P, const double* q, const double* r)
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

// The same from plain arrays (m entries each).
void fill_prev_arrays(ra_problem* P, const double* q, const double* r)
{
    if (P->dt == 0)
        fill_prev_t<float>(P, q, r);
    else
        fill_prev_t<double>(P, q, r);
}

void fill_prev(ra_problem* P, const std::vector<double>& q, const std::vector<double>& r)
{
    fill_prev_arrays(P, q.data(), r.data());
}

// The vectorised dual kernels need T, and demand vectors when set, 16-byte
// aligned.
bool dual_vec(const ra_problem* P)
{
    return P->vec_ok && (!P->dvec || reinterpret_cast<uintptr_t>(P->dvec) % 16 == 0);
}

ra_status ensure_support_ws(ra_problem* P)
{
    ra_ctx* ctx = P->ctx;
    if (!P->jpair_ws) RA_HIP(ctx, hipMalloc(&P->jpair_ws, (size_t)P->n * 4));
    if (!P->tpair_ws) RA_HIP(ctx, hipMalloc(&P->tpair_ws, (size_t)P->n * 2 * elt(P->dt)));
    return RA_OK;
}

// Queue one evaluation on the context stream (no synchronisation).  With
// `signal` (solver passes: no per-job outputs, no separate lower bound) the
// reduction writes its results straight into P->h_out and raises P->h_flag;
// otherwise the results are copied to P->h_out and the caller synchronises.
ra_status enqueue_eval(ra_problem* P, bool lb, int16_t* jpair_user, void* xpair_user,
                       int16_t* j1_user, bool signal = false)
{
    ra_ctx* ctx = P->ctx;
    hipStream_t st = ctx->stream;
    // the vectorised kernels take their prices as a kernel argument
    if (!ra::dual_is_vec(P->dt, P->m, dual_vec(P)))
        RA_HIP(ctx, hipMemcpyAsync(P->pblock, P->h_pblock, price_block_bytes(P->dt),
                                   hipMemcpyHostToDevice, st));
    int16_t* jp = jpair_user ? jpair_user : (lb ? P->jpair_ws : nullptr);
    void* tp = lb ? P->tpair_ws : nullptr;
    if (ctx->timing) RA_HIP(ctx, hipEventRecord(ctx->ev0, st));
    RA_HIP(ctx, ra::launch_dual(P->dt, P->m, dual_vec(P), P->grid, st, P->T, P->prm, P->n,
                                P->pblock, P->h_pblock, P->eps, P->partial, jp,
                                jpair_user ? xpair_user : nullptr, tp, j1_user, P->dem, P->dvec));
    if (ctx->timing) {
        RA_HIP(ctx, hipEventRecord(ctx->ev1, st));
        ctx->timed_pending = true;
    }
    if (signal) {
        RA_HIP(ctx, ra::launch_reduce_cols(st, P->partial, P->grid, ra::partial_cols(P->m),
                                           P->h_out, P->ticket, P->h_flag));
        return RA_OK;
    }
    RA_HIP(ctx, ra::launch_reduce_cols(st, P->partial, P->grid, ra::partial_cols(P->m), P->dout));
    if (lb) {
        RA_HIP(ctx, ra::launch_lower(P->dt, P->lgrid, st, jp, tp, P->prm, P->n, P->m, P->Rdev,
                                     P->dout, P->eps, P->partial2, P->dem));
        RA_HIP(ctx, ra::launch_reduce_cols(st, P->partial2, P->lgrid, 2, P->dout + P->m + 1));
    }
    RA_HIP(ctx, hipMemcpyAsync(P->h_out, P->dout, sizeof(double) * (P->m + 3),
                               hipMemcpyDeviceToHost, st));
    return RA_OK;
}

// Add the last timed launch to the totals.
ra_status collect_timing(ra_ctx* ctx)
{
    if (!ctx->timed_pending) return RA_OK;
    RA_HIP(ctx, hipEventSynchronize(ctx->ev1));
    float ms = 0.f;
    RA_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    ctx->timed_ms += ms;
    ctx->timed_launches += 1;
    ctx->timed_pending = false;
    return RA_OK;
}

ra_status capture_graph(ra_problem* P)
{
    ra_ctx* ctx = P->ctx;
    if (P->gexec) return RA_OK;
    RA_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    ra_status st = enqueue_eval(P, false, nullptr, nullptr, nullptr, true);
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

// The paper's data-dependent starting prices (§5, eq. e-initialization) into
// p (host, m): the uniform share x = R/n (R/(kappa n) when kappa = 1^T R/n
// exceeds 1) goes to the device as the price block's p, one pass sums
// u_i'(a_i^T x) a_i, and the column sums are divided by n.
ra_status init_prices(ra_problem* P, double* p)
{
    ra_ctx* ctx = P->ctx;
    hipStream_t st = ctx->stream;
    const int m = P->m;
    const double n = (double)P->n;
    double kappa = 0.0;
    for (int j = 0; j < m; ++j) kappa += P->R[j] / n;
    const double scale = kappa > 1.0 ? 1.0 / (kappa * n) : 1.0 / n;
    std::vector<double> x(m);
    for (int j = 0; j < m; ++j) x[j] = P->R[j] * scale;
    (void)fill_prices(P, x.data(), nullptr);
    RA_HIP(ctx, hipMemcpyAsync(P->pblock, P->h_pblock, price_block_bytes(P->dt),
                               hipMemcpyHostToDevice, st));
    RA_HIP(ctx, ra::launch_init(P->dt, m, dual_vec(P), P->grid, st, P->T, P->prm, P->n,
                                P->pblock, P->eps, P->partial, P->dvec));
    RA_HIP(ctx, ra::launch_reduce_cols(st, P->partial, P->grid, m, P->dout));
    RA_HIP(ctx, hipMemcpyAsync(P->h_out, P->dout, sizeof(double) * m, hipMemcpyDeviceToHost, st));
    RA_HIP(ctx, hipStreamSynchronize(st));
    for (int j = 0; j < m; ++j) {
        p[j] = P->h_out[j] / n;
        if (!std::isfinite(p[j]) || p[j] < 0.0)
            return fail(ctx, RA_ENUMERIC, "initial price %d is %g", j, p[j]);
    }
    return RA_OK;
}

// One pass over T at p: dual value and usage at p (p_eval = p as rounded for
// the kernel) and, when prev is given, the utility lost by scaling prev's
// allocation (sdu), all from one launch of the dual kernel.
ra_status run_pass(ra_problem* P, const std::vector<double>& p, const ra::Point* prev,
                   bool use_graph, std::vector<double>& p_eval, double& g, std::vector<double>& r,
                   double& sdu)
{
    ra_ctx* ctx = P->ctx;
    p_eval.resize(P->m);
    const double pR = fill_prices(P, p.data(), &p_eval);
    if (prev) fill_prev(P, prev->p, prev->r);
    __atomic_store_n(P->h_flag, 0u, __ATOMIC_RELEASE);
    const bool vec = ra::dual_is_vec(P->dt, P->m, dual_vec(P));
    // a small problem on the generic kernels: one launch with the prices as
    // its argument, its sums written straight to the host
    if (!vec && !ctx->timing && P->n <= ra::SMALL_MAX_N && P->m <= ra::SMALL_MAX_M && !P->dvec) {
        RA_HIP(ctx, ra::launch_dual_small(P->dt, ctx->stream, P->T, P->prm, P->n, P->m,
                                          P->h_pblock, P->eps, P->dem, P->partial, P->ticket,
                                          P->h_out, P->h_flag));
    } else if (use_graph && !ctx->timing && !vec) {
        // a captured graph would keep the kernel arguments of its capture, so
        // the vectorised kernels (prices as an argument) are launched directly
        ra_status st = capture_graph(P);
        if (st != RA_OK) return st;
        RA_HIP(ctx, hipGraphLaunch(P->gexec, ctx->stream));
    } else {
        ra_status st = enqueue_eval(P, false, nullptr, nullptr, nullptr, true);
        if (st != RA_OK) return st;
    }
    ra_status ws = wait_flag(ctx, P->h_flag);
    if (ws != RA_OK) return ws;
    if (collect_timing(ctx) != RA_OK) return RA_EDEVICE;
    const double* o = P->h_out;
    g = pR + o[P->m];
    r.assign(o, o + P->m);
    sdu = o[P->m + 2];
    if (!std::isfinite(g)) return fail(ctx, RA_ENUMERIC, "non-finite dual value");
    for (double v : r)
        if (!std::isfinite(v)) return fail(ctx, RA_ENUMERIC, "non-finite usage");
    if (prev && !std::isfinite(sdu)) return fail(ctx, RA_ENUMERIC, "non-finite duality gap");
    return RA_OK;
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
    if (scratch_address(c->dev, &c->scratch) != hipSuccess) {
        delete c;
        return RA_EDEVICE;
    }
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
    (void)hipFree(ctx->feat_ws);
    ctx->batch_ws.reset();  // waits for its launches on the stream
    ctx->batch_ws2.reset();
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
    if (P->dl_gexec) (void)hipGraphExecDestroy(P->dl_gexec);
    if (P->dl_graph) (void)hipGraphDestroy(P->dl_graph);
    (void)hipFree(P->dloop);
    (void)hipFree(P->dprices);
    if (P->h_dl) (void)hipHostFree(P->h_dl);
    if (P->h_dlstage) (void)hipHostFree(P->h_dlstage);
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
    (void)hipFree(P->ticket);
    (void)hipFree(P->dem);
    (void)hipFree(P->w0);
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
    P->grid_cap = P->grid;
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
    RA_ALLOC(hipHostMalloc((void**)&P->h_out, sizeof(double) * (m + 4), hipHostMallocCoherent));
    P->h_flag = reinterpret_cast<unsigned*>(P->h_out + m + 3);
    *P->h_flag = 0u;
    RA_ALLOC(hipMalloc((void**)&P->ticket, sizeof(unsigned)));
    RA_ALLOC(hipMemsetAsync(P->ticket, 0, sizeof(unsigned), ctx->stream));
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
    P->alpha_fair = (bad & 16) != 0;
    bad &= ~16;
    if (validate && bad) {
        return cleanup(fail(ctx, RA_EINVAL, "invalid input:%s%s%s%s",
                            (bad & 1) ? " w <= 0 or non-finite;" : "",
                            (bad & 2) ? " cap or alpha-fair exponent c < 0 or non-finite;" : "",
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
    std::vector<double> pe(P->m);
    const double pR = fill_prices(P, p, &pe);
    ra_status st = enqueue_eval(P, lb, j_pair, x_pair, j1);
    if (st != RA_OK) return st;
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (collect_timing(ctx) != RA_OK) return RA_EDEVICE;
    const double* o = P->h_out;
    const double gv = pR + o[P->m];
    if (!std::isfinite(gv)) return fail(ctx, RA_ENUMERIC, "non-finite dual value");
    for (int j = 0; j < P->m; ++j)
        if (!std::isfinite(o[j])) return fail(ctx, RA_ENUMERIC, "non-finite usage");
    if (lb) {
        // U(X~) = g - [p^T (R - r) + sum_i (u(t_i) - u(t~_i))]
        double pq = 0.0;
        for (int j = 0; j < P->m; ++j) pq += pe[j] * (P->R[j] - o[j]);
        const double U = gv - (pq + o[P->m + 2]);
        if (!std::isfinite(U)) return fail(ctx, RA_ENUMERIC, "non-finite lower bound");
        *lower_bound = U;
    }
    *g = gv;
    for (int j = 0; j < P->m; ++j) grad[j] = P->R[j] - o[j];
    return RA_OK;
}

ra_status ra_dual_eval_noalloc(ra_ctx* ctx, const ra_problem* prob, const double* p,
                               double* g, double* grad, double* lower_bound)
{
    if (!ctx) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!p || !g || !grad) return fail(ctx, RA_EINVAL, "p, g and grad are required");
    if (!ctx->scratch) return fail(ctx, RA_EDEVICE, "device scratch address unknown");
    ra_problem* P = const_cast<ra_problem*>(prob);
    const int m = P->m;
    for (int j = 0; j < m; ++j)
        if (!(p[j] >= 0.0) || !std::isfinite(p[j]))
            return fail(ctx, RA_EINVAL, "p[%d] = %g must be >= 0 and finite", j, p[j]);
    // the block partials of at most NOALLOC_PARTIAL / (m + 3) blocks fit the
    // scratch; the dual kernels stride over the tiles, so a launch with fewer
    // blocks than the problem's usual grid covers every job
    const int ncols = ra::partial_cols(m);
    const int grid = std::min(P->grid, NOALLOC_PARTIAL / ncols);
    if (grid < 1 || ncols > NOALLOC_OUT)
        return fail(ctx, RA_EINVAL, "m = %d needs more scratch than the %d doubles held", m,
                    NOALLOC_PARTIAL + NOALLOC_OUT);
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    hipStream_t st = ctx->stream;
    double* part = ctx->scratch;
    double* dsum = ctx->scratch + NOALLOC_PARTIAL;
    const bool vec = ra::dual_is_vec(P->dt, m, dual_vec(P));
    double pe[RA_MAX_RESOURCES], o[NOALLOC_OUT], r[RA_MAX_RESOURCES];
    // one pass at p, or (pass 2) at p again with the certificate of p: every
    // job solved at q = p and its allocation scaled by the column scales of
    // r(p) (§5), in place of the per-job support workspace of ra_dual_eval
    auto pass = [&](bool with_prev) -> ra_status {
        (void)fill_prices(P, p, nullptr);
        if (with_prev) fill_prev_arrays(P, pe, r);
        if (!vec)
            RA_HIP(ctx, hipMemcpyAsync(P->pblock, P->h_pblock, price_block_bytes(P->dt),
                                       hipMemcpyHostToDevice, st));
        RA_HIP(ctx, ra::launch_dual(P->dt, m, dual_vec(P), grid, st, P->T, P->prm, P->n,
                                    P->pblock, P->h_pblock, P->eps, part, nullptr, nullptr,
                                    nullptr, nullptr, P->dem, P->dvec));
        RA_HIP(ctx, ra::launch_reduce_cols(st, part, grid, ncols, dsum));
        RA_HIP(ctx, hipMemcpyAsync(o, dsum, sizeof(double) * ncols, hipMemcpyDeviceToHost, st));
        RA_HIP(ctx, hipStreamSynchronize(st));
        return RA_OK;
    };
    double pR = 0.0;
    for (int j = 0; j < m; ++j) {
        pe[j] = P->dt == 0 ? (double)(float)p[j] : p[j];
        pR += pe[j] * P->R[j];
    }
    ra_status s1 = pass(false);
    if (s1 != RA_OK) return s1;
    const double gv = pR + o[m];
    if (!std::isfinite(gv)) return fail(ctx, RA_ENUMERIC, "non-finite dual value");
    for (int j = 0; j < m; ++j) {
        if (!std::isfinite(o[j])) return fail(ctx, RA_ENUMERIC, "non-finite usage");
        r[j] = o[j];
    }
    if (lower_bound) {
        ra_status s2 = pass(true);
        if (s2 != RA_OK) return s2;
        // U(X~) = g - [p^T (R - r) + sum_i (u(t_i) - u(t~_i))]
        double pq = 0.0;
        for (int j = 0; j < m; ++j) pq += pe[j] * (P->R[j] - r[j]);
        const double U = gv - (pq + o[m + 2]);
        if (!std::isfinite(U)) return fail(ctx, RA_ENUMERIC, "non-finite lower bound");
        *lower_bound = U;
    }
    *g = gv;
    for (int j = 0; j < m; ++j) grad[j] = P->R[j] - r[j];
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
    o->stall_evals = 0;
    o->init_step = 0.0;
    o->tol_abs = 0.0;
    o->device_loop = 0;
    o->stall_restarts = 0;
    o->warm_stall_restarts = -1;
    o->warm_stall_evals = 0;
}

static bool valid_opts(const ra_solve_opts& o)
{
    return o.tol_rel >= 0.0 && o.max_iter >= 0 && o.max_evals >= 0 && o.stall_evals >= 0 &&
           o.lbfgs_mem >= 1 && o.lbfgs_mem <= 64 && (o.method == 0 || o.method == 1) &&
           (o.init >= 0 && o.init <= 2) && o.init_step >= 0.0 && o.init_step <= 10.0 &&
           o.tol_abs >= 0.0 && std::isfinite(o.tol_abs) &&
           (o.device_loop == 0 || o.device_loop == 1) && o.stall_restarts >= 0 &&
           o.warm_stall_restarts >= -1 && o.warm_stall_evals >= 0;
}

namespace {

// Captured evaluation graphs hold the kernels' arguments; drop them when the
// problem's inputs to those kernels change.
void drop_graphs(ra_problem* P)
{
    // spare passes of a device-loop solve may still be queued
    if (P->dl_gexec) (void)hipStreamSynchronize(P->ctx->stream);
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->dl_gexec) (void)hipGraphExecDestroy(P->dl_gexec);
    if (P->dl_graph) (void)hipGraphDestroy(P->dl_graph);
    P->gexec = nullptr;
    P->graph = nullptr;
    P->dl_gexec = nullptr;
    P->dl_graph = nullptr;
}

// Passes per replay of the device loop's graph: one host synchronisation
// per this many passes (later passes of a chunk return at once once the loop
// has ended).
constexpr int DL_CHUNK = 6;

bool device_loop_applies(const ra_problem* P, const ra_solve_opts& o)
{
    const ra_ctx* ctx = P->ctx;
    return o.device_loop && ra::dual_is_vec(P->dt, P->m, dual_vec(P)) &&
           P->m <= ra::DL_MAX_M && o.lbfgs_mem <= ra::DL_MAX_MEM && !ctx->timing &&
           !o.verbose && ctx->stream != nullptr;
}

// The price block of a vectorised pass at prices p (no previous point), in
// the layout of PriceArgs<m>: p, 1/p, q, 1/q, s, 1 - s (m floats each), then
// has_prev.
void first_price_args(int m, const std::vector<double>& p, std::vector<double>& pe,
                      const std::vector<double>& R, double& pR, std::vector<float>& a)
{
    a.assign(6 * (size_t)m + 1, 0.f);
    pR = 0.0;
    pe.resize(m);
    for (int j = 0; j < m; ++j) {
        const float pf = (float)std::max(p[j], 0.0);
        a[j] = pf;
        a[m + j] = pf > 0.f ? 1.0f / pf : INFINITY;
        a[2 * m + j] = 0.f;
        a[3 * m + j] = INFINITY;
        a[4 * m + j] = 1.f;
        a[5 * m + j] = 0.f;
        pe[j] = (double)pf;
        pR += (double)pf * R[j];
    }
    // the last word (has_prev) stays 0
}

ra_status capture_dev_loop(ra_problem* P)
{
    ra_ctx* ctx = P->ctx;
    if (P->dl_gexec) return RA_OK;
    hipStream_t st = ctx->stream;
    const int* skip = &P->dloop->done;
    RA_HIP(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < DL_CHUNK && e == hipSuccess; ++k) {
        e = ra::launch_dual_dev(P->m, P->grid, st, P->T, P->prm, P->n, P->eps, P->partial, P->dem,
                                P->dvec, P->dprices, skip);
        if (e == hipSuccess)
            e = ra::launch_reduce_step(P->m, st, P->partial, P->grid, P->dloop, P->dout,
                                       P->dprices, P->h_dl);
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &g);
    if (e == hipSuccess) e = ee;
    if (e == hipSuccess) e = hipGraphInstantiate(&P->dl_gexec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        P->dl_gexec = nullptr;
        return fail(ctx, RA_EDEVICE, "device loop graph: %s", hipGetErrorString(e));
    }
    P->dl_graph = g;
    return RA_OK;
}

// Algorithm 2 with the price update on the device: the host writes the
// loop's configuration and first prices, then replays a graph of DL_CHUNK
// passes [dual kernel -> column sums and step], keeping one replay queued
// ahead of the device, until the step that ends the loop publishes the
// outcome in pinned memory.  Spare passes of the last replays return at once;
// they may still be queued on the stream when this returns.
ra_status solve_device(ra_problem* P, const ra_solve_opts& o, const std::vector<double>& p0,
                       double* p_inout, ra_solve_info* info,
                       std::chrono::steady_clock::time_point t0)
{
    ra_ctx* ctx = P->ctx;
    hipStream_t st = ctx->stream;
    const int m = P->m;
    if (!P->dloop) {
        RA_HIP(ctx, hipMalloc((void**)&P->dloop, sizeof(ra::DevLoop)));
        // the reduction's ticket starts at zero
        RA_HIP(ctx, hipMemsetAsync(P->dloop, 0, sizeof(ra::DevLoop), st));
    }
    if (!P->dprices) RA_HIP(ctx, hipMalloc(&P->dprices, sizeof(float) * (6 * ra::DL_MAX_M + 1)));
    if (!P->h_dl)
        RA_HIP(ctx, hipHostMalloc((void**)&P->h_dl, sizeof(ra::DevStatus), hipHostMallocCoherent));
    // the header, then the first pass's price block
    constexpr size_t hbytes = offsetof(ra::DevLoop, res_p);
    if (!P->h_dlstage)
        RA_HIP(ctx, hipHostMalloc(&P->h_dlstage, sizeof(ra::DevLoop) + 4096, hipHostMallocDefault));
    // the previous solve's copies from this buffer ended before its passes
    ra::DevLoop* h = new (P->h_dlstage) ra::DevLoop();
    h->m = m;
    h->mem = o.lbfgs_mem;
    h->method = o.method;
    h->max_iter = o.max_iter;
    h->max_evals = o.max_evals;
    h->stall_evals = o.stall_evals;
    h->stall_restarts = o.stall_restarts;
    h->n = (double)P->n;
    h->tol_rel = o.tol_rel;
    h->tol_abs = o.tol_abs;
    h->init_step = o.init_step;
    for (int j = 0; j < m; ++j) h->R[j] = P->R[j];
    std::vector<double> pe;
    double pR = 0.0;
    std::vector<float> a;
    first_price_args(m, p0, pe, P->R, pR, a);
    for (int j = 0; j < m; ++j) h->pe[j] = pe[j];
    h->pR = pR;
    h->lam = 1.0;
    // earlier replays may still be queued: the new header is written in
    // stream order after them, and none of them writes the status record
    ra::DevStatus* hs = P->h_dl;
    __atomic_store_n(&hs->passes, 0, __ATOMIC_RELAXED);
    __atomic_store_n(&hs->done, 0, __ATOMIC_RELEASE);
    char* pb = static_cast<char*>(P->h_dlstage) + sizeof(ra::DevLoop);
    std::memcpy(pb, a.data(), sizeof(float) * a.size());
    RA_HIP(ctx, hipMemcpyAsync(P->dloop, h, hbytes, hipMemcpyHostToDevice, st));
    RA_HIP(ctx, hipMemcpyAsync(P->dprices, pb, sizeof(float) * a.size(), hipMemcpyHostToDevice,
                               st));
    ra_status cs = capture_dev_loop(P);
    if (cs != RA_OK) return cs;
    // the number of passes cannot exceed the budget, or 21 per iteration
    // (20 halvings and a subgradient step) plus the final certification
    const int64_t bound = o.max_evals > 0 ? (int64_t)o.max_evals : (int64_t)(o.max_iter + 2) * 21;
    const int64_t max_chunks = bound / DL_CHUNK + 2;
    int64_t launched = 0;
    for (uint64_t k = 0;; ++k) {
        const int done = __atomic_load_n(&hs->done, __ATOMIC_ACQUIRE);
        if (done) break;
        const int64_t passes = __atomic_load_n(&hs->passes, __ATOMIC_RELAXED);
        // keep one replay queued behind the one the device is running
        if (launched < max_chunks && passes >= (launched - 1) * DL_CHUNK) {
            const hipError_t e = hipGraphLaunch(P->dl_gexec, st);
            if (e != hipSuccess) {
                // no earlier replay may outlive this call: a later solve
                // resets the status record they write
                (void)hipStreamSynchronize(st);
                return fail(ctx, RA_EDEVICE, "device loop launch: %s", hipGetErrorString(e));
            }
            ++launched;
            continue;
        }
        if ((k & 4095) == 0) {
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess) {
                if (__atomic_load_n(&hs->done, __ATOMIC_ACQUIRE)) break;
                if (launched >= max_chunks)
                    return fail(ctx, RA_EDEVICE,
                                "the device price loop did not end within its budget");
                continue;
            }
            if (e != hipErrorNotReady)
                return fail(ctx, RA_EDEVICE, "device price loop failed: %s", hipGetErrorString(e));
        }
        __builtin_ia32_pause();
    }
    if (hs->done == 2) return fail(ctx, RA_ENUMERIC, "non-finite dual value, usage or gap");
    const bool conv = hs->converged != 0;
    for (int j = 0; j < m; ++j) p_inout[j] = hs->p[j];
    if (info) {
        info->iters = hs->iters;
        info->dual_evals = hs->evals;
        info->fell_back = hs->fallbacks;
        info->converged = conv ? 1 : 0;
        info->g = hs->g;
        info->U_lb = hs->certified ? hs->U : NAN;
        info->rel_gap = hs->certified ? hs->rel : INFINITY;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->restarted = 0;
        info->warm_evals = 0;
    }
    return conv ? RA_OK : RA_ENOTCONV;
}

}  // namespace

ra_status ra_solve(ra_ctx* ctx, const ra_problem* prob, const ra_solve_opts* opts,
                   double* p_inout, ra_solve_info* info)
{
    if (!ctx) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!p_inout) return fail(ctx, RA_EINVAL, "p_inout is required");
    ra_solve_opts o;
    ra_solve_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return fail(ctx, RA_EINVAL, "invalid solve options");
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
    if (o.init == 2) {
        ra_status st = init_prices(P, p.data());
        if (st != RA_OK) return st;
    }

    if (device_loop_applies(P, o)) return solve_device(P, o, p, p_inout, info, t0);

    ra::PriceLoop L(m, P->n, P->R.data(), o, p.data());
    std::vector<double> pe, rr;
    double gv = 0.0, sdu = 0.0;
    while (!L.done()) {
        const int nc = L.ncertified();
        ra_status st = run_pass(P, L.next(), L.pending(), graph, pe, gv, rr, sdu);
        if (st != RA_OK) return st;
        L.feed(pe, gv, rr.data(), sdu);
        if (o.verbose && L.ncertified() > nc) {
            const ra::Point& c = L.last_certified();
            fprintf(stderr, "iteration %02d | utility=%.6f | dual_value=%.6f | gap=%.2e\n",
                    L.ncertified() - 1, c.U / (double)P->n, c.g / (double)P->n,
                    c.gap / (double)P->n);
        }
    }
    // the last reduction may still be retiring after its flag
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const ra::Point& ret = L.result();
    const bool conv = L.converged();
    if (o.verbose)
        fprintf(stderr, "%s in %03d iterations, with residual %g\n",
                conv ? "Converged" : "Stopped", L.iters(), ret.gap / (double)P->n);
    for (int j = 0; j < m; ++j) p_inout[j] = ret.p[j];
    if (info) {
        info->iters = L.iters();
        info->dual_evals = L.evals();
        info->fell_back = L.fallbacks();
        info->converged = conv ? 1 : 0;
        info->g = ret.g;
        info->U_lb = ret.certified ? ret.U : NAN;
        info->rel_gap = ret.certified ? ret.rel : INFINITY;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->restarted = 0;
        info->warm_evals = 0;
    }
    return conv ? RA_OK : RA_ENOTCONV;
}

ra_status ra_problem_set_demands(ra_ctx* ctx, ra_problem* P, const void* d)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!P || P->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    hipStream_t st = ctx->stream;
    const size_t bytes = (size_t)P->n * elt(P->dt);
    // captured graphs hold the previous demand pointer
    drop_graphs(P);
    if (d && P->dvec)
        return fail(ctx, RA_EINVAL, "the problem has demand vectors; remove them first");
    if (!d) {
        if (!P->dem) return RA_OK;
        RA_HIP(ctx, ra::launch_demands(P->dt, st, 2, nullptr, P->w0, P->n, P->prm, nullptr, nullptr));
        RA_HIP(ctx, hipStreamSynchronize(st));
        (void)hipFree(P->dem);
        P->dem = nullptr;
        return RA_OK;
    }
    if (!P->w0) {
        RA_HIP(ctx, hipMalloc(&P->w0, bytes));
        RA_HIP(ctx, ra::launch_demands(P->dt, st, 0, nullptr, P->w0, P->n, P->prm, nullptr, nullptr));
    }
    const bool fresh = P->dem == nullptr;
    if (fresh) RA_HIP(ctx, hipMalloc(&P->dem, bytes));
    int* dbad = nullptr;
    RA_HIP(ctx, hipMalloc((void**)&dbad, sizeof(int)));
    int bad = 0;
    hipError_t e = hipMemsetAsync(dbad, 0, sizeof(int), st);
    if (e == hipSuccess) e = ra::launch_demands(P->dt, st, 1, d, P->w0, P->n, P->prm, P->dem, dbad);
    if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(dbad);
    if (e != hipSuccess) return fail(ctx, RA_EDEVICE, "set demands: %s", hipGetErrorString(e));
    if (bad) {
        // leave the problem as it was before demands: weights restored, no demands
        RA_HIP(ctx, ra::launch_demands(P->dt, st, 2, nullptr, P->w0, P->n, P->prm, nullptr, nullptr));
        RA_HIP(ctx, hipStreamSynchronize(st));
        (void)hipFree(P->dem);
        P->dem = nullptr;
        return fail(ctx, RA_EINVAL, "demands must be positive and finite");
    }
    return RA_OK;
}

ra_status ra_problem_set_demand_vectors(ra_ctx* ctx, ra_problem* P, const void* D)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!P || P->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (D && P->dem)
        return fail(ctx, RA_EINVAL, "the problem has scalar demands; remove them first");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    hipStream_t st = ctx->stream;
    if (D) {
        int* dbad = nullptr;
        RA_HIP(ctx, hipMalloc((void**)&dbad, sizeof(int)));
        int zero = 0, bad = 0;
        hipError_t e = hipMemcpyAsync(dbad, &zero, sizeof(int), hipMemcpyHostToDevice, st);
        if (e == hipSuccess)
            e = ra::launch_validate_T(P->dt, st, D, P->n * (int64_t)P->m, dbad, true);
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, dbad, sizeof(int), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        (void)hipFree(dbad);
        if (e != hipSuccess)
            return fail(ctx, RA_EDEVICE, "set demand vectors: %s", hipGetErrorString(e));
        if (bad) return fail(ctx, RA_EINVAL, "demand vectors must be positive and finite");
    }
    // captured graphs hold the previous kernel and its arguments
    drop_graphs(P);
    P->dvec = D;
    const int g = ra::dual_grid(ctx->cus, P->m, P->dt, P->n, dual_vec(P), D != nullptr);
    if (g > P->grid_cap) {
        RA_HIP(ctx, hipStreamSynchronize(st));
        (void)hipFree(P->partial);
        P->partial = nullptr;
        P->grid_cap = 0;
        RA_HIP(ctx, hipMalloc(&P->partial, sizeof(double) * (size_t)g * ra::partial_cols(P->m)));
        P->grid_cap = g;
    }
    P->grid = g;
    return RA_OK;
}

ra_status ra_init_prices(ra_ctx* ctx, const ra_problem* prob, double* p_out)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!p_out) return fail(ctx, RA_EINVAL, "p_out is required");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    return init_prices(const_cast<ra_problem*>(prob), p_out);
}

ra_status ra_predict_prices(ra_ctx* ctx, const ra_problem* prob, ra_mlp* mlp, double* p_out)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!mlp || !p_out) return fail(ctx, RA_EINVAL, "network and p_out are required");
    ra_problem* P = const_cast<ra_problem*>(prob);
    if (P->dt != 0 || P->m > 64)
        return fail(ctx, RA_EUNSUPPORTED, "learned warm start needs an FP32 problem with m <= 64");
    if (ra::mlp_out_dim(mlp) != P->m || ra::mlp_in_dim(mlp) != 8 * P->m + 16)
        return fail(ctx, RA_EINVAL, "network dimensions do not match the problem (in 8m+16, out m)");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    std::vector<double> p0;
    ra_status st = ra::predict_prices(mlp, P, p0);
    if (st != RA_OK) return st;
    for (int j = 0; j < P->m; ++j) p_out[j] = p0[j];
    return RA_OK;
}

// Learned warm start with a cold restart when the warm run does not improve
// its starting certificate within `window` certified points.
ra_status ra_solve_learned(ra_ctx* ctx, const ra_problem* prob, ra_mlp* mlp,
                           const ra_solve_opts* opts, int32_t window, double* p_out,
                           ra_solve_info* info)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!mlp || !p_out) return fail(ctx, RA_EINVAL, "network and p_out are required");
    ra_problem* P = const_cast<ra_problem*>(prob);
    const int m = P->m;
    if (P->dt != 0 || m > 64)
        return fail(ctx, RA_EUNSUPPORTED, "learned warm start needs an FP32 problem with m <= 64");
    if (ra::mlp_out_dim(mlp) != m || ra::mlp_in_dim(mlp) != 8 * m + 16)
        return fail(ctx, RA_EINVAL, "network dimensions do not match the problem (in 8m+16, out m)");
    if (window < 1) return fail(ctx, RA_EINVAL, "fallback_window must be >= 1");
    ra_solve_opts o;
    ra_solve_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return fail(ctx, RA_EINVAL, "invalid solve options");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    const auto t0 = std::chrono::steady_clock::now();
    const bool graph = o.use_graph && ctx->stream != nullptr;

    std::vector<double> p0;
    ra_status st = ra::predict_prices(mlp, P, p0);
    if (st != RA_OK) return st;
    bool warm_ok = true;
    for (double v : p0) warm_ok = warm_ok && std::isfinite(v) && v >= 0.0;
    int warm_evals = 0;
    // 1: the warm run was abandoned early (or could not start), 2: it stalled
    int restarted = warm_ok ? 0 : 1;
    std::vector<double> pe, rr;
    double gv = 0.0, sdu = 0.0;
    // a predicted start is expected within a few percent of p*: the first
    // step is kept to that scale so that it does not undo the prediction
    ra_solve_opts ow = o;
    if (ow.init_step == 0.0) ow.init_step = 0.005;
    if (o.warm_stall_restarts >= 0) ow.stall_restarts = o.warm_stall_restarts;
    if (o.warm_stall_evals > 0) ow.stall_evals = o.warm_stall_evals;
    ra::PriceLoop W(m, P->n, P->R.data(), ow, warm_ok ? p0.data() : std::vector<double>(m, 1.0).data());
    if (warm_ok) {
        double rel0 = INFINITY;
        while (!W.done()) {
            st = run_pass(P, W.next(), W.pending(), graph, pe, gv, rr, sdu);
            if (st == RA_ENUMERIC) {
                restarted = 1;
                break;
            }
            if (st != RA_OK) return st;
            W.feed(pe, gv, rr.data(), sdu);
            if (W.ncertified() == 1 && !std::isfinite(rel0)) rel0 = W.last_certified().rel;
            if (W.ncertified() >= window && !W.done()) {
                const double best = W.result().certified ? W.result().rel : INFINITY;
                if (!(best < rel0)) restarted = 1;  // the gap did not fall: go cold
                break;
            }
        }
        if (!restarted) {
            while (!W.done()) {
                st = run_pass(P, W.next(), W.pending(), graph, pe, gv, rr, sdu);
                if (st != RA_OK) return st;
                W.feed(pe, gv, rr.data(), sdu);
            }
            // a warm run that stalled short of the tolerance hands over to a
            // cold solve while the pass budget lasts
            if (o.warm_stall_restarts >= 0 && W.stalled() && !W.converged() &&
                (o.max_evals == 0 || W.evals() < o.max_evals))
                restarted = 2;
        }
        warm_evals = W.evals();
    }
    ra_solve_opts oc = o;
    oc.init = 0;
    if (restarted && o.max_evals > 0) oc.max_evals = o.max_evals - warm_evals;  // >= 1
    std::vector<double> ones(m, 1.0);
    ra::PriceLoop C(m, P->n, P->R.data(), oc, ones.data());
    if (restarted) {
        while (!C.done()) {
            st = run_pass(P, C.next(), C.pending(), graph, pe, gv, rr, sdu);
            if (st != RA_OK) return st;
            C.feed(pe, gv, rr.data(), sdu);
        }
    }
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    // the outcome: the warm run's, the cold run's after an early abandon, and
    // after a stall the better certified point of the two
    const ra::PriceLoop* L = restarted ? &C : &W;
    if (restarted == 2) {
        const ra::Point& a = W.result();
        const ra::Point& b = C.result();
        if (!C.converged() && a.certified && (!b.certified || a.rel <= b.rel)) L = &W;
    }
    const ra::Point* out = &L->result();
    for (int j = 0; j < m; ++j) p_out[j] = out->p[j];
    const bool conv = L->converged();
    if (info) {
        // a run that never started counts zero
        info->iters = W.iters() + C.iters();
        info->dual_evals = W.evals() + C.evals();
        info->fell_back = W.fallbacks() + C.fallbacks();
        info->converged = conv ? 1 : 0;
        info->g = out->g;
        info->U_lb = out->certified ? out->U : NAN;
        info->rel_gap = out->certified ? out->rel : INFINITY;
        info->seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->restarted = restarted;
        info->warm_evals = restarted ? warm_evals : 0;
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

// ---------------------------------------------------------------------------
// Batched price discovery.
// ---------------------------------------------------------------------------
namespace {

size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

struct BatchWs {
    int B = 0, Wmax = 0;
    // table sections (offsets into htab / dtab) of the current layout;
    // tab_bytes is the allocation, tab_used what a round copies
    size_t off_items = 0, off_prices = 0, off_chunk = 0, off_segbase = 0, off_seg = 0,
           off_header = 0, tab_bytes = 0, tab_used = 0;
    // compact: each round lays its table out for its own wave and problem
    // counts (the copy then moves only what the round uses); otherwise the
    // layout is the fixed one of the allocation, as a captured graph needs
    bool compact = false;
    char* dtab = nullptr;
    char* htab = nullptr;
    double* partial = nullptr;
    bool used = false;
    bool demands = false;     // some problem of the batch has per-job demands
    bool alpha_fair = false;  // some problem of the batch has alpha-fair jobs
    hipStream_t st_sync = nullptr;
    double* hout = nullptr;     // fine-grained host memory: B rows of results, then the flag
    unsigned* hflag = nullptr;
    unsigned* ticket = nullptr;  // device block counter of the reduction
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    int graph_grid = 0, graph_tf = 0, graph_lds = 0;
    bool graph_dem = false, graph_af = false;  // kernel variant of the captured graph
    // the launch shape of the next rounds
    int tf = 2048, lds_floats = 0;
    ~BatchWs()
    {
        // launches that use these buffers must have finished
        if (used) (void)hipStreamSynchronize(st_sync);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipFree(dtab);
        (void)hipFree(partial);
        (void)hipFree(ticket);
        if (htab) (void)hipHostFree(htab);
        if (hout) (void)hipHostFree(hout);
    }
    ra::BatchItem* items() { return reinterpret_cast<ra::BatchItem*>(htab + off_items); }
    float* prices() { return reinterpret_cast<float*>(htab + off_prices); }
    int* chunk() { return reinterpret_cast<int*>(htab + off_chunk); }
    int* segbase() { return reinterpret_cast<int*>(htab + off_segbase); }
    int* seg() { return reinterpret_cast<int*>(htab + off_seg); }
    int* header() { return reinterpret_cast<int*>(htab + off_header); }
    // section offsets for W waves and A problems: header, chunk (W + 1),
    // segbase (W + 1), seg (2 A), items (A + 1), prices (A rows of
    // 6 BATCH_MAX_M floats)
    void layout(int W, int A)
    {
        size_t o = 0;
        off_header = o;
        o = align16(o + sizeof(int) * 4);
        off_chunk = o;
        o = align16(o + sizeof(int) * (size_t)(W + 1));
        off_segbase = o;
        o = align16(o + sizeof(int) * (size_t)(W + 1));
        off_seg = o;
        o = align16(o + sizeof(int) * 2 * (size_t)A);
        off_items = o;
        o = align16(o + sizeof(ra::BatchItem) * (size_t)(A + 1));
        off_prices = o;
        o = align16(o + sizeof(float) * 6 * ra::BATCH_MAX_M * (size_t)A);
        tab_used = o;
    }
};

ra_status batch_alloc(ra_ctx* ctx, BatchWs& ws, int B, int Wmax)
{
    ws.used = true;
    ws.st_sync = ctx->stream;
    ws.B = B;
    ws.Wmax = Wmax;
    // the fixed layout is the largest: every compact one fits in it
    ws.layout(Wmax, B);
    ws.tab_bytes = ws.tab_used;
    RA_HIP(ctx, hipMalloc(&ws.dtab, ws.tab_bytes));
    // coherent: the table copy kernel reads it over the bus
    RA_HIP(ctx, hipHostMalloc((void**)&ws.htab, ws.tab_bytes, hipHostMallocCoherent));
    std::memset(ws.htab, 0, ws.tab_bytes);
    RA_HIP(ctx, hipMalloc(&ws.partial,
                          sizeof(double) * ra::BATCH_COLS * (size_t)(Wmax + B)));
    RA_HIP(ctx, hipHostMalloc((void**)&ws.hout, sizeof(double) * (ra::BATCH_COLS * (size_t)B + 1),
                              hipHostMallocCoherent));
    ws.hflag = reinterpret_cast<unsigned*>(ws.hout + ra::BATCH_COLS * (size_t)B);
    *ws.hflag = 0u;
    RA_HIP(ctx, hipMalloc((void**)&ws.ticket, sizeof(unsigned)));
    RA_HIP(ctx, hipMemsetAsync(ws.ticket, 0, sizeof(unsigned), ctx->stream));
    return RA_OK;
}

// Spread per-problem work over the context's host threads when there is
// enough of it; fn(lo, hi) handles problems [lo, hi).
void for_problems(ra::HostPool* pool, int A, const std::function<void(int, int)>& fn)
{
    if (pool && A >= 64)
        pool->run(A, fn);
    else
        fn(0, A);
}

// LDS floats per wave of a tile of `rows` rows for m resources (T staged
// with the padded stride, then (w, c) and, with demands, d per row), a
// multiple of 4 so that every wave's tile stays 16-byte aligned.
int batch_lds_floats(int m, int rows, bool demands)
{
    const int f = rows * (ra::batch_stride(m) + 2 + (demands ? 1 : 0));
    return (f + 3) & ~3;
}

// Fill the tables of one round for the active problems `act` (ascending) with
// W waves: items, prices (next point and, if any, the point to certify),
// per-wave tile chunks balanced by cost (T.cost, ns per job of each m class,
// else 4 m + 8 bytes per job), partial slots.  force_prev: every problem
// also certifies (its next point, with unit scales): the tuner's rounds do
// the work of a solver round.  Sets ws.tf and ws.lds_floats.  Returns the
// tile count.
int64_t batch_fill(BatchWs& ws, const std::vector<ra_problem*>& probs,
                   const std::vector<ra::PriceLoop>& loops, const std::vector<int>& act, int W,
                   std::vector<std::vector<double>>& p_eval, ra::HostPool* pool,
                   const ra::BatchTuned& T, bool force_prev = false)
{
    const int A = (int)act.size();
    if (ws.compact)
        ws.layout(W, A);
    else
        ws.layout(ws.Wmax, ws.B);
    ra::BatchItem* it = ws.items();
    float* pr = ws.prices();
    std::vector<int64_t> tiles(A);
    std::vector<double> cost(A);
    int64_t tt = 0;
    double C = 0.0;
    int lds = 4;
    for (int a = 0; a < A; ++a) {
        const int m = probs[act[a]]->m;
        lds = std::max(lds, batch_lds_floats(m, T.shape.rows[ra::batch_class(m)], ws.demands));
    }
    ws.tf = T.shape.tile_floats;
    ws.lds_floats = lds;
    // each problem's record and price rows (independent per problem)
    for_problems(pool, A, [&](int lo, int hi) {
    for (int a = lo; a < hi; ++a) {
        const ra_problem* P = probs[act[a]];
        const ra::PriceLoop& L = loops[act[a]];
        const int cls = ra::batch_class(P->m);
        const int tr = T.shape.rows[cls];
        tiles[a] = (P->n + tr - 1) / tr;
        cost[a] = (double)tr * (T.cost[cls] > 0.0 ? T.cost[cls] : (double)(4 * P->m + 8));
        it[a].T = static_cast<const float*>(P->T);
        it[a].prm = static_cast<const float2*>(P->prm);
        it[a].n = P->n;
        it[a].m = P->m;
        it[a].rows = tr;
        it[a].eps = (float)P->eps;
        const ra::Point* prev = L.pending();
        it[a].has_prev = (prev || force_prev) ? 1 : 0;
        it[a].dem = static_cast<const float*>(P->dem);
        float* row = pr + (size_t)a * 6 * ra::BATCH_MAX_M;
        const std::vector<double>& nx = L.next();
        p_eval[a].resize(P->m);
        for (int j = 0; j < P->m; ++j) {
            const float pf = (float)nx[j];
            p_eval[a][j] = pf;
            row[j] = pf;
            row[ra::BATCH_MAX_M + j] = pf > 0.f ? 1.0f / pf : INFINITY;
            if (prev) {
                const float qf = (float)prev->p[j];
                row[2 * ra::BATCH_MAX_M + j] = qf;
                row[3 * ra::BATCH_MAX_M + j] = qf > 0.f ? 1.0f / qf : INFINITY;
                const bool over = prev->r[j] > P->R[j];
                row[4 * ra::BATCH_MAX_M + j] = over ? (float)(P->R[j] / prev->r[j]) : 1.0f;
                row[5 * ra::BATCH_MAX_M + j] =
                    over ? (float)((prev->r[j] - P->R[j]) / prev->r[j]) : 0.0f;
            } else if (force_prev) {
                row[2 * ra::BATCH_MAX_M + j] = pf;
                row[3 * ra::BATCH_MAX_M + j] = row[ra::BATCH_MAX_M + j];
                row[4 * ra::BATCH_MAX_M + j] = 1.0f;
                row[5 * ra::BATCH_MAX_M + j] = 0.0f;
            }
        }
    }
    });
    // tile offsets in problem order
    for (int a = 0; a < A; ++a) {
        it[a].tile0 = (int)tt;
        tt += tiles[a];
        C += (double)tiles[a] * cost[a];
    }
    it[A].tile0 = (int)tt;
    // wave w starts at the first tile whose cumulative cost reaches w C / W
    int* ch = ws.chunk();
    {
        int a = 0;
        double cc = 0.0;  // cost before problem a
        for (int w = 0; w <= W; ++w) {
            const double target = C * (double)w / (double)W;
            while (a < A && cc + (double)tiles[a] * cost[a] <= target) {
                cc += (double)tiles[a] * cost[a];
                ++a;
            }
            if (a >= A || w == W) {
                ch[w] = (int)tt;
            } else {
                int64_t k = (int64_t)std::ceil((target - cc) / cost[a]);
                k = std::min<int64_t>(std::max<int64_t>(k, 0), tiles[a]);
                ch[w] = it[a].tile0 + (int)k;
            }
        }
        for (int w = 1; w <= W; ++w) ch[w] = std::max(ch[w], ch[w - 1]);
        ch[W] = (int)tt;
    }
    // partial slots: one per (wave, problem it touches), contiguous per problem
    int* sb = ws.segbase();
    int* sg = ws.seg();
    for (int a = 0; a < A; ++a) sg[2 * a] = -1;
    int slot = 0, a = 0;
    for (int w = 0; w < W; ++w) {
        sb[w] = slot;
        if (ch[w] >= ch[w + 1]) continue;
        while (it[a + 1].tile0 <= ch[w]) ++a;
        int b = a;
        while (it[b + 1].tile0 < ch[w + 1]) ++b;
        for (int k = a; k <= b; ++k, ++slot) {
            if (sg[2 * k] < 0) sg[2 * k] = slot;
            sg[2 * k + 1] = slot;
        }
    }
    sb[W] = slot;
    ws.header()[0] = A;
    return tt;
}

ra_status batch_enqueue(ra_ctx* ctx, BatchWs& ws, int grid)
{
    hipStream_t st = ctx->stream;
    // a compact round's table is copied by a kernel (launched without
    // holding the host); a captured graph keeps its copy node
    if (ws.compact)
        RA_HIP(ctx, ra::launch_copy_table(ws.htab, ws.dtab, ws.tab_used, st));
    else
        RA_HIP(ctx, hipMemcpyAsync(ws.dtab, ws.htab, ws.tab_used, hipMemcpyHostToDevice, st));
    // the reduction takes a block per active problem (up to 256); every
    // block raises a system-wide fence, so a compact round launches no idle
    // ones (a captured graph keeps the capacity)
    const int red_items = ws.compact ? std::max(1, ws.header()[0]) : ws.B;
    RA_HIP(ctx, ra::launch_batch(ws.tf, ws.lds_floats, grid, red_items, st,
                                 reinterpret_cast<const ra::BatchItem*>(ws.dtab + ws.off_items),
                                 reinterpret_cast<const float*>(ws.dtab + ws.off_prices),
                                 reinterpret_cast<const int*>(ws.dtab + ws.off_chunk),
                                 reinterpret_cast<const int*>(ws.dtab + ws.off_segbase),
                                 reinterpret_cast<const int*>(ws.dtab + ws.off_seg),
                                 reinterpret_cast<const int*>(ws.dtab + ws.off_header), ws.partial,
                                 ws.hout, ws.ticket, ws.hflag, ws.demands, ws.alpha_fair));
    return RA_OK;
}

// Queue one round (table copy, batched kernel, reduction) on the context's
// stream, from a captured graph when use_graph (fixed layout only), and
// return without waiting: the round raises ws.hflag when its results are in
// ws.hout.
ra_status batch_launch(ra_ctx* ctx, BatchWs& ws, int grid, bool use_graph)
{
    __atomic_store_n(ws.hflag, 0u, __ATOMIC_RELEASE);
    if (use_graph && !ctx->timing && !ws.compact) {
        if (!ws.gexec || ws.graph_grid != grid || ws.graph_tf != ws.tf ||
            ws.graph_lds != ws.lds_floats || ws.graph_dem != ws.demands ||
            ws.graph_af != ws.alpha_fair) {
            if (ws.gexec) (void)hipGraphExecDestroy(ws.gexec);
            if (ws.graph) (void)hipGraphDestroy(ws.graph);
            ws.gexec = nullptr;
            ws.graph = nullptr;
            RA_HIP(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
            ra_status s = batch_enqueue(ctx, ws, grid);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(ctx->stream, &g);
            if (s != RA_OK) {
                if (g) (void)hipGraphDestroy(g);
                return s;
            }
            if (e != hipSuccess)
                return fail(ctx, RA_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&ws.gexec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                return fail(ctx, RA_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
            }
            ws.graph = g;
            ws.graph_grid = grid;
            ws.graph_tf = ws.tf;
            ws.graph_lds = ws.lds_floats;
            ws.graph_dem = ws.demands;
            ws.graph_af = ws.alpha_fair;
        }
        RA_HIP(ctx, hipGraphLaunch(ws.gexec, ctx->stream));
        return RA_OK;
    }
    return batch_enqueue(ctx, ws, grid);
}


std::string batch_signature(const std::vector<ra_problem*>& probs, bool demands, bool alpha_fair)
{
    // number of problems, total MiB of T (rounded), the m histogram and the
    // kernel variant
    int64_t bytes = 0;
    int hist[4] = {0, 0, 0, 0};
    for (const ra_problem* P : probs) {
        bytes += P->n * (int64_t)P->m * 4;
        hist[ra::batch_class(P->m)]++;
    }
    char buf[160];
    snprintf(buf, sizeof(buf), "B%zu_MiB%lld_m%d.%d.%d.%d_d%d_a%d", probs.size(),
             (long long)(bytes >> 20), hist[0], hist[1], hist[2], hist[3], demands ? 1 : 0,
             alpha_fair ? 1 : 0);
    return buf;
}

const int kBatchMs[4] = {4, 8, 16, 32};

// batches of at least this many problems run as two interleaved groups
const int kBatchGroupsMin = 16;

// A shape is usable for a batch when every m class present has a valid tile
// height under the shape's budget.
bool shape_fits(const ra::BatchShape& sh, const bool (&have)[4])
{
    if (sh.tile_floats != 1024 && sh.tile_floats != 2048 && sh.tile_floats != 4096) return false;
    for (int c = 0; c < 4; ++c)
        if (have[c] && !ra::batch_rows_ok(sh.tile_floats, kBatchMs[c], sh.rows[c])) return false;
    return true;
}

// The tuning cache file (RESALLOC_TUNE_CACHE): one line per batch signature,
// "signature tile_floats rows4 rows8 rows16 rows32 blocks_per_cu cost4 cost8
// cost16 cost32".  Lines that do not parse are skipped.
void tune_cache_load(ra_ctx* ctx)
{
    const char* path = std::getenv("RESALLOC_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        char key[200];
        ra::BatchTuned t;
        if (std::sscanf(line, "%199s %d %d %d %d %d %d %lf %lf %lf %lf", key, &t.shape.tile_floats,
                        &t.shape.rows[0], &t.shape.rows[1], &t.shape.rows[2], &t.shape.rows[3],
                        &t.shape.bpc, &t.cost[0], &t.cost[1], &t.cost[2], &t.cost[3]) == 11 &&
            t.shape.bpc >= 1)
            ctx->batch_tuned.emplace(key, t);
    }
    std::fclose(f);
}

void tune_cache_store(const ra_ctx* ctx)
{
    const char* path = std::getenv("RESALLOC_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "w");
    if (!f) return;
    for (const auto& kv : ctx->batch_tuned) {
        const ra::BatchTuned& t = kv.second;
        std::fprintf(f, "%s %d %d %d %d %d %d %.6g %.6g %.6g %.6g\n", kv.first.c_str(),
                     t.shape.tile_floats, t.shape.rows[0], t.shape.rows[1], t.shape.rows[2],
                     t.shape.rows[3], t.shape.bpc, t.cost[0], t.cost[1], t.cost[2], t.cost[3]);
    }
    std::fclose(f);
}

// LDS floats per wave that a batch's tiles need under shape T.
int batch_lds_of(const std::vector<ra_problem*>& P, const std::vector<int>& act,
                 const ra::BatchTuned& T, bool demands)
{
    int lds = 4;
    for (int b : act)
        lds = std::max(lds, batch_lds_floats(P[b]->m, T.shape.rows[ra::batch_class(P[b]->m)],
                                             demands));
    return lds;
}

// Autotuner of the batched launch shape.  For each tile budget (1024 floats
// only without m = 32 problems, 2048, 4096) and each m class present, one
// round of that class's problems alone is timed per tile height (64, 128,
// 256, 512 rows within the budget) at the most resident blocks; the fastest
// height gives the class's cost per job.  Then one round of the whole batch,
// its tiles split by those costs, is timed per blocks-per-CU count, and the
// budget and block count of the fastest whole round are kept.  Rounds are
// timed with HIP events (one warm-up launch, then the best of two), at the
// batch's first prices, every problem also certifying so that a round does
// a solver round's work.  The candidates and their times are recorded as
// JSON in ctx->batch_tune_log.
ra_status batch_tune(ra_ctx* ctx, BatchWs& ws, const std::vector<ra_problem*>& P,
                     const std::vector<ra::PriceLoop>& loops,
                     std::vector<std::vector<double>>& p_eval, ra::HostPool* pool,
                     const std::string& sig, ra::BatchTuned& out)
{
    const int B = (int)P.size();
    bool have[4] = {false, false, false, false};
    std::vector<int> by[4];
    int64_t jobs[4] = {0, 0, 0, 0};
    for (int b = 0; b < B; ++b) {
        const int c = ra::batch_class(P[b]->m);
        have[c] = true;
        by[c].push_back(b);
        jobs[c] += P[b]->n;
    }
    std::vector<int> all(B);
    for (int b = 0; b < B; ++b) all[b] = b;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    RA_HIP(ctx, hipEventCreate(&e0));
    RA_HIP(ctx, hipEventCreate(&e1));
    std::string log = "{\"signature\": \"" + sig + "\", \"candidates\": [";
    bool first_entry = true;
    char buf[256];
    ra_status st = RA_OK;
    // time one round of problems `act` under shape T at bpc blocks per CU
    auto time_round = [&](const std::vector<int>& act, const ra::BatchTuned& T, int bpc,
                          float& ms_out) -> ra_status {
        const int grid = ctx->cus * bpc;
        batch_fill(ws, P, loops, act, grid * 4, p_eval, pool, T, true);
        float best = INFINITY;
        for (int rep = 0; rep < 3; ++rep) {
            RA_HIP(ctx, hipEventRecord(e0, ctx->stream));
            ra_status s = batch_enqueue(ctx, ws, grid);
            if (s != RA_OK) return s;
            RA_HIP(ctx, hipEventRecord(e1, ctx->stream));
            RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
            float ms = 0.f;
            RA_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) best = std::min(best, ms);
        }
        ms_out = best;
        return RA_OK;
    };
    auto occ_of = [&](const ra::BatchTuned& T, const std::vector<int>& act) {
        const int lds = batch_lds_of(P, act, T, ws.demands);
        // a launch of more blocks than fit would queue its waves behind the
        // first ones and leave their chunks for a second pass
        return std::max(1, std::min(8, ra::batch_blocks_per_cu(T.shape.tile_floats, ws.demands,
                                                               ws.alpha_fair, lds)));
    };
    float best_all = INFINITY;
    const int tfs[3] = {1024, 2048, 4096};
    for (int tf : tfs) {
        if (tf == 1024 && have[3]) continue;
        ra::BatchTuned T;
        T.shape.tile_floats = tf;
        for (int c = 0; c < 4; ++c) {
            if (!have[c]) continue;
            float best_c = INFINITY;
            int rows_c = 64;
            for (int rows = 64; rows <= 64 * ra::BATCH_MAX_JPL; rows *= 2) {
                if (!ra::batch_rows_ok(tf, kBatchMs[c], rows)) continue;
                ra::BatchTuned Tc = T;
                Tc.shape.rows[c] = rows;
                const int occ = occ_of(Tc, by[c]);
                float ms = 0.f;
                st = time_round(by[c], Tc, occ, ms);
                if (st != RA_OK) break;
                snprintf(buf, sizeof(buf),
                         "%s{\"tile_floats\": %d, \"m\": %d, \"rows\": %d, \"bpc\": %d, "
                         "\"ms\": %.5f}",
                         first_entry ? "" : ", ", tf, kBatchMs[c], rows, occ, ms);
                log += buf;
                first_entry = false;
                if (ms < best_c) {
                    best_c = ms;
                    rows_c = rows;
                }
            }
            if (st != RA_OK) break;
            T.shape.rows[c] = rows_c;
            // a class's time per job is trusted when its round gave every
            // wave at least a job per lane; smaller rounds mostly time the
            // launch
            const int occ = occ_of(T, by[c]);
            if (jobs[c] >= (int64_t)64 * 4 * ctx->cus * occ)
                T.cost[c] = 1e6 * (double)best_c / (double)jobs[c];
        }
        if (st != RA_OK) break;
        {
            // classes without a trusted time: their bytes per job at the
            // measured classes' mean time per byte (all zero when none was
            // measured: the split then weighs bytes)
            double nspb = 0.0;
            int k = 0;
            for (int c = 0; c < 4; ++c)
                if (T.cost[c] > 0.0) {
                    nspb += T.cost[c] / (double)(4 * kBatchMs[c] + 8);
                    ++k;
                }
            for (int c = 0; c < 4; ++c)
                if (T.cost[c] <= 0.0 && k > 0) T.cost[c] = nspb / k * (double)(4 * kBatchMs[c] + 8);
        }
        const int occ = occ_of(T, all);
        for (int bpc = 1; bpc <= occ; ++bpc) {
            float ms = 0.f;
            st = time_round(all, T, bpc, ms);
            if (st != RA_OK) break;
            snprintf(buf, sizeof(buf),
                     "%s{\"tile_floats\": %d, \"m\": 0, \"rows\": [%d, %d, %d, %d], \"bpc\": %d, "
                     "\"ms\": %.5f}",
                     first_entry ? "" : ", ", tf, T.shape.rows[0], T.shape.rows[1],
                     T.shape.rows[2], T.shape.rows[3], bpc, ms);
            log += buf;
            first_entry = false;
            if (ms < best_all) {
                best_all = ms;
                out = T;
                out.shape.bpc = bpc;
            }
        }
        if (st != RA_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RA_OK) return st;
    snprintf(buf, sizeof(buf),
             "], \"chosen\": {\"tile_floats\": %d, \"rows\": [%d, %d, %d, %d], \"bpc\": %d, "
             "\"ms\": %.5f, \"cost_ns_per_job\": [%.5g, %.5g, %.5g, %.5g]}}",
             out.shape.tile_floats, out.shape.rows[0], out.shape.rows[1], out.shape.rows[2],
             out.shape.rows[3], out.shape.bpc, best_all, out.cost[0], out.cost[1], out.cost[2],
             out.cost[3]);
    log += buf;
    ctx->batch_tune_log = log;
    return RA_OK;
}

}  // namespace

extern "C" ra_status ra_batch_solve(ra_ctx* ctx, int32_t B, ra_problem* const* probs,
                                    const ra_solve_opts* opts, const double* tol_each,
                                    double* p_inout, ra_solve_info* infos)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (B < 1 || !probs || !p_inout) return fail(ctx, RA_EINVAL, "B >= 1, probs and p_inout are required");
    ra_solve_opts o;
    ra_solve_opts_default(&o);
    if (opts) o = *opts;
    if (!valid_opts(o)) return fail(ctx, RA_EINVAL, "invalid solve options");
    std::vector<ra_problem*> P(probs, probs + B);
    std::vector<size_t> off(B + 1, 0);
    for (int b = 0; b < B; ++b) {
        if (!P[b] || P[b]->ctx != ctx)
            return fail(ctx, RA_EINVAL, "problem %d is NULL or from another context", b);
        const int m = P[b]->m;
        if (P[b]->dt != 0 || !P[b]->vec_ok || !(m == 4 || m == 8 || m == 16 || m == 32))
            return fail(ctx, RA_EUNSUPPORTED,
                        "problem %d: the batched kernel takes FP32, 16-byte aligned T with m in "
                        "{4, 8, 16, 32}", b);
        if (P[b]->dvec)
            return fail(ctx, RA_EUNSUPPORTED,
                        "problem %d: demand vectors are not supported by the batched kernel "
                        "(use ra_solve)", b);
        if (P[b]->n > ((int64_t)1 << 36))
            return fail(ctx, RA_EUNSUPPORTED, "problem %d too large for the batched kernel", b);
        if (tol_each && !(tol_each[b] >= 0.0))
            return fail(ctx, RA_EINVAL, "tol_each[%d] must be >= 0", b);
        off[b + 1] = off[b] + m;
    }
    bool have[4] = {false, false, false, false};
    int64_t total_rows = 0;
    for (int b = 0; b < B; ++b) {
        have[ra::batch_class(P[b]->m)] = true;
        total_rows += P[b]->n + 63;
    }
    if (ctx->batch_fixed && !shape_fits(ctx->batch_fixed_shape.shape, have))
        return fail(ctx, RA_EINVAL,
                    "the launch shape fixed by ra_batch_set_shape has no valid tile for an m "
                    "class of this batch");
    // tiles have at least 64 rows
    if (total_rows / 64 >= ((int64_t)1 << 31))
        return fail(ctx, RA_EUNSUPPORTED, "batch has too many tiles");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    const auto t0 = std::chrono::steady_clock::now();

    std::vector<ra::PriceLoop> loops;
    loops.reserve(B);
    for (int b = 0; b < B; ++b) {
        ra_solve_opts ob = o;
        if (tol_each) ob.tol_rel = tol_each[b];
        std::vector<double> p0(P[b]->m, 1.0);
        if (o.init == 1)
            for (int j = 0; j < P[b]->m; ++j) {
                const double v = p_inout[off[b] + j];
                if (!std::isfinite(v) || v < 0.0)
                    return fail(ctx, RA_EINVAL, "p_inout of problem %d must be >= 0 and finite", b);
                p0[j] = v;
            }
        if (o.init == 2) {
            ra_status st = init_prices(P[b], p0.data());
            if (st != RA_OK) return st;
        }
        loops.emplace_back(P[b]->m, P[b]->n, P[b]->R.data(), ob, p0.data());
    }

    // enough waves for any launch shape (at most 8 blocks of 4 waves per CU);
    // the workspace (device tables, partial slots, pinned results, captured
    // graph) stays with the context for later batches of at most its size
    // Batches of kBatchGroupsMin problems or more run as two groups whose
    // rounds alternate on the stream, each with a workspace of its own: while
    // the GPU runs one group's round, the host takes the other group's
    // results, steps its price loops and queues its next round, so that the
    // host's work and the launch latency hide behind the other group's
    // kernels.  These rounds are launched directly with compact tables.  A
    // smaller batch is one group, replayed from a captured graph.
    const int Wmax = ctx->cus * 8 * 4;
    const int NG = B >= kBatchGroupsMin ? 2 : 1;
    BatchWs* wss[2] = {nullptr, nullptr};
    for (int g = 0; g < NG; ++g) {
        std::shared_ptr<void>& slot = g == 0 ? ctx->batch_ws : ctx->batch_ws2;
        BatchWs* wsp = static_cast<BatchWs*>(slot.get());
        if (!wsp || wsp->B < B || wsp->Wmax != Wmax) {
            slot.reset();
            std::shared_ptr<BatchWs> nw = std::make_shared<BatchWs>();
            if (batch_alloc(ctx, *nw, B, Wmax) != RA_OK) return RA_ENOMEM;
            slot = nw;
            wsp = nw.get();
        }
        wss[g] = wsp;
    }
    BatchWs& ws = *wss[0];
    ws.demands = false;
    ws.alpha_fair = false;
    for (int b = 0; b < B; ++b) {
        ws.demands = ws.demands || P[b]->dem != nullptr;
        ws.alpha_fair = ws.alpha_fair || P[b]->alpha_fair;
    }
    const bool graph = NG == 1 && o.use_graph && ctx->stream != nullptr;
    ws.compact = !graph;
    if (NG == 2) {
        wss[1]->demands = ws.demands;
        wss[1]->alpha_fair = ws.alpha_fair;
        wss[1]->compact = true;
    }

    // host threads for the per-problem work between rounds (created once per
    // context, for batches large enough to use them)
    if (B >= 64 && !ctx->pool) {
        const int hw = (int)std::thread::hardware_concurrency();
        const int workers = std::min(hw, 16) - 1;
        if (workers >= 1) {
            try {
                ctx->pool.reset(new ra::HostPool(workers));
            } catch (...) {  // no threads: the work stays on this thread
                ctx->pool.reset();
            }
        }
    }
    ra::HostPool* pool = ctx->pool.get();
    std::vector<char> bad;

    // launch shape: fixed by the caller, cached for this batch signature, or
    // tuned now (timing candidate rounds at the first prices)
    std::vector<std::vector<double>> p_eval(B);
    ra::BatchTuned tuned;
    if (ctx->batch_fixed) {
        tuned = ctx->batch_fixed_shape;
    } else {
        if (ctx->batch_tuned.empty()) tune_cache_load(ctx);
        const std::string sig = batch_signature(P, ws.demands, ws.alpha_fair);
        auto found = ctx->batch_tuned.find(sig);
        if (found != ctx->batch_tuned.end() && shape_fits(found->second.shape, have)) {
            tuned = found->second;
        } else {
            ra_status s = batch_tune(ctx, ws, P, loops, p_eval, pool, sig, tuned);
            if (s != RA_OK) return s;
            ctx->batch_tuned[sig] = tuned;
            tune_cache_store(ctx);
        }
    }
    int bpc = tuned.shape.bpc;
    {
        std::vector<int> all(B);
        for (int b = 0; b < B; ++b) all[b] = b;
        const int lds = batch_lds_of(P, all, tuned, ws.demands);
        const int occ = std::max(1, std::min(8, ra::batch_blocks_per_cu(tuned.shape.tile_floats,
                                                                        ws.demands,
                                                                        ws.alpha_fair, lds)));
        bpc = bpc >= 1 ? std::min(bpc, occ) : occ;
    }
    const int grid = ctx->cus * bpc;

    // the groups: problems by their work in a round (jobs times the tuned
    // cost per job of their m class, else 4 m + 8 bytes per job), dealt
    // 0 1 1 0 0 1 ... so that both groups get about half of it; each
    // group's members ascending
    std::vector<int> members[2];
    {
        std::vector<double> work(B);
        for (int b = 0; b < B; ++b) {
            const int c = ra::batch_class(P[b]->m);
            work[b] = (double)P[b]->n *
                      (tuned.cost[c] > 0.0 ? tuned.cost[c] : (double)(4 * P[b]->m + 8));
        }
        std::vector<int> order(B);
        for (int b = 0; b < B; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return work[x] > work[y]; });
        for (int k = 0; k < B; ++k) members[NG == 2 ? ((k + 1) >> 1) & 1 : 0].push_back(order[k]);
        for (int g = 0; g < NG; ++g) std::sort(members[g].begin(), members[g].end());
    }
    std::vector<int> gact[2];
    std::vector<std::vector<double>> gp_eval[2];
    bool queued[2] = {false, false};
    for (int g = 0; g < NG; ++g) gp_eval[g].resize(members[g].size());
    // fill and queue group g's next round, if it has active problems
    auto queue_round = [&](int g) -> ra_status {
        std::vector<int>& A = gact[g];
        A.clear();
        for (int b : members[g])
            if (!loops[b].done()) A.push_back(b);
        queued[g] = !A.empty();
        if (!queued[g]) return RA_OK;
        batch_fill(*wss[g], P, loops, A, grid * 4, gp_eval[g], pool, tuned);
        return batch_launch(ctx, *wss[g], grid, graph);
    };
    // wait for group g's round and step the price loop of each of its
    // problems (independent per problem); a non-finite dual value is
    // reported for the first such problem after all have been visited
    auto take_round = [&](int g) -> ra_status {
        BatchWs& wg = *wss[g];
        ra_status s = ra::wait_flag(ctx, wg.hflag);
        if (s != RA_OK) return s;
        const std::vector<int>& A = gact[g];
        const int nA = (int)A.size();
        bad.assign(nA, 0);
        for_problems(pool, nA, [&](int lo, int hi) {
            double rr[ra::BATCH_MAX_M];
            for (int a = lo; a < hi; ++a) {
                const int b = A[a];
                const ra_problem* Pb = P[b];
                const double* row = wg.hout + (size_t)a * ra::BATCH_COLS;
                double pR = 0.0;
                for (int j = 0; j < Pb->m; ++j) pR += gp_eval[g][a][j] * Pb->R[j];
                const double gv = pR + row[ra::BATCH_MAX_M];
                if (!std::isfinite(gv)) {
                    bad[a] = 1;
                    continue;
                }
                for (int j = 0; j < Pb->m; ++j) rr[j] = row[j];
                loops[b].feed(gp_eval[g][a], gv, rr, row[ra::BATCH_MAX_M + 2]);
            }
        });
        for (int a = 0; a < nA; ++a)
            if (bad[a]) return fail(ctx, RA_ENUMERIC, "problem %d: non-finite dual value", A[a]);
        return RA_OK;
    };
    {
        ra_status s = RA_OK;
        for (int g = 0; g < NG && s == RA_OK; ++g) s = queue_round(g);
        while (s == RA_OK && (queued[0] || queued[1])) {
            for (int g = 0; g < NG && s == RA_OK; ++g) {
                if (!queued[g]) continue;
                s = take_round(g);
                if (s == RA_OK) s = queue_round(g);
            }
        }
        if (s != RA_OK) {
            // a round of the other group may still be queued: let it finish
            // before the workspaces are touched again
            (void)hipStreamSynchronize(ctx->stream);
            return s;
        }
    }
    // the last reduction may still be retiring after its flag
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    for (int b = 0; b < B; ++b) {
        const ra::Point& ret = loops[b].result();
        for (int j = 0; j < P[b]->m; ++j) p_inout[off[b] + j] = ret.p[j];
        all = all && loops[b].converged();
        if (infos) {
            infos[b].iters = loops[b].iters();
            infos[b].dual_evals = loops[b].evals();
            infos[b].fell_back = loops[b].fallbacks();
            infos[b].converged = loops[b].converged() ? 1 : 0;
            infos[b].g = ret.g;
            infos[b].U_lb = ret.certified ? ret.U : NAN;
            infos[b].rel_gap = ret.certified ? ret.rel : INFINITY;
            infos[b].seconds = secs;
            infos[b].restarted = 0;
            infos[b].warm_evals = 0;
        }
    }
    return all ? RA_OK : RA_ENOTCONV;
}

extern "C" ra_status ra_batch_set_shape(ra_ctx* ctx, int32_t tile_floats, const int32_t* rows,
                                        int32_t blocks_per_cu)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (tile_floats == 0) {
        ctx->batch_fixed = false;
        return RA_OK;
    }
    if (tile_floats != 1024 && tile_floats != 2048 && tile_floats != 4096)
        return fail(ctx, RA_EINVAL, "tile_floats must be 0, 1024, 2048 or 4096");
    if (!rows) return fail(ctx, RA_EINVAL, "rows is required");
    if (blocks_per_cu < 0 || blocks_per_cu > 8)
        return fail(ctx, RA_EINVAL, "blocks_per_cu must be in [0, 8]");
    ra::BatchTuned t;
    t.shape.tile_floats = tile_floats;
    for (int c = 0; c < 4; ++c) {
        const int m = 4 << c;
        if (rows[c] != 0 && !ra::batch_rows_ok(tile_floats, m, rows[c]))
            return fail(ctx, RA_EINVAL,
                        "rows[%d] = %d: a tile of m = %d needs a multiple of 64 rows, at most "
                        "%d, with rows * m <= tile_floats (or 0: no such problems)",
                        c, rows[c], m, 64 * ra::BATCH_MAX_JPL);
        t.shape.rows[c] = rows[c];
    }
    t.shape.bpc = blocks_per_cu;
    ctx->batch_fixed_shape = t;
    ctx->batch_fixed = true;
    return RA_OK;
}

extern "C" ra_status ra_batch_tuning(const ra_ctx* ctx, char* buf, size_t cap, size_t* len)
{
    if (!ctx) return RA_EINVAL;
    const std::string& s = ctx->batch_tune_log;
    if (len) *len = s.size();
    if (!buf) return RA_OK;
    if (cap < s.size() + 1) return RA_EINVAL;
    std::memcpy(buf, s.c_str(), s.size() + 1);
    return RA_OK;
}
