// One step of the price-discovery loop on the device (§5, Algorithm 2): one
// wave, lane j holding coordinate j.  It reads the column sums of the pass
// that just ran (usage r, the sum of net utilities, the utility lost by
// scaling the previous point's allocation), certifies the previous point,
// updates the projected L-BFGS state exactly as the host loop does
// (price_loop.hpp) and writes the prices of the next pass.  Dot products are
// wave reductions, so their rounding order differs from the host's
// sequential sums.  The step runs in the kernel that reduces the pass's
// column sums, on a copy of the state in LDS.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>

#include "colsum.hpp"
#include "dev_loop.hpp"
#include "ra_kernels.h"

namespace ra {
namespace {

// Wave-wide reductions for the one-wave step (all 64 lanes active): data
// movement within rows of 16 lanes by DPP (xor 1, xor 2, half-row mirror,
// row mirror), then the four row results read from lanes 0, 16, 32, 48 and
// combined in the same order on every lane.
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp((int)u, (int)u, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(u >> 32), (int)(u >> 32), CTRL, 0xf, 0xf,
                                               false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double lane_value(double v, int lane)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)u, lane);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

constexpr int DPP_XOR1 = 0xb1;        // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4e;        // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;

__device__ __forceinline__ double wsum(double v)
{
    v += dpp<DPP_XOR1>(v);
    v += dpp<DPP_XOR2>(v);
    v += dpp<DPP_HALF_MIRROR>(v);
    v += dpp<DPP_MIRROR>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

__device__ __forceinline__ double wmax(double v)
{
    v = fmax(v, dpp<DPP_XOR1>(v));
    v = fmax(v, dpp<DPP_XOR2>(v));
    v = fmax(v, dpp<DPP_HALF_MIRROR>(v));
    v = fmax(v, dpp<DPP_MIRROR>(v));
    return fmax(fmax(lane_value(v, 0), lane_value(v, 16)),
                fmax(lane_value(v, 32), lane_value(v, 48)));
}

__device__ __forceinline__ bool wany(bool b) { return __any(b); }

// The step's view of the state: lane j's coordinate of every vector, the
// scalars in the shared DevLoop record (every lane writes the same value).
struct Step {
    DevLoop* L;
    int j;
    bool on;

    __device__ double dot(const double* a, const double* b) const
    {
        return wsum(on ? a[j] * b[j] : 0.0);
    }
    __device__ double inf_norm(const double* a) const { return wmax(on ? fabs(a[j]) : 0.0); }
    __device__ bool budget_left() const { return L->max_evals == 0 || L->evals < L->max_evals; }

    __device__ void copy_point(DevPoint& dst, const DevPoint& src) const
    {
        if (on) {
            dst.p[j] = src.p[j];
            dst.r[j] = src.r[j];
            dst.grad[j] = src.grad[j];
        }
        dst.g = src.g;
        dst.f = src.f;
        dst.U = src.U;
        dst.gap = src.gap;
        dst.rel = src.rel;
        dst.certified = src.certified;
    }

    __device__ bool met(const DevPoint& e) const
    {
        return e.rel <= L->tol_rel || (L->tol_abs > 0.0 && e.gap <= L->tol_abs);
    }

    __device__ void go_final()
    {
        if (L->have_pend && !L->pend.certified && budget_left()) {
            if (on) L->next[j] = L->pend.p[j];
            L->state = 3;
        } else {
            L->state = 4;
        }
    }

    __device__ void next_line_search_point()
    {
        if (!budget_left()) {
            go_final();
            return;
        }
        if (on) L->next[j] = fmax(L->cur.p[j] + L->lam * L->d[j], 0.0);
    }

    __device__ void start_subgradient()
    {
        if (!budget_left()) {
            go_final();
            return;
        }
        L->sg_steps += 1;
        L->fallbacks += 1;
        const double gi = inf_norm(L->cur.grad), pi = inf_norm(L->cur.p);
        const double a0 = gi > 0.0 ? 0.1 * (pi > 0.0 ? pi : 1.0) / gi : 0.0;
        const double ak = a0 / sqrt((double)L->sg_steps);
        if (on) L->next[j] = fmax(L->cur.p[j] - ak * L->cur.grad[j], 0.0);
        L->state = 2;
    }

    __device__ void start_iteration()
    {
        if (L->iters >= L->max_iter || !budget_left()) {
            go_final();
            return;
        }
        if (L->method == 1) {
            start_subgradient();
            return;
        }
        const int M = L->mem;
        const int np = L->npairs;
        double q = on ? L->cur.grad[j] : 0.0;
        for (int h = 0; h < np; ++h) {
            const int s = (L->head - 1 - h + M) % M;
            const double a = L->rho[s] * wsum(on ? L->S[s][j] * q : 0.0);
            L->alpha[h] = a;
            if (on) q -= a * L->Y[s][j];
        }
        if (np > 0) {
            const int s = (L->head - 1 + M) % M;
            const double gam = dot(L->S[s], L->Y[s]) / dot(L->Y[s], L->Y[s]);
            q *= gam;
        }
        for (int h = np - 1; h >= 0; --h) {
            const int s = (L->head - 1 - h + M) % M;
            const double b = L->rho[s] * wsum(on ? L->Y[s][j] * q : 0.0);
            if (on) q += L->S[s][j] * (L->alpha[h] - b);
        }
        const double pj = on ? L->cur.p[j] : 0.0;
        const double gj = on ? L->cur.grad[j] : 0.0;
        double dj = (pj <= 0.0 && q > 0.0) ? 0.0 : -q;
        if (wsum(on ? dj * gj : 0.0) >= 0.0) {
            L->npairs = 0;
            dj = (pj <= 0.0 && gj > 0.0) ? 0.0 : -gj;
        }
        if (on) L->d[j] = dj;
        const double dn = wmax(on ? fabs(dj) : 0.0);
        if (dn == 0.0) {
            go_final();
            return;
        }
        double lam = 1.0;
        if (L->npairs == 0) {
            const double pi = inf_norm(L->cur.p);
            const double s0 = L->init_step > 0.0 ? L->init_step : 0.1;
            lam = s0 * (pi > 0.0 ? pi : 1.0) / dn;
        }
        L->lam = lam;
        L->ls = 0;
        L->state = 1;
        next_line_search_point();
    }

    // The host loop's feed() for the pass just completed: certify the
    // pending point with the pass's sum of utility lost by scaling, then
    // take the evaluated point into the L-BFGS state machine.
    __device__ void feed(double g, double rj, double sdu)
    {
        bool restart = false;
        if (L->have_pend && !L->pend.certified) {
            DevPoint& e = L->pend;
            const double pq = wsum(on ? e.p[j] * (L->R[j] - e.r[j]) : 0.0);
            e.gap = pq + sdu;
            e.U = e.g - e.gap;
            const double den = fmax(fabs(e.g), fabs(e.U));
            e.rel = e.gap / (den > 0.0 ? den : 1.0);
            e.certified = 1;
            L->ncert += 1;
            if (!L->best.certified || e.rel < L->best.rel) {
                if (!L->best.certified || e.rel < 0.999 * L->best.rel) L->improved_at = L->evals;
                copy_point(L->best, e);
            }
            if (met(e)) {
                L->state = 4;
                return;
            }
            if (L->stall_evals > 0 && L->evals - L->improved_at >= L->stall_evals) {
                if (L->restarts < L->stall_restarts && (L->state == 1 || L->state == 2)) {
                    L->restarts += 1;  // restart from the best point once e is taken in
                    restart = true;
                } else {
                    L->stalled = 1;
                    L->state = 4;
                    return;
                }
            }
        }
        // the evaluated point
        const double nn = L->n;
        DevPoint& e = L->pend;
        if (on) {
            e.p[j] = L->pe[j];
            e.r[j] = rj;
            e.grad[j] = (L->R[j] - rj) / nn;
        }
        e.g = g;
        e.f = g / nn;
        e.certified = 0;
        e.U = 0.0;
        e.gap = 0.0;
        e.rel = INFINITY;
        L->evals += 1;
        L->have_pend = 1;
        const int was = L->state;
        if (restart) {
            // a new window from the best certified point (the point just
            // evaluated is still certified by the next pass)
            L->improved_at = L->evals;
            copy_point(L->cur, L->best);
            L->npairs = 0;
            start_iteration();
            return;
        }
        if (was == 0) {
            copy_point(L->cur, e);
            start_iteration();
        } else if (was == 1) {
            const double step = on ? e.p[j] - L->cur.p[j] : 0.0;
            const double dec = wsum(on ? L->cur.grad[j] * step : 0.0);
            if (e.f <= L->cur.f + 1e-4 * dec) {
                const double y = on ? e.grad[j] - L->cur.grad[j] : 0.0;
                const double sy = wsum(step * y);
                const double ss = wsum(step * step), yy = wsum(y * y);
                if (sy > 1e-12 * sqrt(ss * yy)) {
                    const int M = L->mem;
                    const int h = L->head;
                    if (on) {
                        L->S[h][j] = step;
                        L->Y[h][j] = y;
                    }
                    L->rho[h] = 1.0 / sy;
                    L->head = (h + 1) % M;
                    L->npairs = L->npairs + 1 < M ? L->npairs + 1 : M;
                }
                copy_point(L->cur, e);
                L->iters += 1;
                start_iteration();
            } else {
                L->lam *= 0.5;
                L->ls += 1;
                if (L->ls >= 20) {
                    L->npairs = 0;
                    start_subgradient();
                } else {
                    next_line_search_point();
                }
            }
        } else if (was == 2) {
            copy_point(L->cur, e);
            L->iters += 1;
            start_iteration();
        } else {
            L->state = 4;
        }
    }
};

// The step after a pass, taken by one wave on the state staged in LDS.
template <int M>
__device__ __forceinline__ void loop_step(DevLoop* L, const double* __restrict__ out,
                                          PriceArgs<M>* __restrict__ pa,
                                          DevStatus* __restrict__ hs)
{
    // a new solve must not see the previous solve's best point (the working
    // state is not part of the header the host writes)
    if (L->state == 0) L->best.certified = 0;
    Step S{L, (int)threadIdx.x, (int)threadIdx.x < M};
    const int j = S.j;
    const bool on = S.on;
    const double rj = on ? out[j] : 0.0;
    const double g = L->pR + out[M];
    const double sdu = out[M + 2];
    const bool had_prev = L->have_pend && !L->pend.certified;
    const bool bad =
        !isfinite(g) || wany(on && !isfinite(rj)) || (had_prev && !isfinite(sdu));
    if (!bad) S.feed(g, rj, sdu);
    if (bad || L->state == 4) {
        // the outcome: the certified point with the smallest gap, else the
        // last point evaluated
        const DevPoint& res = L->best.certified ? L->best : L->pend;
        L->converged = !bad && L->best.certified && S.met(L->best);
        L->error = bad ? 1 : 0;
        L->done = 1;
        if (on) hs->p[j] = res.p[j];
        if (j == 0) {
            hs->g = res.g;
            hs->U = res.U;
            hs->rel = res.rel;
            hs->certified = res.certified;
            hs->iters = L->iters;
            hs->evals = L->evals;
            hs->fallbacks = L->fallbacks;
            hs->converged = L->converged;
        }
        __threadfence_system();
        if (j == 0)
            __hip_atomic_store(&hs->done, bad ? 2 : 1, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
        return;
    }
    if (j == 0)
        __hip_atomic_store(&hs->passes, L->evals, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    // the prices of the next pass, rounded to FP32 as the host does, and the
    // previous point (still uncertified) whose lower bound that pass forms
    const float pf = on ? (float)L->next[j] : 0.f;
    if (on) {
        L->pe[j] = (double)pf;
        pa->p[j] = pf;
        pa->invp[j] = pf > 0.f ? 1.0f / pf : INFINITY;
    }
    L->pR = wsum(on ? (double)pf * L->R[j] : 0.0);
    const bool prev = L->have_pend && !L->pend.certified;
    if (on) {
        const float qf = prev ? (float)L->pend.p[j] : 0.f;
        pa->q[j] = qf;
        pa->invq[j] = qf > 0.f ? 1.0f / qf : INFINITY;
        const double rr = prev ? L->pend.r[j] : 0.0;
        const bool over = prev && rr > L->R[j];
        pa->s[j] = over ? (float)(L->R[j] / rr) : 1.f;
        pa->sc[j] = over ? (float)((rr - L->R[j]) / rr) : 0.f;
    }
    pa->has_prev = prev ? 1 : 0;
}

// Copies the parts of the state a step reads or writes (everything before
// the L-BFGS pairs, the first mem pairs, rho and alpha) in 8-byte words, by
// a block of 256 threads: every load is issued before the first store.
constexpr int ST_HEAD = (int)(offsetof(DevLoop, S) / 8);
constexpr int ST_Y = (int)(offsetof(DevLoop, Y) / 8);
constexpr int ST_RHO = (int)(offsetof(DevLoop, rho) / 8);
constexpr int ST_MAX = ST_HEAD + 2 * DL_MAX_MEM * DL_MAX_M + 2 * DL_MAX_MEM;
constexpr int ST_PER = (ST_MAX + 255) / 256;
static_assert(offsetof(DevLoop, alpha) == offsetof(DevLoop, rho) + 8 * DL_MAX_MEM,
              "rho and alpha must be adjacent");

__device__ __forceinline__ int stage_word(int k, int rows)
{
    if (k < ST_HEAD + rows) return k;  // the head, then the S rows
    if (k < ST_HEAD + 2 * rows) return ST_Y + (k - ST_HEAD - rows);
    return ST_RHO + (k - ST_HEAD - 2 * rows);
}

__device__ __forceinline__ void stage(double* __restrict__ dst, const double* __restrict__ src,
                                      int mem)
{
    const int rows = mem * DL_MAX_M;
    const int total = ST_HEAD + 2 * rows + 2 * DL_MAX_MEM;
    double v[ST_PER];
#pragma unroll
    for (int i = 0; i < ST_PER; ++i) {
        const int k = threadIdx.x + 256 * i;
        if (k < total) v[i] = src[stage_word(k, rows)];
    }
#pragma unroll
    for (int i = 0; i < ST_PER; ++i) {
        const int k = threadIdx.x + 256 * i;
        if (k < total) dst[stage_word(k, rows)] = v[i];
    }
}

// Column sums of a dual pass (block b of the grid reduces column b, in the
// fixed order of the plain column reduction), then the last block to finish
// stages the loop state in LDS and its first wave takes the step.
template <int M>
__global__ void __launch_bounds__(256) k_reduce_step(const double* __restrict__ partial, int nb,
                                                     DevLoop* __restrict__ L,
                                                     double* __restrict__ out,
                                                     PriceArgs<M>* __restrict__ pa,
                                                     DevStatus* __restrict__ hs)
{
    if (L->done) return;  // the loop has ended: a spare pass of the last replay
    __shared__ double red[256];
    __shared__ int last;
    __shared__ DevLoop sl;
    const int j = blockIdx.x;
    const double s = column_sum(partial, nb, M + 3, j, red);
    if (threadIdx.x == 0) {
        out[j] = s;
        __threadfence();
        last = atomicAdd(&L->ticket, 1u) == gridDim.x - 1u;
        if (last) atomicExch(&L->ticket, 0u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // every block's column is visible past this point
    const int mem = min(max(L->mem, 1), DL_MAX_MEM);
    stage(reinterpret_cast<double*>(&sl), reinterpret_cast<const double*>(L), mem);
    __syncthreads();
    if (threadIdx.x < 64) loop_step<M>(&sl, out, pa, hs);
    __syncthreads();
    stage(reinterpret_cast<double*>(L), reinterpret_cast<const double*>(&sl), mem);
}

}  // namespace

hipError_t launch_reduce_step(int m, hipStream_t st, const double* partial, int nb, DevLoop* L,
                              double* out, void* pa, DevStatus* hs)
{
    const dim3 g(m + 3);
    switch (m) {
    case 4: k_reduce_step<4><<<g, 256, 0, st>>>(partial, nb, L, out, static_cast<PriceArgs<4>*>(pa), hs); break;
    case 8: k_reduce_step<8><<<g, 256, 0, st>>>(partial, nb, L, out, static_cast<PriceArgs<8>*>(pa), hs); break;
    case 16: k_reduce_step<16><<<g, 256, 0, st>>>(partial, nb, L, out, static_cast<PriceArgs<16>*>(pa), hs); break;
    case 32: k_reduce_step<32><<<g, 256, 0, st>>>(partial, nb, L, out, static_cast<PriceArgs<32>*>(pa), hs); break;
    case 64: k_reduce_step<64><<<g, 256, 0, st>>>(partial, nb, L, out, static_cast<PriceArgs<64>*>(pa), hs); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace ra
