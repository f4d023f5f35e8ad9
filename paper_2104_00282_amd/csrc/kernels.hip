// gfx950 kernels of the price-discovery hot path.
//
// Per job i (row a = a_i of the efficiency matrix T, prices p), the kernels
// solve the subproblem of §3 (eq. e-subprob): maximise u(t) - p^T x over
// x >= 0, 1^T x <= 1, t = a^T x.  §4.1 shows the cost c(t) of reaching
// throughput t is the lower convex envelope of the points (0, 0) and
// (a_j, p_j); §4.2 maximises u(t) - c(t) one envelope segment at a time with
// the closed forms eq. e-opt-t-log (log utility) and eq. e-opt-t-target
// (capped-linear utility), and the allocation on a segment is eq. e-xixj.
//
// Instead of building all m(m+1)/2 segments (Algorithm 1), a job walks the
// envelope from the origin: the first vertex is the resource with the
// largest a_j / p_j, each further vertex the one with the smallest slope
// (p_j - p_c) / (a_j - a_c) among a_j > a_c.  Since u - c is concave, the
// walk stops at the first segment whose maximiser lies before its right end.
// It visits only the segments up to the optimum and costs one pass over the
// row per visited vertex.
//
// Layout: T is n x m row-major in HBM.  A wavefront owns a tile of 64
// consecutive jobs (64 m contiguous elements) and loads it with 16-byte
// loads that each cover 1 KiB of consecutive bytes, stages it in LDS with a
// padded row stride (conflict-free 16-byte row reads), and each lane then
// solves one job from its own row.  The next tile is prefetched into
// registers (non-temporal loads) while the current one is solved.  Resource usage r_j is summed
// per tile in a per-wave LDS histogram, folded into per-lane FP64
// accumulators after every tile, reduced across the block in a fixed order
// and written as one row of block partials; no global atomics are used, so
// results are reproducible bit for bit.
#include "colsum.hpp"
#include "ra_kernels.h"

#include <math.h>

#include <algorithm>

namespace ra {

template <typename F> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename F> using V2 = typename Vec2<F>::type;

// FP32: the hardware base-2 logarithm times ln 2 (about 1 ulp of log2 x);
// FP64: the device library.
__device__ __forceinline__ float dlog(float x)
{
    return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
}
__device__ __forceinline__ double dlog(double x) { return log(x); }
// 1/x: FP32 with the hardware reciprocal (about 1 ulp), FP64 exactly rounded.
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
// x^y for x >= 0 and y != 0 (every use here: a base t + eps or w / alpha,
// an exponent 1 - a or 1 / a), as 2^(y log2 x) with the hardware's base-2
// logarithm and exponential: relative error about (|y log2 x| + 1) 2^-23,
// below 3e-6 for the magnitudes met here, at a fraction of powf's cost.
__device__ __forceinline__ float dpow(float x, float y)
{
    return __builtin_amdgcn_exp2f(y * __builtin_amdgcn_logf(x));
}
__device__ __forceinline__ double dpow(double x, double y) { return pow(x, y); }
// e^x - 1, FP32: a degree-5 Taylor polynomial for |x| < 1/32 (truncation
// below 2e-10 relative), else the hardware base-2 exponential minus one
// (relative error below 1e-5 where |e^x - 1| >= 0.03).  FP64: the library.
__device__ __forceinline__ float dexpm1(float x)
{
    const float poly =
        x * (1.f + x * (0.5f + x * (1.f / 6.f + x * (1.f / 24.f + x * (1.f / 120.f)))));
    const float big = __builtin_amdgcn_exp2f(x * 1.44269504088896341f) - 1.f;
    return fabsf(x) < 0.03125f ? poly : big;
}
__device__ __forceinline__ double dexpm1(double x) { return expm1(x); }

// Packed utility code c of a job (second field of prm), told apart by its
// sign bit: clear (c >= +0) capped linear w min(t, c) (the target-priority
// utility plus a constant); set: the alpha-fair family of §2.2 with exponent
// a = -c, kept at full precision: c = -1 (a = 1) is the log utility
// w log(t + eps), any other a gives w (t + eps)^(1 - a) / (1 - a) (c = -0,
// a = 0: linear).
template <typename F>
__device__ __forceinline__ bool is_capped(F c) { return !__builtin_signbit(c); }
template <typename F>
__device__ __forceinline__ F afair_exponent(F c) { return -c; }

// u(t) of §2.2: log utility w log(t + eps) or capped linear w min(t, c).
// AF = false compiles the alpha-fair branches out (for problems without such jobs).
template <typename F, bool AF = true>
__device__ __forceinline__ F utility(bool caplin, F w, F c, F eps, F t)
{
    if (caplin) return w * (t < c ? t : c);
    if (!AF || c == F(-1)) return w * dlog(t + eps);
    const F e = F(1) - afair_exponent(c);
    return w * dpow(t + eps, e) * frcp(e);
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename F>
struct Job {
    int jlo, jhi, j1;  // support (-1 = none) and first envelope vertex
    F xlo, xhi;        // allocation on jlo / jhi
    F tlo, thi;        // a_jlo x_lo and a_jhi x_hi
    F v;               // net utility u(t) - p^T x
};

// The prices one job pays per unit of each resource.  SharedPrices: the price
// vector p, alike for every job; P and IP (= 1/p) are read with wave-uniform
// indices in unrolled scans, Pdyn with a per-lane index.
template <typename F>
struct SharedPrices {
    const F* __restrict__ P;
    const F* __restrict__ IP;
    const F* Pdyn;
    __device__ __forceinline__ F get(int j) const { return P[j]; }
    __device__ __forceinline__ F inv(int j) const { return IP[j]; }
    __device__ __forceinline__ F at(int j) const { return Pdyn[j]; }
};

// The prices of a kernel argument block (vectorised kernels): wave-uniform
// scalar reads from the argument segment (PREV: the previous prices q),
// per-lane reads from a copy in LDS.
template <int M>
using ArgPtr = const __attribute__((address_space(4))) PriceArgs<M>*;

template <int M, bool PREV>
struct ArgPrices {
    ArgPtr<M> a;
    const float* tab;
    __device__ __forceinline__ float get(int j) const { return PREV ? a->q[j] : a->p[j]; }
    __device__ __forceinline__ float inv(int j) const { return PREV ? a->invq[j] : a->invp[j]; }
    __device__ __forceinline__ float at(int j) const { return tab[j]; }
};

// A job with a demand vector d (§7, extensions) pays d_j p_j per unit of x_j:
// the base prices B scaled by the job's demands, read by D as Row reads its
// throughputs.
template <typename F, class B, class D>
struct DemandPrices {
    B b;
    D d;
    __device__ __forceinline__ F get(int j) const { return b.get(j) * d.get(j); }
    __device__ __forceinline__ F inv(int j) const { return b.inv(j) * frcp(d.get(j)); }
    __device__ __forceinline__ F at(int j) const { return b.at(j) * d.at(j); }
};

// First envelope vertex (§4.1): the largest key a_j * (1/p_j); a_j = 0 never
// wins (key 0, or NaN when p_j = 0); equal finite keys go to the lowest j.
// FREE (some price is zero): every free resource with a_j > 0 has key +inf,
// and of those the one with the largest a_j (then the lowest j) is the
// vertex: the cost is zero up to the farthest free point, so the nearer free
// points lie inside an envelope segment.  Taking the first of them instead
// would make the walk step through every free resource in turn.
template <typename F, int M, bool FREE, class Row, class Px>
__device__ __forceinline__ int scan_first(const Row& a, int mm, const Px& px)
{
    F best = F(0), abest = F(0);
    int j1 = -1;
    auto step = [&](int j) {
        const F aj = a.get(j);
        const F key = aj * px.inv(j);
        bool b = key > best;
        if constexpr (FREE) b = b | ((key == best) & (key == F(INFINITY)) & (aj > abest));
        best = b ? key : best;
        if constexpr (FREE) abest = b ? aj : abest;
        j1 = b ? j : j1;
    };
    if constexpr (M > 0) {
#pragma unroll
        for (int j = 0; j < M; ++j) step(j);
    } else {
        for (int j = 0; j < mm; ++j) step(j);
    }
    return j1;
}

// Next envelope vertex after (ac, pc): smallest slope (p_j - pc)/(a_j - ac)
// over a_j > ac, compared by cross-multiplication; lowest j on ties; -1 if
// no resource is more efficient than the current vertex.  The cost curve is
// nondecreasing, so every point right of an envelope vertex costs at least
// as much (p_j >= pc where a_j > ac); the price difference is clamped at 0,
// which also makes the comparison false for every a_j <= ac (its left side
// is >= 0, its right side <= 0) without a second test.
template <typename F, int M, class Row, class Px>
__device__ __forceinline__ int scan_next(const Row& a, int mm, const Px& px, F ac, F pc)
{
    F bn = F(1), bd = F(0);
    int jn = -1;
    auto step = [&](int j) {
        const F d = a.get(j) - ac;
        const F nm = fmax(px.get(j) - pc, F(0));
        const bool b = nm * bd < bn * d;
        bn = b ? nm : bn;
        bd = b ? d : bd;
        jn = b ? j : jn;
    };
    if constexpr (M > 0) {
#pragma unroll
        for (int j = 0; j < M; ++j) step(j);
    } else {
        for (int j = 0; j < mm; ++j) step(j);
    }
    return jn;
}

// Next envelope vertex after a free vertex (ac, 0): the smallest slope
// p_j / (a_j - ac) over a_j > ac is the largest key (a_j - ac) * (1/p_j),
// one subtraction and one product per entry instead of scan_next's
// cross-multiplied comparison.  Keys of a_j <= ac are <= 0 and never win;
// a free resource has a_j <= ac (the free vertex has the largest free a_j),
// so its key is -inf or NaN and never wins either.  Lowest j on equal keys;
// -1 if no resource lies beyond ac.
template <int M, class Row, class Px>
__device__ __forceinline__ int scan_next_free(const Row& a, const Px& px, float ac)
{
    float best = 0.f;
    int jn = -1;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const float key = (a.get(j) - ac) * px.inv(j);
        const bool b = key > best;
        best = b ? key : best;
        jn = b ? j : jn;
    }
    return jn;
}

// Maximiser of u(t) minus the cost on the envelope segment from (alo, plo) to
// (ahi, phi) (§4.2), of slope alpha = (phi - plo) / (ahi - alo):
//   log, eq. e-opt-t-log: clip((u')^{-1}(alpha), alo, ahi) with
//     (u')^{-1}(alpha) = w / alpha - eps (+inf for alpha = 0); the alpha-fair
//     family: (w / alpha)^(1/a) - eps, and for a = 0 (linear) the right end
//     if w > alpha, else the left end;
//   capped linear, eq. e-opt-t-target: the left end if w <= alpha, else the
//     cap clipped to the segment.
// `on` tells whether the unclipped maximiser reaches the right end, i.e.
// whether the optimum may lie on a later segment.
template <typename F, bool AF>
__device__ __forceinline__ F segment_argmax(bool caplin, F w, F c, F eps, F alo, F plo, F ahi,
                                            F phi, bool& on)
{
    const F num = phi - plo, den = ahi - alo;
    if (!caplin) {
        F tu;
        if (!AF || c == F(-1)) {
            tu = w * den * frcp(num) - eps;
        } else {
            const F a = afair_exponent(c);
            if (a == F(0))
                tu = (w * den > num) ? F(INFINITY) : F(-INFINITY);
            else
                tu = dpow(w * den * frcp(num), frcp(a)) - eps;
        }
        on = tu >= ahi;
        return fmin(fmax(tu, alo), ahi);
    }
    if (w * den <= num) {
        on = false;
        return alo;
    }
    on = c >= ahi;
    return fmin(fmax(c, alo), ahi);
}

// The segment of the envelope that holds a job's optimum: ends lo, hi
// (lo = -1: the origin; hi = -1: nothing to buy) and the optimal throughput t.
template <typename F>
struct Seg {
    int lo, hi, j1;
    F alo, plo, ahi, phi, t;
};

// Algorithm 1 of §4.2 as an envelope walk from the origin: the first vertex
// by the largest efficiency per price, then further vertices only while the
// segment's maximiser reaches its right end (u - c is concave, so the first
// segment whose maximiser lies before its right end holds the optimum).
// a.get(j): entry j in an unrolled scan; a.at(j): entry j for a per-lane j;
// px: the job's prices (SharedPrices, ArgPrices or DemandPrices); fr: some
// price is zero (wave-uniform).
template <typename F, int M, bool AF, class Row, class Px>
__device__ __forceinline__ Seg<F> walk_job(const Row& a, int mm, const Px& px, F w, F c,
                                           bool caplin, F eps, bool fr)
{
    Seg<F> S;
    S.j1 = fr ? scan_first<F, M, true>(a, mm, px) : scan_first<F, M, false>(a, mm, px);
    // An all-zero row (j1 < 0) buys nothing: t = 0.  It runs through the same
    // code with an empty segment so that every result has one definition.
    const bool any = S.j1 >= 0;
    S.lo = -1;
    S.hi = any ? S.j1 : -1;
    S.alo = F(0);
    S.plo = F(0);
    S.ahi = any ? a.at(S.j1) : F(1);
    S.phi = any ? px.at(S.j1) : F(0);
    S.t = F(0);
    bool walk = any;
    while (walk) {
        S.t = segment_argmax<F, AF>(caplin, w, c, eps, S.alo, S.plo, S.ahi, S.phi, walk);
        if (walk) {
            const int jn = scan_next<F, M>(a, mm, px, S.ahi, S.phi);
            if (jn < 0) {  // right end of the curve: t = max_j a_j
                walk = false;
            } else {
                S.lo = S.hi;
                S.alo = S.ahi;
                S.plo = S.phi;
                S.hi = jn;
                S.ahi = a.at(jn);
                S.phi = px.at(jn);
            }
        }
    }
    return S;
}


// ------------------------------------------------------------------------
// Envelope walk shared by the lanes of a wavefront (vectorised kernels).
// ------------------------------------------------------------------------
// A lane-per-job walk makes the whole wave scan a full row whenever any of
// its 64 jobs needs a further vertex, and usually few do.  Here every lane
// first finds its job's first vertex and first segment; then, while some
// jobs still need a further vertex, the W walkers of the wave are ranked and
// each is given G = 64 / W lanes (rounded down to a power of two, at most
// M / 4): lane k G + s scans entries [s M/G, (s + 1) M/G) of walker k's row,
// read from the staged tile, and a butterfly over the G lanes keeps the
// smallest slope (on equal slopes the lower part, so the lowest j).  The
// walker then moves to that vertex and takes the closed form on the new
// segment (segment_argmax), as in walk_from.

// One lane's part of a shared next-vertex scan: entries [s E, (s + 1) E),
// E = M / G, of the row at rowp (LDS).  G = 1: every lane scans the whole row,
// so the prices are read at wave-uniform indices (px.get, argument block);
// otherwise from the price table in LDS, four at a time.
template <int M, int G, class Px>
__device__ __forceinline__ void coop_scan_part(const float* rowp, int s, float ac, float pc,
                                               const Px& px, float& bn, float& bd, int& jn)
{
    constexpr int E = M / G;
    const int j0 = G == 1 ? 0 : s * E;
    bn = 1.f;
    bd = 0.f;
    jn = -1;
    // the LDS reads of up to 8 chunks (32 entries) at a time, then their
    // compare chain: the latency is paid once per batch
    constexpr int NC = E / 4, BC = NC < 8 ? NC : 8;
#pragma unroll
    for (int c0 = 0; c0 < NC; c0 += BC) {
        float4 a4[BC], p4[G == 1 ? 1 : BC];
#pragma unroll
        for (int e = 0; e < BC; ++e) {
            a4[e] = *reinterpret_cast<const float4*>(rowp + j0 + 4 * (c0 + e));
            if constexpr (G > 1)
                p4[e] = *reinterpret_cast<const float4*>(px.tab + j0 + 4 * (c0 + e));
        }
#pragma unroll
        for (int e = 0; e < BC; ++e) {
            const float av[4] = {a4[e].x, a4[e].y, a4[e].z, a4[e].w};
            float pv[4];
            if constexpr (G == 1) {
#pragma unroll
                for (int k = 0; k < 4; ++k) pv[k] = px.get(4 * (c0 + e) + k);
            } else {
                pv[0] = p4[e].x;
                pv[1] = p4[e].y;
                pv[2] = p4[e].z;
                pv[3] = p4[e].w;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int j = j0 + 4 * (c0 + e) + k;
                const float d = av[k] - ac;
                const float nm = fmaxf(pv[k] - pc, 0.f);  // as scan_next
                const bool b = nm * bd < bn * d;
                bn = b ? nm : bn;
                bd = b ? d : bd;
                jn = b ? j : jn;
            }
        }
    }
    // butterfly over the G lanes of this walker: lanes with bit `off` set
    // hold the upper part of the pair
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        const float obn = __shfl_xor(bn, off), obd = __shfl_xor(bd, off);
        const int ojn = __shfl_xor(jn, off);
        const bool upper = (threadIdx.x & off) != 0;
        const float abn = upper ? obn : bn, abd = upper ? obd : bd;
        const int ajn = upper ? ojn : jn;
        const float ubn = upper ? bn : obn, ubd = upper ? bd : obd;
        const int ujn = upper ? jn : ojn;
        const bool take = (ujn >= 0) & ((ajn < 0) | (ubn * abd < abn * ubd));
        bn = take ? ubn : abn;
        bd = take ? ubd : abd;
        jn = take ? ujn : ajn;
    }
}

// Continue the walks of the lanes with `walking` set (S: their current
// segment, amax: their row's largest throughput) until every job of the
// wave holds its final segment.  All 64 lanes must call it together.
// tile: the staged tile (row r at tile + r * RS); slots: 64 ints of LDS.
template <int M, int RS, bool AF, class Row, class Px>
__device__ __forceinline__ void coop_walk(Seg<float>& S, bool walking, float amax, const Row& a,
                                          const Px& px, const float* tile, int* slots, int lane,
                                          float w, float c, bool caplin, float eps)
{
    constexpr int GMAX = M / 4 < 16 ? M / 4 : 16;
    for (;;) {
        const uint64_t mask = __ballot(walking);
        if (mask == 0ull) break;
        const int W = __popcll(mask);
        const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        const int G0 = W > 32 ? 1 : W > 16 ? 2 : W > 8 ? 4 : W > 4 ? 8 : 16;
        const int G = G0 < GMAX ? G0 : GMAX;
        float bn = 1.f, bd = 0.f;
        int jn = -1;
        if (G == 1) {
            // more than 32 walkers: every lane scans its own row (no ranking)
            coop_scan_part<M, 1>(tile + lane * RS, 0, S.ahi, S.phi, px, bn, bd, jn);
            if (walking) {
                if (jn < 0) {
                    walking = false;
                } else {
                    S.lo = S.hi;
                    S.alo = S.ahi;
                    S.plo = S.phi;
                    S.hi = jn;
                    S.ahi = a.at(jn);
                    S.phi = px.at(jn);
                    bool on;
                    S.t = segment_argmax<float, AF>(caplin, w, c, eps, S.alo, S.plo, S.ahi,
                                                    S.phi, on);
                    walking = on & (S.ahi < amax);
                }
            }
            continue;
        }
        if (walking) slots[rank] = lane;
        wave_sync();
        // lane = k G + s works for walker k
        const int k = lane / G, s = lane & (G - 1);
        const int wl = k < W ? slots[k] : lane;
        const float ac = __shfl(S.ahi, wl), pc = __shfl(S.phi, wl);
        const float* rowp = tile + wl * RS;
        if constexpr (GMAX >= 2) {
            if (G == 2)
                coop_scan_part<M, 2>(rowp, s, ac, pc, px, bn, bd, jn);
            else if constexpr (GMAX >= 4) {
                if (G == 4)
                    coop_scan_part<M, 4>(rowp, s, ac, pc, px, bn, bd, jn);
                else if constexpr (GMAX >= 8) {
                    if (G == 8)
                        coop_scan_part<M, 8>(rowp, s, ac, pc, px, bn, bd, jn);
                    else if constexpr (GMAX >= 16)
                        coop_scan_part<M, 16>(rowp, s, ac, pc, px, bn, bd, jn);
                }
            }
        }
        // walker `rank` reads its result from lane rank G
        const int jw = __shfl(jn, (rank * G) & 63);
        wave_sync();  // the slots are written again in the next round
        if (walking) {
            if (jw < 0) {  // no point beyond: t = a_hi already
                walking = false;
            } else {
                S.lo = S.hi;
                S.alo = S.ahi;
                S.plo = S.phi;
                S.hi = jw;
                S.ahi = a.at(jw);
                S.phi = px.at(jw);
                bool on;
                S.t = segment_argmax<float, AF>(caplin, w, c, eps, S.alo, S.plo, S.ahi, S.phi, on);
                walking = on & (S.ahi < amax);
            }
        }
    }
}

// The first segment of a job from its first vertex j1: its closed form, and
// whether the walk goes on (the maximiser reaches the segment's right end
// and some resource lies beyond it).
template <bool AF, class Row, class Px>
__device__ __forceinline__ Seg<float> first_segment(const Row& a, const Px& px, int j1, float amax,
                                                    float w, float c, bool caplin, float eps,
                                                    bool& walking)
{
    Seg<float> S;
    const bool any = j1 >= 0;
    S.j1 = j1;
    S.lo = -1;
    S.hi = any ? j1 : -1;
    S.alo = 0.f;
    S.plo = 0.f;
    S.ahi = any ? a.at(j1) : 1.f;
    S.phi = any ? px.at(j1) : 0.f;
    S.t = 0.f;
    walking = false;
    if (any) {
        bool on;
        S.t = segment_argmax<float, AF>(caplin, w, c, eps, S.alo, S.plo, S.ahi, S.phi, on);
        walking = on & (S.ahi < amax);
    }
    return S;
}


// The start of a job's walk when some price is zero, with the row in
// registers.  A free resource costs nothing, so the first vertex is the free
// resource with the largest throughput a_F (scan_first's rule), found by a
// pass over the free entries alone (the index test is wave-uniform) that
// also takes the row's largest throughput; when the maximiser passes a_F,
// the next vertex from (a_F, 0) comes from one scan, which a later
// walk round would otherwise do (scan_next_free).  Rows with no free
// throughput (a_j = 0 on every free resource) take the first vertex by
// efficiency per price.
// Every lane of the wave must call it together.
template <int M, bool AF, class Row, class Px>
__device__ __forceinline__ Seg<float> free_start(const Row& a, const Px& px, float w, float c,
                                                 bool caplin, float eps, float& amax,
                                                 bool& walking)
{
    float aF = 0.f, am = 0.f;
    int jF = -1;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        const float aj = a.get(j);
        am = fmaxf(am, aj);
        if (px.get(j) == 0.f) {
            const bool b = aj > aF;
            aF = b ? aj : aF;
            jF = b ? j : jF;
        }
    }
    amax = am;
    int j1 = jF;
    if (__ballot(jF < 0) != 0ull) {
        const int jk = scan_first<float, M, true>(a, M, px);
        j1 = jF >= 0 ? jF : jk;
    }
    Seg<float> S = first_segment<AF>(a, px, j1, amax, w, c, caplin, eps, walking);
    const bool from_free = walking & (jF >= 0);
    if (__ballot(from_free) != 0ull) {
        const int jn = scan_next_free<M>(a, px, S.ahi);
        if (from_free) {
            if (jn < 0) {
                walking = false;
            } else {
                S.lo = S.hi;
                S.alo = S.ahi;
                S.plo = S.phi;
                S.hi = jn;
                S.ahi = a.at(jn);
                S.phi = px.at(jn);
                bool on;
                S.t = segment_argmax<float, AF>(caplin, w, c, eps, S.alo, S.plo, S.ahi, S.phi,
                                                on);
                walking = on & (S.ahi < amax);
            }
        }
    }
    return S;
}

// Allocation and net value on the final segment (eq. e-xixj; lo = -1: the
// origin, x_hi = t / a_hi), v = u(t) - (p_lo x_lo + p_hi x_hi).
template <typename F, bool AF>
__device__ __forceinline__ void finish_job(const Seg<F>& S, F w, F c, bool caplin, F eps,
                                           Job<F>& J)
{
    const F den = S.ahi - S.alo;
    const F rden = frcp(den);
    const F xh = (S.t - S.alo) * rden;
    const F xl = (S.lo >= 0) ? (S.ahi - S.t) * rden : F(0);
    J.j1 = S.j1;
    J.v = utility<F, AF>(caplin, w, c, eps, S.t) - (S.plo * xl + S.phi * xh);
    // a zero share is not part of the support; a single resource is
    // reported as (j_lo, j_hi) = (-1, j).  Written with selects only, so the
    // result stays in registers.
    const bool left = xh == F(0);   // t at the left end: only `lo` (or nothing)
    const bool right = xl == F(0);  // only `hi`
    J.jhi = left ? S.lo : S.hi;
    J.jlo = (left | right) ? -1 : S.lo;
    J.xhi = left ? xl : xh;
    J.xlo = (left | right) ? F(0) : xl;
    J.thi = left ? S.alo * xl : S.ahi * xh;
    J.tlo = (left | right) ? F(0) : S.alo * xl;
}

// One job's subproblem (§3, eq. e-subprob) by the envelope walk.
template <typename F, int M, bool AF = true, class Row, class Px>
__device__ __forceinline__ void solve_job(const Row& a, int mm, const Px& px, F w, F c,
                                          bool caplin, F eps, bool fr, Job<F>& J)
{
    finish_job<F, AF>(walk_job<F, M, AF>(a, mm, px, w, c, caplin, eps, fr), w, c, caplin, eps, J);
}

// log(1 + x) for x >= 0, FP32: a degree-5 Taylor polynomial below 1/32
// (truncation below 1e-8 relative), else the hardware logarithm of u = 1 + x
// with the rounding of u undone by the factor x / (u - 1) (u - 1 is exact);
// relative error a few 1e-7.  The device library's log1pf costs about ten
// times as many instructions.  FP64: the library.
__device__ __forceinline__ float dlog1p(float x)
{
    const float poly =
        x * (1.f + x * (-0.5f + x * (1.f / 3.f + x * (-0.25f + x * 0.2f))));
    const float u = 1.f + x;
    const float big = dlog(u) * (x * frcp(u - 1.f));
    return x < 0.03125f ? poly : big;
}
__device__ __forceinline__ double dlog1p(double x) { return log1p(x); }

// Lower-bound contribution of one job (§5): its allocation on (lo, hi) with
// throughput parts tlo = a_lo x_lo, thi = a_hi x_hi is scaled per column by
// s_j = min(1, R_j / r_j).  U = u(t~) with t~ = s_lo tlo + s_hi thi, and the
// utility lost, du = u(t) - u(t~), is formed from t - t~ = (1 - s_lo) tlo +
// (1 - s_hi) thi (1 - s_j given in FP64-rounded form) so that it keeps its
// relative accuracy when the scales are close to 1.
template <typename F, bool AF = true>
__device__ __forceinline__ void scaled_utility(bool caplin, F w, F c, F eps, int jlo, int jhi,
                                               F tlo, F thi, const F* S, const F* SC, F& U,
                                               F& du)
{
    const F tt = (jlo >= 0 ? S[jlo] * tlo : F(0)) + (jhi >= 0 ? S[jhi] * thi : F(0));
    const F dt = (jlo >= 0 ? SC[jlo] * tlo : F(0)) + (jhi >= 0 ? SC[jhi] * thi : F(0));
    U = utility<F, AF>(caplin, w, c, eps, tt);
    if (!caplin && (!AF || c == F(-1))) {
        du = w * dlog1p(dt * frcp(tt + eps));
    } else if (!caplin) {
        // u(t) - u(t~) = U ((1 + dt / (t~ + eps))^(1 - a) - 1)
        const F e = F(1) - afair_exponent(c);
        du = U * dexpm1(e * dlog1p(dt * frcp(tt + eps)));
    } else {
        const F t = tlo + thi;
        du = (tt >= c) ? F(0) : (t <= c ? w * dt : w * (c - tt));
    }
}

// 16-byte streaming load with the non-temporal hint: every byte of T is read
// once per evaluation, so it should not displace reusable lines in the caches.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 stream_load(const float4* p)
{
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// The same loads through pointers known to be global (the batched kernel
// reads its problems' base pointers from memory, which would otherwise give
// flat loads, and flat loads also count against the LDS/scalar counter).
typedef __attribute__((address_space(1))) const f32x4 global_f32x4;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const f32x2 global_f32x2;
__device__ __forceinline__ float4 stream_load_global(const float4* p)
{
    const f32x4 v = __builtin_nontemporal_load((global_f32x4*)p);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 load_global(const float2* p)
{
    const f32x2 v = *(global_f32x2*)p;
    return make_float2(v.x, v.y);
}

template <int M>
struct RegRow {
    float v[M];
    const float* lds;
    __device__ __forceinline__ float get(int j) const { return v[j]; }
    __device__ __forceinline__ float at(int j) const { return lds[j]; }
};

// A job's row of a staged tile, read from LDS on every use (demand vectors).
struct LdsRow {
    const float* lds;
    __device__ __forceinline__ float get(int j) const { return lds[j]; }
    __device__ __forceinline__ float at(int j) const { return lds[j]; }
};

template <typename F>
struct GlobalRow {
    const F* __restrict__ r;
    __device__ __forceinline__ F get(int j) const { return r[j]; }
    __device__ __forceinline__ F at(int j) const { return r[j]; }
};

// ------------------------------------------------------------------------
// Dual kernel, FP32, m = M in {4, 8, 16, 32, 64}, T 16-byte aligned.
// ------------------------------------------------------------------------
// The price block is the first kernel argument, so it starts the argument
// segment (the AMDGPU kernel ABI lays arguments out in order from offset 0).
template <int M, bool DEM, bool DV>
__global__ void __launch_bounds__(256, DV ? 1 : 2) k_dual_vec(
    const PriceArgs<M> pa, const float* __restrict__ T, const float2* __restrict__ prm, int64_t n,
    float eps, double* __restrict__ partial,
    int* __restrict__ jpair, float2* __restrict__ xpair, float2* __restrict__ tpair,
    int16_t* __restrict__ j1out, const float* __restrict__ dem, const float* __restrict__ dvec,
    const PriceArgs<M>* __restrict__ dpa, const int* __restrict__ skip)
{
    // dpa (optional): the prices in device memory, written by the device
    // price loop, instead of the argument block; skip (optional): when *skip
    // is set the pass is not needed (the loop has ended) and the kernel
    // returns at once.
    if (skip && *skip) return;
    // dem (DEM, optional): per-job demands d_i; prm then holds w_i / d_i, so
    // each job is solved at prices p unchanged, and its net value, usage and
    // certificate terms are scaled by d_i (the subproblem at prices d_i p).
    // dvec (DV): per-job demand vectors, n x M like T, staged through LDS
    // with T; job i is solved at the prices d_i * p and adds d_ij x_ij to r_j.
    constexpr int Q = M / 4;                    // 16-byte chunks per row
    constexpr int S = M + ((Q & 1) ? 0 : 4);    // LDS row stride in words
    constexpr int TR = 64;                      // rows per wave tile
    __shared__ __attribute__((aligned(16))) float tile[4][TR * S];
    __shared__ __attribute__((aligned(16))) float dtile[DV ? 4 : 1][DV ? TR * S : 4];
    __shared__ float hist[4][M];
    __shared__ __attribute__((aligned(16))) float ptab[M], qtab[M];
    __shared__ float stab[M], sctab[M];
    __shared__ int wslot[4][64];  // walkers of a shared walk round (coop_walk)

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const bool prev = (dpa ? dpa->has_prev : pa.has_prev) != 0;
    if (threadIdx.x < M) {
        const int t = threadIdx.x;
        ptab[t] = dpa ? dpa->p[t] : pa.p[t];
        qtab[t] = dpa ? dpa->q[t] : pa.q[t];
        stab[t] = dpa ? dpa->s[t] : pa.s[t];
        sctab[t] = dpa ? dpa->sc[t] : pa.sc[t];
    }
    if (lane < M) hist[wv][lane] = 0.f;
    __syncthreads();
    // some price zero (wave-uniform): the first-vertex scans then order free
    // resources by throughput
    const bool freep = __ballot(ptab[lane % M] == 0.f) != 0ull;
    const bool freeq = prev && (__ballot(qtab[lane % M] == 0.f) != 0ull);

    double racc = 0.0, vacc = 0.0, uacc = 0.0, duacc = 0.0;
    const int64_t ntiles = (n + TR - 1) / TR;
    const int64_t nw = (int64_t)gridDim.x * 4;
    int64_t ti = (int64_t)blockIdx.x * 4 + wv;
    float* tl = tile[wv];
    float* dtl = dtile[DV ? wv : 0];
    float4 pre[Q];
    float4 dpre[DV ? Q : 1];
    float2 wcn = make_float2(0.f, 0.f);
    float dn = 1.f;

    auto load_tile = [&](int64_t tix) {
        const int64_t row0 = tix * TR;
        const int64_t rows = (n - row0) < TR ? (n - row0) : TR;
        const float4* src = reinterpret_cast<const float4*>(T + row0 * M);
        const float4* dsrc = DV ? reinterpret_cast<const float4*>(dvec + row0 * M) : nullptr;
        if (rows == TR) {
#pragma unroll
            for (int k = 0; k < Q; ++k) pre[k] = stream_load(src + lane + 64 * k);
            if constexpr (DV) {
#pragma unroll
                for (int k = 0; k < Q; ++k) dpre[k] = stream_load(dsrc + lane + 64 * k);
            }
            wcn = prm[row0 + lane];
            if constexpr (DEM) dn = dem[row0 + lane];
        } else {
            // rows past n: zero throughputs, unit demands (never used)
            const int valid = (int)rows * Q;
#pragma unroll
            for (int k = 0; k < Q; ++k) {
                const int ch = lane + 64 * k;
                pre[k] = (ch < valid) ? stream_load(src + ch) : make_float4(0.f, 0.f, 0.f, 0.f);
                if constexpr (DV)
                    dpre[k] =
                        (ch < valid) ? stream_load(dsrc + ch) : make_float4(1.f, 1.f, 1.f, 1.f);
            }
            wcn = (lane < rows) ? prm[row0 + lane] : make_float2(1.f, -1.f);
            if constexpr (DEM) dn = (lane < rows) ? dem[row0 + lane] : 1.f;
        }
    };

    // Per-job outputs of a tile are kept in registers and stored at the start
    // of the next iteration, before the following tile's loads are issued:
    // the vector-memory counter retires in order, so waiting for a tile's
    // loads then never waits for stores issued after them.
    int64_t pend_i = -1;
    int pend_jp = 0;
    int16_t pend_j1 = 0;
    float2 pend_x = make_float2(0.f, 0.f), pend_t = make_float2(0.f, 0.f);
    auto flush_outputs = [&]() {
        if (pend_i >= 0) {
            if (jpair) jpair[pend_i] = pend_jp;
            if (xpair) xpair[pend_i] = pend_x;
            if (tpair) tpair[pend_i] = pend_t;
            if (j1out) j1out[pend_i] = pend_j1;
        }
    };

    if (ti < ntiles) load_tile(ti);
    for (; ti < ntiles; ti += nw) {
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int ch = lane + 64 * k;
            const int r = ch / Q, q = ch % Q;
            *reinterpret_cast<float4*>(tl + r * S + 4 * q) = pre[k];
            if constexpr (DV) *reinterpret_cast<float4*>(dtl + r * S + 4 * q) = dpre[k];
        }
        const float2 wc = wcn;
        const float dj = DEM ? dn : 1.f;
        wave_sync();
        flush_outputs();
        if (ti + nw < ntiles) load_tile(ti + nw);

        const int64_t i = ti * TR + lane;
        pend_i = -1;
        RegRow<M> row;
        row.lds = tl + lane * S;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float4 v = *reinterpret_cast<const float4*>(row.lds + 4 * q);
            row.v[4 * q + 0] = v.x;
            row.v[4 * q + 1] = v.y;
            row.v[4 * q + 2] = v.z;
            row.v[4 * q + 3] = v.w;
        }
        const bool caplin = is_capped(wc.y);
        // the price block at the start of the argument segment, its address
        // made opaque once per tile: the prices are then read again for
        // every tile instead of being held in scalar registers across the
        // loop (4 M of them would not fit)
        ArgPtr<M> pk = dpa ? (ArgPtr<M>)dpa : (ArgPtr<M>)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(pk));
        Job<float> J, K;
        if constexpr (DV) {
            // demand vectors: each job walks its own envelope at d_i * p; the
            // usage and value at p are taken before the walk at q, which keeps
            // fewer values live (the demand row then stays in registers)
            if (i < n) {
                // the job's demand row in registers for the unrolled scans
                // (per-lane indices read the staged tile)
                RegRow<M> drow;
                drow.lds = dtl + lane * S;
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    const float4 v = *reinterpret_cast<const float4*>(drow.lds + 4 * q);
                    drow.v[4 * q + 0] = v.x;
                    drow.v[4 * q + 1] = v.y;
                    drow.v[4 * q + 2] = v.z;
                    drow.v[4 * q + 3] = v.w;
                }
                using PA = ArgPrices<M, false>;
                using PB = ArgPrices<M, true>;
                const DemandPrices<float, PA, RegRow<M>> pp{PA{pk, ptab}, drow};
                finish_job<float, true>(
                    walk_job<float, M, true>(row, M, pp, wc.x, wc.y, caplin, eps, freep), wc.x,
                    wc.y, caplin, eps, J);
                if (J.jlo >= 0) atomicAdd(&hist[wv][J.jlo], drow.at(J.jlo) * J.xlo);
                if (J.jhi >= 0) atomicAdd(&hist[wv][J.jhi], drow.at(J.jhi) * J.xhi);
                vacc += (double)J.v;
                if (prev) {
                    const DemandPrices<float, PB, RegRow<M>> pq{PB{pk, qtab}, drow};
                    finish_job<float, true>(
                        walk_job<float, M, true>(row, M, pq, wc.x, wc.y, caplin, eps, freeq),
                        wc.x, wc.y, caplin, eps, K);
                    float u, loss;
                    scaled_utility(caplin, wc.x, wc.y, eps, K.jlo, K.jhi, K.tlo, K.thi, stab,
                                   sctab, u, loss);
                    uacc += (double)u;
                    duacc += (double)loss;
                }
                pend_i = i;
                pend_jp = (J.jlo & 0xffff) | (J.jhi << 16);
                pend_x = make_float2(J.xlo, J.xhi);
                pend_t = make_float2(J.tlo, J.thi);
                pend_j1 = (int16_t)J.j1;
            }
        } else {
            // every lane takes part (rows past n are zero: nothing to buy),
            // the walks beyond the first segment shared by the wave
            // both walk starts read the row from registers; the walks read rows
            // from the staged tile, so the registers are free then.  The row's
            // largest throughput (where every walk ends) is found only in waves
            // where some walk goes on.
            const ArgPrices<M, false> pp{pk, ptab};
            const ArgPrices<M, true> pq{pk, qtab};
            float amax = INFINITY;
            bool have_max = false;
            auto row_max = [&](bool on) {
                if (!have_max && __ballot(on) != 0ull) {
                    amax = 0.f;
#pragma unroll
                    for (int j = 0; j < M; ++j) amax = fmaxf(amax, row.get(j));
                    have_max = true;
                }
            };
            bool walking, walking_q = false;
            Seg<float> SP, SQ;
            if (freep) {
                SP = free_start<M, true>(row, pp, wc.x, wc.y, caplin, eps, amax, walking);
                have_max = true;
            } else {
                SP = first_segment<true>(row, pp, scan_first<float, M, false>(row, M, pp), amax,
                                         wc.x, wc.y, caplin, eps, walking);
                row_max(walking);
                walking = walking & (SP.ahi < amax);
            }
            if (prev) {
                if (freeq) {
                    float amq;
                    SQ = free_start<M, true>(row, pq, wc.x, wc.y, caplin, eps, amq, walking_q);
                    amax = amq;
                    have_max = true;
                } else {
                    SQ = first_segment<true>(row, pq, scan_first<float, M, false>(row, M, pq),
                                             amax, wc.x, wc.y, caplin, eps, walking_q);
                    row_max(walking_q);
                    walking_q = walking_q & (SQ.ahi < amax);
                }
            }
            coop_walk<M, S, true>(SP, walking, amax, row, pp, tl, wslot[wv], lane, wc.x, wc.y,
                                  caplin, eps);
            finish_job<float, true>(SP, wc.x, wc.y, caplin, eps, J);
            if (prev) {
                walking = walking_q;
                coop_walk<M, S, true>(SQ, walking, amax, row, pq, tl, wslot[wv], lane, wc.x,
                                      wc.y, caplin, eps);
                finish_job<float, true>(SQ, wc.x, wc.y, caplin, eps, K);
            }
        }
        if (!DV && i < n) {
            if (J.jlo >= 0) atomicAdd(&hist[wv][J.jlo], dj * J.xlo);
            if (J.jhi >= 0) atomicAdd(&hist[wv][J.jhi], dj * J.xhi);
            vacc += (double)J.v * (double)dj;
            if (prev) {  // lower bound of the previous prices, same row
                float u, loss;
                scaled_utility(caplin, wc.x, wc.y, eps, K.jlo, K.jhi, K.tlo, K.thi, stab, sctab,
                               u, loss);
                uacc += (double)u * (double)dj;
                duacc += (double)loss * (double)dj;
            }
            pend_i = i;
            pend_jp = (J.jlo & 0xffff) | (J.jhi << 16);
            pend_x = make_float2(J.xlo, J.xhi);
            pend_t = make_float2(J.tlo, J.thi);
            pend_j1 = (int16_t)J.j1;
        }
        wave_sync();
        if (lane < M) {
            racc += (double)hist[wv][lane];
            hist[wv][lane] = 0.f;
        }
        wave_sync();
    }
    flush_outputs();

#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        vacc += __shfl_xor(vacc, off);
        uacc += __shfl_xor(uacc, off);
        duacc += __shfl_xor(duacc, off);
    }
    constexpr int NC = M + 3;
    __syncthreads();
    double* red = reinterpret_cast<double*>(&tile[0][0]);
    if (lane < M) red[wv * NC + lane] = racc;
    if (lane == 0) {
        red[wv * NC + M] = vacc;
        red[wv * NC + M + 1] = uacc;
        red[wv * NC + M + 2] = duacc;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        const int t = threadIdx.x;
        const double s = ((red[t] + red[NC + t]) + red[2 * NC + t]) + red[3 * NC + t];
        partial[(int64_t)blockIdx.x * NC + t] = s;
    }
}

// ------------------------------------------------------------------------
// Dual kernel, any m <= 256, FP32 or FP64: one lane per job reading its row
// straight from global memory (used for FP64 and for m outside the
// vectorised classes).  DV: per-job demand vectors dvec (n x m, like T), read
// the same way; job i is solved at the prices d_i * p and adds d_ij x_ij.
// ------------------------------------------------------------------------
// One block's share of a generic pass (WPB waves per block, grid-stride over
// 64-job tiles, one lane per job reading its row from global memory): each
// wave's sums of r, of v and, with prev, of u(t~) and u(t) - u(t~) are left
// in red[wave][0..m-1], red[wave][m], [m + 1], [m + 2], for the caller to
// combine.  Prices P, IP at the new point and, with prev, Q, IQ with the
// column scales S, SC of the point to certify.  Every thread of the block
// must call it.
template <typename F, bool DV, int WPB>
__device__ __forceinline__ void gen_block_pass(
    const F* __restrict__ T, const V2<F>* __restrict__ prm, int64_t n, int m, const F* P,
    const F* IP, const F* Q, const F* IQ, const F* S, const F* SC, bool prev, F eps,
    int* __restrict__ jpair, V2<F>* __restrict__ xpair, V2<F>* __restrict__ tpair,
    int16_t* __restrict__ j1out, const F* __restrict__ dem, const F* __restrict__ dvec,
    F (*hist)[256], double (*red)[259])
{
    constexpr int TR = 64;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    for (int j = lane; j < m; j += 64) hist[wv][j] = F(0);
    __syncthreads();
    // some price zero (wave-uniform): see scan_first
    bool zp = false, zq = false;
    for (int j = lane; j < m; j += 64) {
        zp |= P[j] == F(0);
        zq |= prev && Q[j] == F(0);
    }
    const bool freep = __ballot(zp) != 0ull;
    const bool freeq = __ballot(zq) != 0ull;

    double racc[4] = {0.0, 0.0, 0.0, 0.0};
    double vacc = 0.0, uacc = 0.0, duacc = 0.0;
    const int64_t ntiles = (n + TR - 1) / TR;
    const int64_t nw = (int64_t)gridDim.x * WPB;
    for (int64_t ti = (int64_t)blockIdx.x * WPB + wv; ti < ntiles; ti += nw) {
        const int64_t i = ti * TR + lane;
        if (i < n) {
            GlobalRow<F> row{T + i * m};
            const V2<F> wc = prm[i];
            Job<F> J;
            const bool caplin = is_capped(wc.y);
            const F dj = dem ? dem[i] : F(1);
            const GlobalRow<F> drow{DV ? dvec + i * m : nullptr};
            auto solve = [&](const F* Pp, const F* IPp, bool fr, Job<F>& out) {
                if constexpr (DV)
                    solve_job<F, 0>(row, m,
                                    DemandPrices<F, SharedPrices<F>, GlobalRow<F>>{
                                        SharedPrices<F>{Pp, IPp, Pp}, drow},
                                    wc.x, wc.y, caplin, eps, fr, out);
                else
                    solve_job<F, 0>(row, m, SharedPrices<F>{Pp, IPp, Pp}, wc.x, wc.y, caplin, eps,
                                    fr, out);
            };
            solve(P, IP, freep, J);
            if (J.jlo >= 0) atomicAdd(&hist[wv][J.jlo], (DV ? drow.at(J.jlo) : dj) * J.xlo);
            if (J.jhi >= 0) atomicAdd(&hist[wv][J.jhi], (DV ? drow.at(J.jhi) : dj) * J.xhi);
            vacc += (double)J.v * (double)dj;
            if (prev) {  // lower bound of the previous prices, same row
                Job<F> K;
                solve(Q, IQ, freeq, K);
                F u, loss;
                scaled_utility(caplin, wc.x, wc.y, eps, K.jlo, K.jhi, K.tlo, K.thi, S, SC, u, loss);
                uacc += (double)u * (double)dj;
                duacc += (double)loss * (double)dj;
            }
            if (jpair) jpair[i] = (J.jlo & 0xffff) | (J.jhi << 16);
            if (xpair) xpair[i] = V2<F>{J.xlo, J.xhi};
            if (tpair) tpair[i] = V2<F>{J.tlo, J.thi};
            if (j1out) j1out[i] = (int16_t)J.j1;
        }
        wave_sync();
        for (int k = 0; k < 4; ++k) {
            const int j = lane + 64 * k;
            if (j < m) {
                racc[k] += (double)hist[wv][j];
                hist[wv][j] = F(0);
            }
        }
        wave_sync();
    }
    for (int off = 32; off > 0; off >>= 1) {
        vacc += __shfl_xor(vacc, off);
        uacc += __shfl_xor(uacc, off);
        duacc += __shfl_xor(duacc, off);
    }
    for (int k = 0; k < 4; ++k) {
        const int j = lane + 64 * k;
        if (j < m) red[wv][j] = racc[k];
    }
    if (lane == 0) {
        red[wv][m] = vacc;
        red[wv][m + 1] = uacc;
        red[wv][m + 2] = duacc;
    }
    __syncthreads();
}

template <typename F, bool DV>
__global__ void __launch_bounds__(256) k_dual_gen(
    const F* __restrict__ T, const V2<F>* __restrict__ prm, int64_t n, int m,
    const PriceBlock<F>* __restrict__ pb, F eps, double* __restrict__ partial,
    int* __restrict__ jpair, V2<F>* __restrict__ xpair, V2<F>* __restrict__ tpair,
    int16_t* __restrict__ j1out, const F* __restrict__ dem, const F* __restrict__ dvec)
{
    __shared__ F hist[4][256];
    __shared__ double red[4][259];
    gen_block_pass<F, DV, 4>(T, prm, n, m, pb->p, pb->invp, pb->q, pb->invq, pb->s, pb->sc,
                          pb->has_prev != 0, eps, jpair, xpair, tpair, j1out, dem, dvec, hist,
                          red);
    const int nc = m + 3;
    for (int t = threadIdx.x; t < nc; t += 256) {
        const double s = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
        partial[(int64_t)blockIdx.x * nc + t] = s;
    }
}

// A generic solver pass of a small problem (n <= SMALL_MAX_N jobs, m <=
// SMALL_MAX_M, no demand vectors) as one launch of at most four blocks (one
// 64-job tile per wave): the prices come as a kernel argument, each block
// leaves its sums in partial[block], and the block that takes the last
// ticket adds them up in block order and writes the columns of the
// reduction (r, sum v, sum u(t~), sum of the loss) straight into pinned host
// memory, with the completion flag after them.  One launch per pass instead
// of a price copy, the dual kernel and the column reduction.
template <typename F>
__global__ void __launch_bounds__(256) k_dual_small(const F* __restrict__ T,
                                                    const V2<F>* __restrict__ prm, int64_t n,
                                                    int m, const SmallPrices<F> sp, F eps,
                                                    const F* __restrict__ dem,
                                                    double* __restrict__ partial,
                                                    unsigned* __restrict__ ticket,
                                                    double* __restrict__ out,
                                                    unsigned* __restrict__ flag)
{
    __shared__ F hist[4][256];
    __shared__ double red[4][259];
    __shared__ F pt[6][SMALL_MAX_M];
    __shared__ bool last;
    for (int t = threadIdx.x; t < m; t += 256) {
        pt[0][t] = sp.p[t];
        pt[1][t] = sp.invp[t];
        pt[2][t] = sp.q[t];
        pt[3][t] = sp.invq[t];
        pt[4][t] = sp.s[t];
        pt[5][t] = sp.sc[t];
    }
    __syncthreads();
    gen_block_pass<F, false, 4>(T, prm, n, m, pt[0], pt[1], pt[2], pt[3], pt[4], pt[5],
                                sp.has_prev != 0, eps, nullptr, nullptr, nullptr, nullptr, dem,
                                nullptr, hist, red);
    const int nc = m + 3;
    for (int t = threadIdx.x; t < nc; t += 256) {
        partial[(int64_t)blockIdx.x * nc + t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
        __threadfence();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        last = atomicAdd(ticket, 1u) == gridDim.x - 1u;
        if (last) atomicExch(ticket, 0u);
    }
    __syncthreads();
    if (!last) return;
    __threadfence();  // every block's sums are visible past this point
    for (int t = threadIdx.x; t < nc; t += 256) {
        double s = partial[t];
        for (int b = 1; b < (int)gridDim.x; ++b) s += partial[(int64_t)b * nc + t];
        out[t] = s;
        __threadfence_system();
    }
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// ------------------------------------------------------------------------
// Batched dual kernel: many FP32 problems with m in {4, 8, 16, 32} evaluated
// in one persistent launch per price iteration.  A batched tile is `rows`
// consecutive jobs of one problem (BatchShape: a multiple of 64 per m class,
// at most TF floats of T; TF is the register budget the kernel is compiled
// for), so a lane solves rows / 64 jobs of a tile, one per 64-row step.  The
// host lays the active problems' tiles end to end and gives each wavefront a
// contiguous chunk of that tile space, balanced by the measured cost of each
// m class.  The next tile (possibly of the next problem) is loaded into
// registers while the current one is solved from LDS.  Each 64-row step
// solves its jobs as the vectorised kernel does: first vertices from the
// row in registers, then envelope walks shared by the wavefront.  A wave
// keeps FP64 accumulators for the problem it is in and writes them to its
// next partial slot whenever it crosses into another problem, so the slots
// of one problem are contiguous and are summed in a fixed order by
// k_batch_reduce.
// ------------------------------------------------------------------------

// The prices of one problem of a batch: wave-uniform reads of the price rows
// in global memory (scalar loads), per-lane reads from the wave's LDS copy.
struct BatchPrices {
    const float* __restrict__ P;
    const float* __restrict__ IP;
    const float* tab;
    __device__ __forceinline__ float get(int j) const { return P[j]; }
    __device__ __forceinline__ float inv(int j) const { return IP[j]; }
    __device__ __forceinline__ float at(int j) const { return tab[j]; }
};

// Minimum resident blocks per compute unit the batched kernel is compiled
// for (its register budget): the larger the tile, the more registers the
// prefetched tile holds.
constexpr int batch_min_blocks(int tf, bool dem) { return tf <= 1024 ? (dem ? 3 : 4) : tf <= 2048 ? (dem ? 2 : 3) : 2; }

// One staged tile of problem `it` (rows valid rows of height tr, at tl with
// row stride batch_stride(M)): every job solved at the problem's prices P
// and, with prev, at its previous prices Q (certificate); usage into the
// wave's LDS histogram, then into the lane's FP64 accumulators.
template <int M, int JPL, bool DEM, bool AF>
__device__ __forceinline__ void batch_compute(const BatchItem& it, int rows, const float* tl,
                                              const float2* wcl, const float* dml, float* hist, int* slots, const BatchPrices& pp,
                                              const BatchPrices& pq, const float* stab,
                                              const float* sctab, bool prev, bool freep,
                                              bool freeq, int lane, double& racc, double& vacc,
                                              double& uacc, double& duacc)
{
    constexpr int Q = M / 4;
    constexpr int S = M + ((Q & 1) ? 0 : 4);
    const float eps = it.eps;
#pragma unroll
    for (int k = 0; k < JPL; ++k) {
        if (64 * k >= rows) break;  // wave-uniform
        const int r = 64 * k + lane;
        const float* sub = tl + 64 * k * S;  // this step's 64 rows
        RegRow<M> row;
        row.lds = sub + lane * S;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float4 v = *reinterpret_cast<const float4*>(row.lds + 4 * q);
            row.v[4 * q + 0] = v.x;
            row.v[4 * q + 1] = v.y;
            row.v[4 * q + 2] = v.z;
            row.v[4 * q + 3] = v.w;
        }
        // rows past the problem's end are zero (nothing to buy) and never summed
        const float2 wck = wcl[r];
        const float dmk = DEM ? dml[r] : 1.f;
        const float w = wck.x, c = wck.y;
        const bool caplin = is_capped(c);
        float amax = INFINITY;
        bool have_max = false;
        auto row_max = [&](bool on) {
            if (!have_max && __ballot(on) != 0ull) {
                amax = 0.f;
#pragma unroll
                for (int j = 0; j < M; ++j) amax = fmaxf(amax, row.get(j));
                have_max = true;
            }
        };
        bool walking, walking_q = false;
        Seg<float> SP, SQ;
        if (freep) {
            SP = free_start<M, AF>(row, pp, w, c, caplin, eps, amax, walking);
            have_max = true;
        } else {
            SP = first_segment<AF>(row, pp, scan_first<float, M, false>(row, M, pp), amax, w, c,
                                   caplin, eps, walking);
            row_max(walking);
            walking = walking & (SP.ahi < amax);
        }
        if (prev) {
            if (freeq) {
                float amq;
                SQ = free_start<M, AF>(row, pq, w, c, caplin, eps, amq, walking_q);
                amax = amq;
                have_max = true;
            } else {
                SQ = first_segment<AF>(row, pq, scan_first<float, M, false>(row, M, pq), amax, w,
                                       c, caplin, eps, walking_q);
                row_max(walking_q);
                walking_q = walking_q & (SQ.ahi < amax);
            }
        }
        coop_walk<M, S, AF>(SP, walking, amax, row, pp, sub, slots, lane, w, c, caplin, eps);
        Job<float> J;
        finish_job<float, AF>(SP, w, c, caplin, eps, J);
        if (r < rows) {
            if (J.jlo >= 0) atomicAdd(&hist[J.jlo], dmk * J.xlo);
            if (J.jhi >= 0) atomicAdd(&hist[J.jhi], dmk * J.xhi);
            vacc += (double)J.v * (double)dmk;
        }
        if (prev) {
            walking = walking_q;
            coop_walk<M, S, AF>(SQ, walking, amax, row, pq, sub, slots, lane, w, c, caplin, eps);
            Job<float> K;
            finish_job<float, AF>(SQ, w, c, caplin, eps, K);
            if (r < rows) {
                float u, loss;
                scaled_utility<float, AF>(caplin, w, c, eps, K.jlo, K.jhi, K.tlo, K.thi, stab,
                                          sctab, u, loss);
                uacc += (double)u * (double)dmk;
                duacc += (double)loss * (double)dmk;
            }
        }
    }
    wave_sync();
    if (lane < M) {
        racc += (double)hist[lane];
        hist[lane] = 0.f;
    }
    wave_sync();
}

// lds_floats: LDS floats per wave (dynamic shared memory, four waves per
// block) for a staged tile: rows x batch_stride(m) floats of T, then the
// (w, c) pairs of its rows, then (DEM) their demands.
template <bool DEM, bool AF, int TF>
__global__ void __launch_bounds__(256, batch_min_blocks(TF, DEM))
    k_dual_batch(const BatchItem* __restrict__ items, const float* __restrict__ prices,
                 const int* __restrict__ chunk, const int* __restrict__ segbase,
                 double* __restrict__ partial, int lds_floats)
{
    constexpr int V = TF / 256;                                      // float4 per lane of a tile
    constexpr int JPL = TF / 256 < BATCH_MAX_JPL ? TF / 256 : BATCH_MAX_JPL;  // jobs per lane
    extern __shared__ __attribute__((aligned(16))) float batch_tiles[];
    __shared__ float hist[4][BATCH_MAX_M];
    __shared__ __attribute__((aligned(16))) float tabs[4][4][BATCH_MAX_M];
    __shared__ int wslot[4][64];
    const int lane = threadIdx.x & 63;
    // the wave index is uniform: saying so keeps the tile bookkeeping, the
    // problem records and the price reads in scalar registers and scalar
    // loads, which do not wait behind the prefetched tile's vector loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int w = blockIdx.x * 4 + wv;
    const int t0 = chunk[w], t1 = chunk[w + 1];
    float* tl = batch_tiles + wv * lds_floats;
    float* hs = hist[wv];
    if (lane < BATCH_MAX_M) hs[lane] = 0.f;
    wave_sync();
    if (t0 >= t1) return;

    // the tile in flight: up to TF floats of T (V float4 per lane) and the
    // (w, c) of up to JPL jobs per lane; `an` is the problem of the last tile
    // loaded (items[A].tile0 is the total tile count, so the scans stop)
    float4 pre[V];
    float2 wcn[JPL];
    float dmn[JPL];
    int an = 0, nrows = 0;
    auto load = [&](int t) {
        while (items[an + 1].tile0 <= t) ++an;
        const BatchItem& nx = items[an];
        const int m = nx.m;
        const int tr = nx.rows;
        const int64_t row0 = (int64_t)(t - nx.tile0) * tr;
        const int64_t left = nx.n - row0;
        const int rows = left < tr ? (int)left : tr;
        const float4* src = reinterpret_cast<const float4*>(nx.T + row0 * m);
        const int valid = rows * (m / 4);
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int ch = lane + 64 * k;
            pre[k] = (ch < valid) ? stream_load_global(src + ch) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int k = 0; k < JPL; ++k) {
            const int r = 64 * k + lane;
            wcn[k] = (r < rows) ? load_global(nx.prm + row0 + r) : make_float2(1.f, -1.f);
        }
        if (DEM && nx.dem) {
#pragma unroll
            for (int k = 0; k < JPL; ++k) {
                const int r = 64 * k + lane;
                dmn[k] = (r < rows) ? *(__attribute__((address_space(1))) const float*)(nx.dem + row0 + r)
                                    : 1.f;
            }
        } else {
#pragma unroll
            for (int k = 0; k < JPL; ++k) dmn[k] = 1.f;
        }
        nrows = rows;
    };

    int slot = segbase[w];
    int cur = -1;
    bool freep = false, freeq = false;  // some price zero (see scan_first)
    BatchItem it;
    BatchPrices pp{nullptr, nullptr, tabs[wv][0]}, pq{nullptr, nullptr, tabs[wv][1]};
    double racc = 0.0, vacc = 0.0, uacc = 0.0, duacc = 0.0;
    auto flush = [&]() {
        for (int off = 32; off > 0; off >>= 1) {
            vacc += __shfl_xor(vacc, off);
            uacc += __shfl_xor(uacc, off);
            duacc += __shfl_xor(duacc, off);
        }
        double* out = partial + (int64_t)slot * BATCH_COLS;
        if (lane < BATCH_MAX_M) out[lane] = (lane < it.m) ? racc : 0.0;
        if (lane == 0) {
            out[BATCH_MAX_M] = vacc;
            out[BATCH_MAX_M + 1] = uacc;
            out[BATCH_MAX_M + 2] = duacc;
        }
        ++slot;
        racc = vacc = uacc = duacc = 0.0;
    };

    load(t0);
    for (int t = t0; t < t1; ++t) {
        const int a = an;
        const int rows = nrows;
        if (a != cur) {
            if (cur >= 0) flush();
            cur = a;
            it = items[a];
            const float* pr = prices + (int64_t)a * 6 * BATCH_MAX_M;
            pp.P = pr;
            pp.IP = pr + BATCH_MAX_M;
            pq.P = pr + 2 * BATCH_MAX_M;
            pq.IP = pr + 3 * BATCH_MAX_M;
            freep = __ballot(lane < it.m && pr[lane] == 0.f) != 0ull;
            freeq = __ballot(lane < it.m && pr[2 * BATCH_MAX_M + lane] == 0.f) != 0ull;
            if (lane < it.m) {
                tabs[wv][0][lane] = pr[lane];
                tabs[wv][1][lane] = pr[2 * BATCH_MAX_M + lane];
                tabs[wv][2][lane] = pr[4 * BATCH_MAX_M + lane];
                tabs[wv][3][lane] = pr[5 * BATCH_MAX_M + lane];
            }
        }
        // stage the tile in LDS: chunk ch of 16 bytes is row ch / Q, quad
        // ch % Q; the whole tile height is written, so rows past the
        // problem's end are zero
        const int m = it.m;
        const int Q = m >> 2;
        const int lq = m == 4 ? 0 : m == 8 ? 1 : m == 16 ? 2 : 3;
        const int S = batch_stride(m);
        const int height = it.rows * Q;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const int ch = lane + 64 * k;
            if (ch < height)
                *reinterpret_cast<float4*>(tl + (ch >> lq) * S + 4 * (ch & (Q - 1))) = pre[k];
        }
        float2* wcl = reinterpret_cast<float2*>(tl + it.rows * S);
        float* dml = tl + it.rows * (S + 2);
#pragma unroll
        for (int k = 0; k < JPL; ++k) {
            if (64 * k < it.rows) {
                wcl[64 * k + lane] = wcn[k];
                if (DEM) dml[64 * k + lane] = dmn[k];
            }
        }
        wave_sync();
        if (t + 1 < t1) load(t + 1);
        const bool prev = it.has_prev != 0;
        const float* st = tabs[wv][2];
        const float* sct = tabs[wv][3];
        int* sl = wslot[wv];
        switch (m) {
        case 4:
            batch_compute<4, JPL, DEM, AF>(it, rows, tl, wcl, dml, hs, sl, pp, pq, st, sct, prev, freep,
                                      freeq, lane, racc, vacc, uacc, duacc);
            break;
        case 8:
            batch_compute<8, JPL, DEM, AF>(it, rows, tl, wcl, dml, hs, sl, pp, pq, st, sct, prev, freep,
                                      freeq, lane, racc, vacc, uacc, duacc);
            break;
        case 16:
            batch_compute<16, JPL, DEM, AF>(it, rows, tl, wcl, dml, hs, sl, pp, pq, st, sct, prev, freep,
                                       freeq, lane, racc, vacc, uacc, duacc);
            break;
        default:
            batch_compute<32, JPL, DEM, AF>(it, rows, tl, wcl, dml, hs, sl, pp, pq, st, sct, prev, freep,
                                       freeq, lane, racc, vacc, uacc, duacc);
            break;
        }
    }
    flush();
}

// out[a][c] = sum of partial slots [seg[2a], seg[2a+1]] of column c, for the
// active problems a < header[0] (blocks stride over them).  Seven groups of
// BATCH_COLS lanes take every seventh slot, and their sums are added in
// group order (a fixed order, so results are reproducible).  With `flag`,
// out is host memory the host polls: lane c of a block writes column c of
// the block's rows, and one lane makes them visible system-wide and takes a
// ticket; the block with the last ticket resets the counter and raises
// *flag = 1.
constexpr int BATCH_RED_GROUPS = 7;  // 7 x 35 lanes of a 256-lane block

// A round's table from pinned host memory (read over the bus, each 16-byte
// word once) to device memory: a kernel launch, which queues behind the
// stream's earlier work without holding the host, unlike a small
// host-to-device copy.
__global__ void __launch_bounds__(256) k_copy_table(const uint4* __restrict__ src,
                                                    uint4* __restrict__ dst, int64_t n16)
{
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n16;
         k += (int64_t)gridDim.x * 256)
        dst[k] = src[k];
}

__global__ void __launch_bounds__(256) k_batch_reduce(const double* __restrict__ partial,
                                                      const int* __restrict__ seg,
                                                      const int* __restrict__ header,
                                                      double* __restrict__ out,
                                                      unsigned* __restrict__ ticket,
                                                      unsigned* __restrict__ flag)
{
    __shared__ double grp[BATCH_RED_GROUPS][BATCH_COLS];
    const int tid = threadIdx.x;
    const int g = tid / BATCH_COLS, c = tid % BATCH_COLS;
    const int A = header[0];
    for (int a = blockIdx.x; a < A; a += gridDim.x) {
        if (g < BATCH_RED_GROUPS) {
            double s = 0.0;
            const int k1 = seg[2 * a + 1];
#pragma unroll 4
            for (int k = seg[2 * a] + g; k <= k1; k += BATCH_RED_GROUPS)
                s += partial[(int64_t)k * BATCH_COLS + c];
            grp[g][c] = s;
        }
        __syncthreads();
        if (tid < BATCH_COLS) {
            double s = grp[0][tid];
            for (int h = 1; h < BATCH_RED_GROUPS; ++h) s += grp[h][tid];
            out[(int64_t)a * BATCH_COLS + tid] = s;
        }
        __syncthreads();
    }
    if (flag && tid == 0) {
        __threadfence_system();
        if (atomicAdd(ticket, 1u) == (unsigned)gridDim.x - 1u) {
            atomicExch(ticket, 0u);
            __threadfence_system();
            __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

// ------------------------------------------------------------------------
// Data-dependent starting prices (§5, eq. e-initialization): with the uniform
// share x (wave-uniform, pb->p), each job's derivative d_i = u_i'(a_i^T x)
// (log: w / (t + eps); capped linear: w below the cap, 0 at or above it), and
// partial[b][j] = sum over the block's jobs of d_i a_ij.  The host divides
// the column sums by n.
// FP32, m = M in {4, 8, 16, 32, 64}, T 16-byte aligned: tiles staged as in
// k_dual_vec; lane = job for the derivative, then lane = column for the
// tile's weighted column sum (column reads of the padded tile are
// conflict-free).
// ------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(256) k_init_vec(const float* __restrict__ T,
                                                  const float2* __restrict__ prm, int64_t n,
                                                  const PriceBlock<float>* __restrict__ pb,
                                                  float eps, double* __restrict__ partial)
{
    constexpr int Q = M / 4;
    constexpr int S = M + ((Q & 1) ? 0 : 4);
    constexpr int TR = 64;
    __shared__ __attribute__((aligned(16))) float tile[4][TR * S];
    __shared__ float dtab[4][TR];
    __shared__ float xtab[M];
    __shared__ double red[4][M];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    if (threadIdx.x < M) xtab[threadIdx.x] = pb->p[threadIdx.x];
    __syncthreads();
    double racc = 0.0;
    const int64_t ntiles = (n + TR - 1) / TR;
    const int64_t nw = (int64_t)gridDim.x * 4;
    float* tl = tile[wv];
    for (int64_t ti = (int64_t)blockIdx.x * 4 + wv; ti < ntiles; ti += nw) {
        const int64_t row0 = ti * TR;
        const int rows = (int)((n - row0) < TR ? (n - row0) : TR);
        const float4* src = reinterpret_cast<const float4*>(T + row0 * M);
        const int valid = rows * Q;
#pragma unroll
        for (int k = 0; k < Q; ++k) {
            const int ch = lane + 64 * k;
            const float4 v = (ch < valid) ? stream_load(src + ch) : make_float4(0.f, 0.f, 0.f, 0.f);
            const int r = ch / Q, q = ch % Q;
            *reinterpret_cast<float4*>(tl + r * S + 4 * q) = v;
        }
        const float2 wc = (lane < rows) ? prm[row0 + lane] : make_float2(0.f, -1.f);
        wave_sync();
        float t = 0.f;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const float4 v = *reinterpret_cast<const float4*>(tl + lane * S + 4 * q);
            t += v.x * xtab[4 * q] + v.y * xtab[4 * q + 1] + v.z * xtab[4 * q + 2] +
                 v.w * xtab[4 * q + 3];
        }
        const bool caplin = is_capped(wc.y);
        float d;
        if (caplin)
            d = t < wc.y ? wc.x : 0.f;
        else if (wc.y == -1.f)
            d = wc.x / (t + eps);
        else
            d = wc.x * powf(t + eps, -afair_exponent(wc.y));
        dtab[wv][lane] = lane < rows ? d : 0.f;
        wave_sync();
        if (lane < M) {
            float s = 0.f;
            for (int r = 0; r < TR; ++r) s += dtab[wv][r] * tl[r * S + lane];
            racc += (double)s;
        }
        wave_sync();
    }
    if (lane < M) red[wv][lane] = racc;
    __syncthreads();
    if (threadIdx.x < M) {
        const int j = threadIdx.x;
        partial[(int64_t)blockIdx.x * M + j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
    }
}

// Any m <= 256, FP32 or FP64: one lane per job reading its row from global
// memory; d_i a_ij added into a per-wave LDS row, flushed per tile.  With
// demand vectors (dvec, n x m) job i adds d_i a_ij / dvec_ij: its
// willingness to pay per unit of resource j it demands.
template <typename F>
__global__ void __launch_bounds__(256) k_init_gen(const F* __restrict__ T,
                                                  const V2<F>* __restrict__ prm, int64_t n,
                                                  int m, const PriceBlock<F>* __restrict__ pb,
                                                  F eps, double* __restrict__ partial,
                                                  const F* __restrict__ dvec)
{
    constexpr int TR = 64;
    __shared__ F hist[4][256];
    __shared__ double red[4][256];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const F* __restrict__ x = pb->p;
    for (int j = lane; j < m; j += 64) hist[wv][j] = F(0);
    __syncthreads();
    double racc[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t ntiles = (n + TR - 1) / TR;
    const int64_t nw = (int64_t)gridDim.x * 4;
    for (int64_t ti = (int64_t)blockIdx.x * 4 + wv; ti < ntiles; ti += nw) {
        const int64_t i = ti * TR + lane;
        if (i < n) {
            const F* a = T + i * m;
            F t = F(0);
            for (int j = 0; j < m; ++j) t += a[j] * x[j];
            const V2<F> wc = prm[i];
            F d;
            if (is_capped(wc.y))
                d = t < wc.y ? wc.x : F(0);
            else if (wc.y == F(-1))
                d = wc.x / (t + eps);
            else
                d = wc.x * dpow(t + eps, -afair_exponent(wc.y));
            if (d != F(0) && dvec) {
                const F* dr = dvec + i * m;
                for (int j = 0; j < m; ++j) atomicAdd(&hist[wv][j], d * a[j] / dr[j]);
            } else if (d != F(0)) {
                for (int j = 0; j < m; ++j) atomicAdd(&hist[wv][j], d * a[j]);
            }
        }
        wave_sync();
        for (int k = 0; k < 4; ++k) {
            const int j = lane + 64 * k;
            if (j < m) {
                racc[k] += (double)hist[wv][j];
                hist[wv][j] = F(0);
            }
        }
        wave_sync();
    }
    for (int k = 0; k < 4; ++k) {
        const int j = lane + 64 * k;
        if (j < m) red[wv][j] = racc[k];
    }
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += 256)
        partial[(int64_t)blockIdx.x * m + j] = ((red[0][j] + red[1][j]) + red[2][j]) + red[3][j];
}

// ------------------------------------------------------------------------
// Column reduction of block partials: one block per column, fixed order.
// ------------------------------------------------------------------------
// With `flag` set, out is host memory the host polls: each block makes its
// column visible system-wide, takes a ticket, and the block holding the last
// ticket resets the ticket counter and raises *flag = 1.
__global__ void __launch_bounds__(256) k_reduce_cols(const double* __restrict__ partial, int nb,
                                                     int ncols, double* __restrict__ out,
                                                     unsigned* __restrict__ ticket,
                                                     unsigned* __restrict__ flag,
                                                     const int* __restrict__ skip)
{
    if (skip && *skip) return;  // the device price loop has ended
    __shared__ double red[256];
    const int j = blockIdx.x;
    const double s = column_sum(partial, nb, ncols, j, red);
    if (threadIdx.x == 0) {
        out[j] = s;
        if (flag) {
            __threadfence_system();
            if (atomicAdd(ticket, 1u) == (unsigned)gridDim.x - 1u) {
                atomicExch(ticket, 0u);
                __threadfence_system();
                __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
}

// ------------------------------------------------------------------------
// Lower bound (§5): column scales s_j = min(1, R_j / r_j), scaled throughput
// t~_i = s_lo a_lo x_lo + s_hi a_hi x_hi, sums of u(t~_i) and of the utility
// lost by scaling, u(t_i) - u(t~_i).  The loss is formed from
// t_i - t~_i = (1 - s_lo) a_lo x_lo + (1 - s_hi) a_hi x_hi, with 1 - s_j
// computed in FP64, so it keeps its relative accuracy when s_j is close to 1.
// ------------------------------------------------------------------------
template <typename F>
__global__ void __launch_bounds__(256) k_lower(const int* __restrict__ jpair,
                                               const V2<F>* __restrict__ tpair,
                                               const V2<F>* __restrict__ prm, int64_t n, int m,
                                               const double* __restrict__ R,
                                               const double* __restrict__ r, F eps,
                                               double* __restrict__ partial2,
                                               const F* __restrict__ dem)
{
    __shared__ F s[256];
    __shared__ F sc[256];
    __shared__ double red[2][4];
    for (int j = threadIdx.x; j < m; j += 256) {
        const bool over = r[j] > R[j];
        s[j] = over ? F(R[j] / r[j]) : F(1);
        sc[j] = over ? F((r[j] - R[j]) / r[j]) : F(0);
    }
    __syncthreads();
    double U = 0.0, du = 0.0;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const int jp = jpair[i];
        const int jlo = (int)(int16_t)(jp & 0xffff);
        const int jhi = jp >> 16;
        const V2<F> tp = tpair[i];
        const V2<F> wc = prm[i];
        F u, loss;
        scaled_utility(is_capped(wc.y), wc.x, wc.y, eps, jlo, jhi, tp.x, tp.y, s, sc, u, loss);
        const double dj = dem ? (double)dem[i] : 1.0;
        U += (double)u * dj;
        du += (double)loss * dj;
    }
    for (int off = 32; off > 0; off >>= 1) {
        U += __shfl_xor(U, off);
        du += __shfl_xor(du, off);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wv] = U;
        red[1][wv] = du;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int k = threadIdx.x;
        partial2[(int64_t)blockIdx.x * 2 + k] = ((red[k][0] + red[k][1]) + red[k][2]) + red[k][3];
    }
}

// ------------------------------------------------------------------------
// Input packing and validation.
// ------------------------------------------------------------------------
template <typename F>
__global__ void k_pack(const F* __restrict__ w, const F* __restrict__ c,
                       const uint8_t* __restrict__ kind, int64_t n, V2<F>* __restrict__ prm,
                       int* __restrict__ bad)
{
    int flags = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint8_t k = kind ? kind[i] : (uint8_t)0;
        const F wi = w[i];
        F ci = F(-1);
        if (!(wi > F(0)) || !isfinite(wi)) flags |= 1;
        if (k == 1) {
            ci = c[i];
            if (!(ci >= F(0)) || !isfinite(ci)) flags |= 2;
            ci = (ci == F(0)) ? F(0) : ci;  // a cap of -0 is stored as +0 (sign bit clear)
        } else if (k == 2) {
            // alpha-fair exponent a >= 0; a = 1 is the log utility
            const F a = c[i];
            if (!(a >= F(0)) || !isfinite(a)) flags |= 2;
            ci = (a == F(1)) ? F(-1) : -a;  // -0 for a = 0: the sign bit marks the family
            if (a != F(1)) flags |= 16;  // the problem has alpha-fair jobs (not an error)
        } else if (k > 2) {
            flags |= 4;
        }
        prm[i] = V2<F>{wi, ci};
    }
    if (flags) atomicOr(bad, flags);
}

template <typename F>
__global__ void k_validate_T(const F* __restrict__ T, int64_t count, int* __restrict__ bad,
                             bool positive)
{
    int flags = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
        const F v = T[e];
        if (!(positive ? v > F(0) : v >= F(0)) || !isfinite(v)) flags |= 8;
    }
    if (flags) atomicOr(bad, flags);
}

template <typename F>
__global__ void k_materialize(const int* __restrict__ jpair, const V2<F>* __restrict__ xpair,
                              int64_t n, int m, const double* __restrict__ R,
                              const double* __restrict__ r, F* __restrict__ X)
{
    __shared__ F s[256];
    for (int j = threadIdx.x; j < m; j += blockDim.x) s[j] = (r[j] > R[j]) ? F(R[j] / r[j]) : F(1);
    __syncthreads();
    const int64_t total = n * m;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t i = e / m;
        const int j = (int)(e - i * m);
        const int jp = jpair[i];
        const int jlo = (int)(int16_t)(jp & 0xffff);
        const int jhi = jp >> 16;
        const V2<F> xp = xpair[i];
        F x = F(0);
        if (jlo == j) x += s[j] * xp.x;
        if (jhi == j) x += s[j] * xp.y;
        X[e] = x;
    }
}

// ------------------------------------------------------------------------
// Host-side launchers.
// ------------------------------------------------------------------------
template <typename K>
static int occupancy_blocks(K kernel)
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, 256, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb;
}

static bool vec_class(int m) { return m == 4 || m == 8 || m == 16 || m == 32 || m == 64; }

template <int M>
static int vec_occupancy(bool dv)
{
    return dv ? occupancy_blocks(k_dual_vec<M, false, true>)
              : occupancy_blocks(k_dual_vec<M, false, false>);
}

int dual_grid(int dev_cus, int m, int dtype, int64_t n, bool vec_ok, bool dv)
{
    // occupancy per kernel: vectorised classes 0-4 (+5 with demand vectors),
    // generic FP32 / FP64 10-11 (+2 with demand vectors)
    static int occ[14] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    int slot;
    if (dtype == 0 && vec_ok && vec_class(m)) {
        slot = (m == 4 ? 0 : m == 8 ? 1 : m == 16 ? 2 : m == 32 ? 3 : 4) + (dv ? 5 : 0);
    } else {
        slot = (dtype == 0 ? 10 : 11) + (dv ? 2 : 0);
    }
    if (occ[slot] == 0) {
        switch (slot % 5 + (slot >= 10 ? 5 : 0)) {
        case 0: occ[slot] = vec_occupancy<4>(dv); break;
        case 1: occ[slot] = vec_occupancy<8>(dv); break;
        case 2: occ[slot] = vec_occupancy<16>(dv); break;
        case 3: occ[slot] = vec_occupancy<32>(dv); break;
        case 4: occ[slot] = vec_occupancy<64>(dv); break;
        default:
            if (dtype == 0)
                occ[slot] = dv ? occupancy_blocks(k_dual_gen<float, true>)
                               : occupancy_blocks(k_dual_gen<float, false>);
            else
                occ[slot] = dv ? occupancy_blocks(k_dual_gen<double, true>)
                               : occupancy_blocks(k_dual_gen<double, false>);
            break;
        }
    }
    const int64_t ntiles = (n + 63) / 64;
    const int64_t want = (ntiles + 3) / 4;
    const int64_t cap = (int64_t)dev_cus * occ[slot];
    int64_t g = want < cap ? want : cap;
    return (int)(g < 1 ? 1 : g);
}

template <int M>
static PriceArgs<M> price_args(const PriceBlock<float>& h)
{
    PriceArgs<M> a;
    for (int j = 0; j < M; ++j) {
        a.p[j] = h.p[j];
        a.invp[j] = h.invp[j];
        a.q[j] = h.q[j];
        a.invq[j] = h.invq[j];
        a.s[j] = h.s[j];
        a.sc[j] = h.sc[j];
    }
    a.has_prev = h.has_prev;
    return a;
}

template <int M>
static void launch_vec(int grid, hipStream_t st, const float* T, const float2* prm, int64_t n,
                       const PriceBlock<float>* h, float eps, double* partial, int* jp,
                       float2* xp, float2* tp, int16_t* j1, const float* dem, const float* dv,
                       const void* dprices = nullptr, const int* skip = nullptr)
{
    // with device prices the argument block is not read
    const PriceArgs<M> a = h ? price_args<M>(*h) : PriceArgs<M>{};
    const auto* dpa = static_cast<const PriceArgs<M>*>(dprices);
    if (dv)
        k_dual_vec<M, false, true><<<grid, 256, 0, st>>>(a, T, prm, n, eps, partial, jp, xp, tp,
                                                         j1, nullptr, dv, dpa, skip);
    else if (dem)
        k_dual_vec<M, true, false><<<grid, 256, 0, st>>>(a, T, prm, n, eps, partial, jp, xp, tp,
                                                         j1, dem, nullptr, dpa, skip);
    else
        k_dual_vec<M, false, false><<<grid, 256, 0, st>>>(a, T, prm, n, eps, partial, jp, xp,
                                                          tp, j1, nullptr, nullptr, dpa, skip);
}

bool dual_is_vec(int dtype, int m, bool vec_ok) { return dtype == 0 && vec_ok && vec_class(m); }

hipError_t launch_dual_dev(int m, int grid, hipStream_t st, const void* T, const void* prm,
                           int64_t n, double eps, double* partial, const void* dem,
                           const void* dvec, const void* dprices, const int* skip)
{
    const float* Tf = static_cast<const float*>(T);
    const float2* pr = static_cast<const float2*>(prm);
    const float e = (float)eps;
    const float* df = static_cast<const float*>(dem);
    const float* dv = static_cast<const float*>(dvec);
    switch (m) {
    case 4: launch_vec<4>(grid, st, Tf, pr, n, nullptr, e, partial, nullptr, nullptr, nullptr, nullptr, df, dv, dprices, skip); break;
    case 8: launch_vec<8>(grid, st, Tf, pr, n, nullptr, e, partial, nullptr, nullptr, nullptr, nullptr, df, dv, dprices, skip); break;
    case 16: launch_vec<16>(grid, st, Tf, pr, n, nullptr, e, partial, nullptr, nullptr, nullptr, nullptr, df, dv, dprices, skip); break;
    case 32: launch_vec<32>(grid, st, Tf, pr, n, nullptr, e, partial, nullptr, nullptr, nullptr, nullptr, df, dv, dprices, skip); break;
    case 64: launch_vec<64>(grid, st, Tf, pr, n, nullptr, e, partial, nullptr, nullptr, nullptr, nullptr, df, dv, dprices, skip); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename F>
static hipError_t launch_small_t(hipStream_t st, const void* T, const void* prm, int64_t n, int m,
                                 const void* host_prices, double eps, const void* dem,
                                 double* partial, unsigned* ticket, double* out, unsigned* flag)
{
    const auto* b = static_cast<const PriceBlock<F>*>(host_prices);
    SmallPrices<F> sp;
    for (int j = 0; j < SMALL_MAX_M; ++j) {
        const bool in = j < m;
        sp.p[j] = in ? b->p[j] : F(0);
        sp.invp[j] = in ? b->invp[j] : F(0);
        sp.q[j] = in ? b->q[j] : F(0);
        sp.invq[j] = in ? b->invq[j] : F(0);
        sp.s[j] = in ? b->s[j] : F(0);
        sp.sc[j] = in ? b->sc[j] : F(0);
    }
    sp.has_prev = b->has_prev;
    const int grid = (int)(((n + 63) / 64 + 3) / 4);
    k_dual_small<F><<<grid, 256, 0, st>>>(static_cast<const F*>(T),
                                          static_cast<const V2<F>*>(prm), n, m, sp, (F)eps,
                                          static_cast<const F*>(dem), partial, ticket, out, flag);
    return hipGetLastError();
}

hipError_t launch_dual_small(int dtype, hipStream_t st, const void* T, const void* prm,
                             int64_t n, int m, const void* host_prices, double eps,
                             const void* dem, double* partial, unsigned* ticket, double* out,
                             unsigned* flag)
{
    if (n < 1 || n > SMALL_MAX_N || m < 1 || m > SMALL_MAX_M) return hipErrorInvalidValue;
    return dtype == 0 ? launch_small_t<float>(st, T, prm, n, m, host_prices, eps, dem, partial,
                                              ticket, out, flag)
                      : launch_small_t<double>(st, T, prm, n, m, host_prices, eps, dem, partial,
                                               ticket, out, flag);
}

hipError_t launch_dual(int dtype, int m, bool vec_ok, int grid, hipStream_t st, const void* T,
                       const void* prm, int64_t n, const void* prices, const void* host_prices,
                       double eps, double* partial, int16_t* jpair, void* xpair, void* tpair,
                       int16_t* j1, const void* dem, const void* dvec)
{
    int* jp = reinterpret_cast<int*>(jpair);
    if (dtype == 0) {
        const float* Tf = static_cast<const float*>(T);
        const float2* pr = static_cast<const float2*>(prm);
        const auto* pb = static_cast<const PriceBlock<float>*>(prices);
        float2* xp = static_cast<float2*>(xpair);
        float2* tp = static_cast<float2*>(tpair);
        const float e = (float)eps;
        const float* df = static_cast<const float*>(dem);
        const float* dv = static_cast<const float*>(dvec);
        if (dual_is_vec(dtype, m, vec_ok)) {
            const auto* h = static_cast<const PriceBlock<float>*>(host_prices);
            switch (m) {
            case 4: launch_vec<4>(grid, st, Tf, pr, n, h, e, partial, jp, xp, tp, j1, df, dv); break;
            case 8: launch_vec<8>(grid, st, Tf, pr, n, h, e, partial, jp, xp, tp, j1, df, dv); break;
            case 16: launch_vec<16>(grid, st, Tf, pr, n, h, e, partial, jp, xp, tp, j1, df, dv); break;
            case 32: launch_vec<32>(grid, st, Tf, pr, n, h, e, partial, jp, xp, tp, j1, df, dv); break;
            default: launch_vec<64>(grid, st, Tf, pr, n, h, e, partial, jp, xp, tp, j1, df, dv); break;
            }
        } else if (dv) {
            k_dual_gen<float, true><<<grid, 256, 0, st>>>(Tf, pr, n, m, pb, e, partial, jp, xp, tp,
                                                          j1, nullptr, dv);
        } else {
            k_dual_gen<float, false><<<grid, 256, 0, st>>>(Tf, pr, n, m, pb, e, partial, jp, xp,
                                                           tp, j1, df, nullptr);
        }
    } else {
        const double* Td = static_cast<const double*>(T);
        const double2* pr = static_cast<const double2*>(prm);
        const auto* pb = static_cast<const PriceBlock<double>*>(prices);
        double2* xp = static_cast<double2*>(xpair);
        double2* tp = static_cast<double2*>(tpair);
        const double* dv = static_cast<const double*>(dvec);
        if (dv)
            k_dual_gen<double, true><<<grid, 256, 0, st>>>(Td, pr, n, m, pb, eps, partial, jp, xp,
                                                           tp, j1, nullptr, dv);
        else
            k_dual_gen<double, false><<<grid, 256, 0, st>>>(Td, pr, n, m, pb, eps, partial, jp,
                                                            xp, tp, j1,
                                                            static_cast<const double*>(dem),
                                                            nullptr);
    }
    return hipGetLastError();
}

hipError_t launch_init(int dtype, int m, bool vec_ok, int grid, hipStream_t st, const void* T,
                       const void* prm, int64_t n, const void* prices, double eps,
                       double* partial, const void* dvec)
{
    if (dtype == 0) {
        const float* Tf = static_cast<const float*>(T);
        const float2* pr = static_cast<const float2*>(prm);
        const auto* pb = static_cast<const PriceBlock<float>*>(prices);
        const float e = (float)eps;
        if (vec_ok && vec_class(m) && !dvec) {
            switch (m) {
            case 4: k_init_vec<4><<<grid, 256, 0, st>>>(Tf, pr, n, pb, e, partial); break;
            case 8: k_init_vec<8><<<grid, 256, 0, st>>>(Tf, pr, n, pb, e, partial); break;
            case 16: k_init_vec<16><<<grid, 256, 0, st>>>(Tf, pr, n, pb, e, partial); break;
            case 32: k_init_vec<32><<<grid, 256, 0, st>>>(Tf, pr, n, pb, e, partial); break;
            default: k_init_vec<64><<<grid, 256, 0, st>>>(Tf, pr, n, pb, e, partial); break;
            }
        } else {
            k_init_gen<float><<<grid, 256, 0, st>>>(Tf, pr, n, m, pb, e, partial,
                                                    static_cast<const float*>(dvec));
        }
    } else {
        k_init_gen<double><<<grid, 256, 0, st>>>(
            static_cast<const double*>(T), static_cast<const double2*>(prm), n, m,
            static_cast<const PriceBlock<double>*>(prices), eps, partial,
            static_cast<const double*>(dvec));
    }
    return hipGetLastError();
}

template <bool DEM, bool AF, int TF>
static int batch_occupancy(int lds_floats)
{
    int nb = 0;
    const size_t lds = sizeof(float) * 4 * (size_t)lds_floats;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_dual_batch<DEM, AF, TF>, 256, lds) !=
            hipSuccess ||
        nb < 1)
        nb = 1;
    return nb;
}

template <bool DEM, bool AF>
static int batch_occupancy_tf(int tf, int lds_floats)
{
    return tf <= 1024   ? batch_occupancy<DEM, AF, 1024>(lds_floats)
           : tf <= 2048 ? batch_occupancy<DEM, AF, 2048>(lds_floats)
                        : batch_occupancy<DEM, AF, 4096>(lds_floats);
}

int batch_blocks_per_cu(int tf, bool demands, bool alpha_fair, int lds_floats)
{
    if (demands && alpha_fair) return batch_occupancy_tf<true, true>(tf, lds_floats);
    if (demands) return batch_occupancy_tf<true, false>(tf, lds_floats);
    if (alpha_fair) return batch_occupancy_tf<false, true>(tf, lds_floats);
    return batch_occupancy_tf<false, false>(tf, lds_floats);
}

template <bool DEM, bool AF>
static void launch_batch_tf(int tf, int lds_floats, int grid, hipStream_t st,
                            const BatchItem* items, const float* prices, const int* chunk,
                            const int* segbase, double* partial)
{
    const size_t lds = sizeof(float) * 4 * (size_t)lds_floats;
    if (tf <= 1024)
        k_dual_batch<DEM, AF, 1024><<<grid, 256, lds, st>>>(items, prices, chunk, segbase, partial,
                                                            lds_floats);
    else if (tf <= 2048)
        k_dual_batch<DEM, AF, 2048><<<grid, 256, lds, st>>>(items, prices, chunk, segbase, partial,
                                                            lds_floats);
    else
        k_dual_batch<DEM, AF, 4096><<<grid, 256, lds, st>>>(items, prices, chunk, segbase, partial,
                                                            lds_floats);
}

hipError_t launch_batch(int tf, int lds_floats, int grid, int max_items, hipStream_t st,
                        const BatchItem* items, const float* prices, const int* chunk,
                        const int* segbase, const int* seg, const int* header, double* partial,
                        double* out, unsigned* ticket, unsigned* flag, bool demands,
                        bool alpha_fair)
{
    if (demands && alpha_fair)
        launch_batch_tf<true, true>(tf, lds_floats, grid, st, items, prices, chunk, segbase, partial);
    else if (demands)
        launch_batch_tf<true, false>(tf, lds_floats, grid, st, items, prices, chunk, segbase, partial);
    else if (alpha_fair)
        launch_batch_tf<false, true>(tf, lds_floats, grid, st, items, prices, chunk, segbase, partial);
    else
        launch_batch_tf<false, false>(tf, lds_floats, grid, st, items, prices, chunk, segbase, partial);
    const int rgrid = max_items < 256 ? max_items : 256;
    k_batch_reduce<<<rgrid, 256, 0, st>>>(partial, seg, header, out, ticket, flag);
    return hipGetLastError();
}

hipError_t launch_copy_table(const void* host_src, void* dst, size_t bytes, hipStream_t st)
{
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    const int64_t want = (n16 + 255) / 256;
    const int grid = (int)(want < 256 ? want : 256);
    k_copy_table<<<grid, 256, 0, st>>>(static_cast<const uint4*>(host_src), static_cast<uint4*>(dst),
                                       n16);
    return hipGetLastError();
}

hipError_t launch_reduce_cols(hipStream_t st, const double* partial, int nb, int ncols,
                              double* out, unsigned* ticket, unsigned* flag, const int* skip)
{
    k_reduce_cols<<<ncols, 256, 0, st>>>(partial, nb, ncols, out, ticket, flag, skip);
    return hipGetLastError();
}

int lower_grid(int dev_cus, int64_t n)
{
    const int64_t want = (n + 255) / 256;
    const int64_t cap = (int64_t)dev_cus * 8;
    int64_t g = want < cap ? want : cap;
    return (int)(g < 1 ? 1 : g);
}

hipError_t launch_lower(int dtype, int grid, hipStream_t st, const int16_t* jpair,
                        const void* tpair, const void* prm, int64_t n, int m, const double* R,
                        const double* r, double eps, double* partial2, const void* dem)
{
    const int* jp = reinterpret_cast<const int*>(jpair);
    if (dtype == 0)
        k_lower<float><<<grid, 256, 0, st>>>(jp, static_cast<const float2*>(tpair),
                                             static_cast<const float2*>(prm), n, m, R, r,
                                             (float)eps, partial2, static_cast<const float*>(dem));
    else
        k_lower<double><<<grid, 256, 0, st>>>(jp, static_cast<const double2*>(tpair),
                                              static_cast<const double2*>(prm), n, m, R, r, eps,
                                              partial2, static_cast<const double*>(dem));
    return hipGetLastError();
}

namespace {
// Per-job demands (§7, extensions): w0 holds the weights as packed, dem the
// demands; the packed weight becomes w0 / d (a job solved at prices d p with
// weight w is solved at prices p with weight w / d, its utilities being
// linear in w).  bad |= 1 for a demand that is not positive and finite.
template <typename F>
__global__ void k_apply_demands(const F* __restrict__ d, const F* __restrict__ w0, int64_t n,
                                V2<F>* __restrict__ prm, F* __restrict__ dem, int* __restrict__ bad)
{
    int flag = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const F di = d ? d[i] : F(1);
        if (!(di > F(0)) || !isfinite(di)) flag = 1;
        dem[i] = di;
        prm[i].x = w0[i] / di;
    }
    if (flag) atomicOr(bad, 1);
}

template <typename F>
__global__ void k_weights(const V2<F>* __restrict__ prm, int64_t n, F* __restrict__ w0)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        w0[i] = prm[i].x;
}

template <typename F>
__global__ void k_restore_weights(const F* __restrict__ w0, int64_t n, V2<F>* __restrict__ prm)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        prm[i].x = w0[i];
}
}  // namespace

hipError_t launch_demands(int dtype, hipStream_t st, int op, const void* d, void* w0, int64_t n,
                          void* prm, void* dem, int* bad)
{
    const int grid = (int)std::min<int64_t>(4096, (n + 255) / 256);
    if (dtype == 0) {
        if (op == 0)
            k_weights<float><<<grid, 256, 0, st>>>(static_cast<const float2*>(prm), n,
                                                   static_cast<float*>(w0));
        else if (op == 1)
            k_apply_demands<float><<<grid, 256, 0, st>>>(static_cast<const float*>(d),
                                                         static_cast<const float*>(w0), n,
                                                         static_cast<float2*>(prm),
                                                         static_cast<float*>(dem), bad);
        else
            k_restore_weights<float><<<grid, 256, 0, st>>>(static_cast<const float*>(w0), n,
                                                           static_cast<float2*>(prm));
    } else {
        if (op == 0)
            k_weights<double><<<grid, 256, 0, st>>>(static_cast<const double2*>(prm), n,
                                                    static_cast<double*>(w0));
        else if (op == 1)
            k_apply_demands<double><<<grid, 256, 0, st>>>(static_cast<const double*>(d),
                                                          static_cast<const double*>(w0), n,
                                                          static_cast<double2*>(prm),
                                                          static_cast<double*>(dem), bad);
        else
            k_restore_weights<double><<<grid, 256, 0, st>>>(static_cast<const double*>(w0), n,
                                                            static_cast<double2*>(prm));
    }
    return hipGetLastError();
}

hipError_t launch_pack(int dtype, hipStream_t st, const void* w, const void* c,
                       const uint8_t* kind, int64_t n, void* prm, int* bad)
{
    const int64_t want = (n + 255) / 256;
    const int grid = (int)(want < 4096 ? (want < 1 ? 1 : want) : 4096);
    if (dtype == 0)
        k_pack<float><<<grid, 256, 0, st>>>(static_cast<const float*>(w),
                                            static_cast<const float*>(c), kind, n,
                                            static_cast<float2*>(prm), bad);
    else
        k_pack<double><<<grid, 256, 0, st>>>(static_cast<const double*>(w),
                                             static_cast<const double*>(c), kind, n,
                                             static_cast<double2*>(prm), bad);
    return hipGetLastError();
}

hipError_t launch_validate_T(int dtype, hipStream_t st, const void* T, int64_t count, int* bad,
                             bool positive)
{
    const int64_t want = (count + 255) / 256;
    const int grid = (int)(want < 8192 ? (want < 1 ? 1 : want) : 8192);
    if (dtype == 0)
        k_validate_T<float><<<grid, 256, 0, st>>>(static_cast<const float*>(T), count, bad,
                                                  positive);
    else
        k_validate_T<double><<<grid, 256, 0, st>>>(static_cast<const double*>(T), count, bad,
                                                   positive);
    return hipGetLastError();
}

hipError_t launch_materialize(int dtype, hipStream_t st, const int16_t* jpair, const void* xpair,
                              int64_t n, int m, const double* R, const double* r, void* X)
{
    const int64_t want = (n * m + 255) / 256;
    const int grid = (int)(want < 8192 ? (want < 1 ? 1 : want) : 8192);
    const int* jp = reinterpret_cast<const int*>(jpair);
    if (dtype == 0)
        k_materialize<float><<<grid, 256, 0, st>>>(jp, static_cast<const float2*>(xpair), n, m, R,
                                                   r, static_cast<float*>(X));
    else
        k_materialize<double><<<grid, 256, 0, st>>>(jp, static_cast<const double2*>(xpair), n, m,
                                                    R, r, static_cast<double*>(X));
    return hipGetLastError();
}

}  // namespace ra
