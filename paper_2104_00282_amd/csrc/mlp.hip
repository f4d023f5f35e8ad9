// Learned warm start: problem features, a small multilayer perceptron with
// hand-written forward, backward and Adam kernels, and its host API.
//
// The network maps per-problem features to log-prices; it is trained on
// prices found by the price-discovery loop and only provides a starting
// point for that loop (the certificate and stopping rule are unchanged).
#include "ra_internal.hpp"
#include "ra_kernels.h"
#include "resalloc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

using ra::fail;

struct ra_mlp {
    ra_ctx* ctx = nullptr;
    int D = 0, H = 0, O = 0;  // in_dim, hidden, out_dim
    int64_t np = 0;           // parameter count
    int64_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0;
    float* params = nullptr;  // device, flat
    float* grads = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    float* norm = nullptr;    // device: x_mean (D), x_std (D), y_mean (O), y_std (O)
    std::vector<float> hnorm;
    int64_t step = 0;
    int cap = 0;              // batch capacity of the activation buffers
    float *Xs = nullptr, *H1 = nullptr, *H2 = nullptr, *Ys = nullptr, *dY = nullptr,
          *dA = nullptr, *dB = nullptr;
    double* dloss = nullptr;
    double* hloss = nullptr;
    float* feat = nullptr;    // device scratch for one feature row and one output row
    float* hy = nullptr;      // pinned host: one predicted output row (O floats)
    unsigned* hflag = nullptr;  // pinned host: completion flag of the one-row forward
};

namespace {

constexpr int FEAT_SAMPLE = 8192;

// ------------------------------------------------------------------ GEMM --
// C[i][j] = act(sum_k A(i, k) B(k, j) + bias[j]),
// A(i, k) = A[i * sai + k * sak], B(k, j) = B[k * sbk + j * sbj]; 64 x 64
// output tiles, 16-deep K steps through LDS, 4 x 4 outputs per thread.
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              int64_t sai, int64_t sak,
                                              const float* __restrict__ B, int64_t sbk,
                                              int64_t sbj, float* __restrict__ C, int64_t ldc,
                                              const float* __restrict__ bias, int relu)
{
    __shared__ float As[16][65];
    __shared__ float Bs[16][65];
    const int tid = threadIdx.x;
    const int ty = tid >> 4, tx = tid & 15;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    float acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.f;
    for (int k0 = 0; k0 < K; k0 += 16) {
        for (int e = tid; e < 64 * 16; e += 256) {
            const int ii = e >> 4, kk = e & 15;
            const int i = i0 + ii, k = k0 + kk;
            As[kk][ii] = (i < M && k < K) ? A[i * sai + k * sak] : 0.f;
            const int jj = e & 63, kb = e >> 6;
            const int j = j0 + jj, k2 = k0 + kb;
            Bs[kb][jj] = (j < N && k2 < K) ? B[k2 * sbk + j * sbj] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int i = i0 + ty * 4 + r, j = j0 + tx * 4 + c;
            if (i < M && j < N) {
                float v = acc[r][c] + (bias ? bias[j] : 0.f);
                if (relu) v = v > 0.f ? v : 0.f;
                C[i * ldc + j] = v;
            }
        }
}

void gemm(hipStream_t st, int M, int N, int K, const float* A, int64_t sai, int64_t sak,
          const float* B, int64_t sbk, int64_t sbj, float* C, int64_t ldc, const float* bias,
          int relu)
{
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    k_gemm<<<grid, 256, 0, st>>>(M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, bias, relu);
}

// x_s = (x - mean) / std, row-major batch x D
__global__ void k_standardize(const float* __restrict__ X, const float* __restrict__ mean,
                              const float* __restrict__ sd, int64_t total, int D,
                              float* __restrict__ Xs)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % D);
        Xs[e] = (X[e] - mean[j]) / sd[j];
    }
}

// y = y_s * std + mean
__global__ void k_destandardize(const float* __restrict__ Ys, const float* __restrict__ mean,
                                const float* __restrict__ sd, int64_t total, int D,
                                float* __restrict__ Y)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int j = (int)(e % D);
        Y[e] = Ys[e] * sd[j] + mean[j];
    }
}

// Mean squared error of standardised outputs and its gradient:
// L = sum (y_s - t_s)^2 / (B O), dY = 2 (y_s - t_s) / (B O); one block,
// fixed-order reduction.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ Ys,
                                             const float* __restrict__ Ty,
                                             const float* __restrict__ mean,
                                             const float* __restrict__ sd, int B, int O,
                                             float* __restrict__ dY, double* __restrict__ loss)
{
    __shared__ double red[256];
    const int total = B * O;
    const float scale = 2.f / (float)total;
    double s = 0.0;
    for (int e = threadIdx.x; e < total; e += 256) {
        const int j = e % O;
        const float ts = (Ty[e] - mean[j]) / sd[j];
        const float d = Ys[e] - ts;
        dY[e] = scale * d;
        s += (double)d * (double)d;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (double)total;
}

// dZ = dA * (act > 0), in place
__global__ void k_relu_back(float* __restrict__ dA, const float* __restrict__ act, int64_t total)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        if (!(act[e] > 0.f)) dA[e] = 0.f;
}

// db[j] = sum_b dZ[b][j], one thread per column, rows in order
__global__ void k_colsum(const float* __restrict__ dZ, int B, int N, float* __restrict__ db)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += dZ[(int64_t)b * N + j];
    db[j] = s;
}

// Adam with bias correction folded into the step size
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int64_t n, float lr_t, float b1, float b2, float eps)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[e];
        const float mi = b1 * m[e] + (1.f - b1) * gi;
        const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
        m[e] = mi;
        v[e] = vi;
        p[e] -= lr_t * mi / (sqrtf(vi) + eps);
    }
}

// --------------------------------------------------------------- features --
// Two kernels.  k_feat_gather: sample k < S is row floor(k n / S); each
// thread of many small blocks reads one sampled row (all m entries, so the
// scattered row reads are spread over many compute units) and its packed
// utility, writes the 32-bit key (kind << 31) | bits(value) of every entry
// to keys[j][k] (values are >= 0, so key order is (kind, value) order and
// the low 31 bits are the value), and each block writes its count of log
// jobs and its weight-histogram counts.  k_feat_select, block j < m: column
// j's keys from memory into LDS; the nearest-rank quantiles of each kind are
// the keys of given global rank in that order, found by a radix select (4
// passes of 8 bits, all six ranks at once) instead of a full sort; the
// column's mean is the FP64 sum of the values the keys hold (each thread its
// keys in order, then waves and the block in a fixed order).  Block m: the
// weight histograms from the block counts.
constexpr int FEAT_GATHER_THREADS = 64;
constexpr int FEAT_GATHER_BLOCKS = FEAT_SAMPLE / FEAT_GATHER_THREADS;

// Layout of the features scratch (ctx->feat_ws): keys [64][FEAT_SAMPLE],
// then per gather block one log-job count and 16 histogram counts.
constexpr size_t FEAT_KEYS_BYTES = sizeof(unsigned) * 64 * FEAT_SAMPLE;
constexpr size_t FEAT_CNT_BYTES = sizeof(int) * 17 * FEAT_GATHER_BLOCKS;
constexpr size_t FEAT_WS_BYTES = FEAT_KEYS_BYTES + FEAT_CNT_BYTES;

__global__ void __launch_bounds__(FEAT_GATHER_THREADS) k_feat_gather(
    const float* __restrict__ T, const float2* __restrict__ prm, int64_t n, int m,
    unsigned* __restrict__ keys, int* __restrict__ cnts)
{
    __shared__ int hc[17];
    const int S = (int)(n < FEAT_SAMPLE ? n : FEAT_SAMPLE);
    const int tid = threadIdx.x;
    const int k = blockIdx.x * FEAT_GATHER_THREADS + tid;
    if (tid < 17) hc[tid] = 0;
    __syncthreads();
    const bool on = k < S;
    const int64_t i = on ? ((int64_t)k * n) / S : 0;
    const float2 wc = on ? prm[i] : make_float2(0.f, 0.f);
    const unsigned kind = __builtin_signbit(wc.y) ? 0u : 1u;
    if (on) {
        int bin = (int)floorf((wc.x - 0.5f) / 0.1875f);
        bin = bin < 0 ? 0 : (bin > 7 ? 7 : bin);
        atomicAdd(&hc[kind * 8 + bin], 1);
        if (kind == 0u) atomicAdd(&hc[16], 1);
    }
    const float* row = T + i * m;
    for (int j = 0; j < m; ++j) {
        const float v = on ? row[j] : 0.f;  // consecutive entries: one cache line per row
        // -0 and +0 share a key
        const unsigned bits = v == 0.f ? 0u : __float_as_uint(v);
        if (on) keys[(int64_t)j * FEAT_SAMPLE + k] = (kind << 31) | (bits & 0x7fffffffu);
    }
    __syncthreads();
    if (tid < 17) cnts[blockIdx.x * 17 + tid] = hc[tid];
}

__global__ void __launch_bounds__(1024) k_feat_select(const unsigned* __restrict__ keys,
                                                      const int* __restrict__ cnts, int64_t n,
                                                      int m, const double* __restrict__ R,
                                                      float* __restrict__ feat)
{
    __shared__ unsigned key[FEAT_SAMPLE];
    __shared__ unsigned hist[2][6][256];
    __shared__ unsigned tpre[6], trank[6];
    __shared__ int tvalid[6], n0s;
    __shared__ double wsum[16];
    const int S = (int)(n < FEAT_SAMPLE ? n : FEAT_SAMPLE);
    const int nb = (S + FEAT_GATHER_THREADS - 1) / FEAT_GATHER_THREADS;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int j = blockIdx.x;
    if (j == m) {
        // wave b < 16: bin b of the weight histograms, its lanes striding
        // over the gather blocks (integer sums)
        if (wv < 16) {
            int c = 0;
            for (int b = lane; b < nb; b += 64) c += cnts[b * 17 + wv];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
            if (lane == 0) feat[8 * m + wv] = (float)c / (float)S;
        }
        return;
    }
    // the column's keys, all loads of a thread issued before their stores
    {
        unsigned v[FEAT_SAMPLE / 1024];
#pragma unroll
        for (int u = 0; u < FEAT_SAMPLE / 1024; ++u) {
            const int k = tid + 1024 * u;
            v[u] = k < S ? keys[(int64_t)j * FEAT_SAMPLE + k] : 0u;
        }
        double cs = 0.0;
#pragma unroll
        for (int u = 0; u < FEAT_SAMPLE / 1024; ++u) {
            const int k = tid + 1024 * u;
            if (k < S) key[k] = v[u];
            cs += (double)__uint_as_float(v[u] & 0x7fffffffu);  // 0 past S
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) cs += __shfl_xor(cs, off);
        if (lane == 0) wsum[wv] = cs;
    }
    // wave 0: the number of log jobs (lanes stride over the gather blocks,
    // then a butterfly)
    if (wv == 0) {
        int c = 0;
        for (int b = lane; b < nb; b += 64) c += cnts[b * 17 + 16];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
        if (lane == 0) n0s = c;
    }
    __syncthreads();
    if (tid == 0) {
        const int n0 = n0s;
        const double qs[3] = {0.1, 0.5, 0.9};
        for (int kind = 0; kind < 2; ++kind) {
            const int base = kind == 0 ? 0 : n0;
            const int cntk = kind == 0 ? n0 : S - n0;
            for (int q = 0; q < 3; ++q) {
                const int t = 3 * kind + q;
                const int idx = cntk > 0 ? (int)floor(qs[q] * (double)(cntk - 1) + 0.5) : 0;
                tvalid[t] = cntk > 0 ? 1 : 0;
                trank[t] = (unsigned)(base + idx);
                tpre[t] = 0u;
            }
        }
    }
    for (int e = tid; e < 6 * 256; e += 1024) (&hist[0][0][0])[e] = 0u;
    __syncthreads();
    for (int pass = 0; pass < 4; ++pass) {
        const int shift = 24 - 8 * pass;
        const unsigned hmask = pass == 0 ? 0u : (0xffffffffu << (shift + 8));
        unsigned(*hs)[256] = hist[pass & 1];
        // ranks whose key prefixes agree share one histogram (every thread
        // forms the grouping itself)
        int grp[6];
        unsigned pre[6];
#pragma unroll
        for (int t = 0; t < 6; ++t) {
            pre[t] = tpre[t];
            grp[t] = t;
        }
#pragma unroll
        for (int t = 1; t < 6; ++t)
#pragma unroll
            for (int u = t - 1; u >= 0; --u)
                if (grp[u] == u && pre[u] == pre[t]) grp[t] = u;
        for (int k = tid; k < S; k += 1024) {
            const unsigned kv = key[k];
            const unsigned d = (kv >> shift) & 255u;
#pragma unroll
            for (int t = 0; t < 6; ++t)
                if (grp[t] == t && (kv & hmask) == pre[t]) atomicAdd(&hs[t][d], 1u);
        }
        __syncthreads();
        if (wv < 6 && tvalid[wv]) {
            // wave t: the digit bin holding rank trank[t] of its prefix group
            const unsigned* h = hs[grp[wv]];
            unsigned c[4], ls = 0u;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                c[q] = h[4 * lane + q];
                ls += c[q];
            }
            unsigned x = ls;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const unsigned y = __shfl_up(x, off);
                if (lane >= off) x += y;
            }
            const unsigned excl = x - ls, r = trank[wv];
            if (excl <= r && r < x) {
                unsigned acc = excl;
                int bsel = 4 * lane + 3;
                for (int q = 0; q < 4; ++q) {
                    if (r < acc + c[q]) {
                        bsel = 4 * lane + q;
                        break;
                    }
                    acc += c[q];
                }
                tpre[wv] = tpre[wv] | ((unsigned)bsel << shift);
                trank[wv] = r - acc;
            }
        } else if (wv >= 6) {
            // the other histogram buffer, for the next pass
            for (int e = tid - 6 * 64; e < 6 * 256; e += 1024 - 6 * 64)
                (&hist[(pass + 1) & 1][0][0])[e] = 0u;
        }
        __syncthreads();
    }
    if (tid == 0) {
        for (int t = 0; t < 6; ++t)
            feat[8 * j + t] = tvalid[t] ? __uint_as_float(tpre[t] & 0x7fffffffu) : 0.f;
        feat[8 * j + 6] = (float)(R[j] / (double)n);
        double colsum = 0.0;
        for (int w = 0; w < 16; ++w) colsum += wsum[w];
        const double mean = colsum / (double)S;
        feat[8 * j + 7] = (float)log(mean > 1e-30 ? mean : 1e-30);
    }
}

// Forward of one feature row in one block (the warm-start prediction):
// standardise, two ReLU layers, output layer, de-standardise.  Each output
// row of a layer gets 16 consecutive threads; thread s reads the 16-byte
// chunks s, s + 16, ... of the row of W (rows are contiguous), so that 16
// threads read 256 consecutive bytes per load; the 16 partial sums meet by
// butterfly.  Rows not 16-byte aligned, or of a length not a multiple of 4,
// are read one float per thread at a time.  y receives the log-prices.
__global__ void __launch_bounds__(1024) k_forward1(const float* __restrict__ P, int64_t oW1,
                                                   int64_t ob1, int64_t oW2, int64_t ob2,
                                                   int64_t oW3, int64_t ob3,
                                                   const float* __restrict__ norm, int D, int H,
                                                   int O, const float* __restrict__ x,
                                                   float* __restrict__ y, unsigned* flag)
{
    extern __shared__ __attribute__((aligned(16))) float fsh[];
    float* xs = fsh;
    float* h1 = fsh + D;
    float* h2 = h1 + H;
    const int tid = threadIdx.x;
    for (int k = tid; k < D; k += blockDim.x) xs[k] = (x[k] - norm[k]) / norm[D + k];
    __syncthreads();
    constexpr int G = 16;
    const int s = tid & (G - 1);
    const int rows_per_pass = (int)blockDim.x / G;
    auto layer = [&](const float* W, const float* bias, const float* in, int K, int N, float* out,
                     bool relu) {
        const bool vec = (K & 3) == 0 && ((uintptr_t)W & 15) == 0 && ((uintptr_t)in & 15) == 0;
        for (int r0 = 0; r0 < N; r0 += rows_per_pass) {
            const int r = r0 + tid / G;
            float acc = 0.f;
            if (r < N) {
                const float* w = W + (int64_t)r * K;
                if (vec) {
                    const float4* w4 = reinterpret_cast<const float4*>(w);
                    const float4* i4 = reinterpret_cast<const float4*>(in);
                    const int K4 = K >> 2;
                    for (int c = s; c < K4; c += G) {
                        const float4 a = w4[c], b = i4[c];
                        acc += a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
                    }
                } else {
                    for (int k = s; k < K; k += G) acc += w[k] * in[k];
                }
            }
#pragma unroll
            for (int off = 1; off < G; off <<= 1) acc += __shfl_xor(acc, off);
            if (r < N && s == 0) {
                const float v = acc + bias[r];
                out[r] = relu ? fmaxf(v, 0.f) : v;
            }
        }
        __syncthreads();
    };
    layer(P + oW1, P + ob1, xs, D, H, h1, true);
    layer(P + oW2, P + ob2, h1, H, H, h2, true);
    layer(P + oW3, P + ob3, h2, H, O, xs, false);  // xs is free again
    const float* ym = norm + 2 * D;
    // wave 0 writes the outputs; with a flag, y is pinned host memory, made
    // visible (one wave's system fence) before the flag is raised
    if (tid < 64) {
        for (int k = tid; k < O; k += 64) y[k] = xs[k] * ym[O + k] + ym[k];
        if (flag) {
            __threadfence_system();
            if (tid == 0) __hip_atomic_store(flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        }
    }
}

int grid_for(int64_t total) { return (int)std::min<int64_t>(4096, (total + 255) / 256 + 1); }

ra_status ensure_cap(ra_mlp* N, int batch)
{
    ra_ctx* ctx = N->ctx;
    if (batch <= N->cap) return RA_OK;
    (void)hipFree(N->Xs);
    (void)hipFree(N->H1);
    (void)hipFree(N->H2);
    (void)hipFree(N->Ys);
    (void)hipFree(N->dY);
    (void)hipFree(N->dA);
    (void)hipFree(N->dB);
    N->Xs = N->H1 = N->H2 = N->Ys = N->dY = N->dA = N->dB = nullptr;
    N->cap = 0;
    const size_t b = (size_t)batch;
    RA_HIP(ctx, hipMalloc(&N->Xs, sizeof(float) * b * N->D));
    RA_HIP(ctx, hipMalloc(&N->H1, sizeof(float) * b * N->H));
    RA_HIP(ctx, hipMalloc(&N->H2, sizeof(float) * b * N->H));
    RA_HIP(ctx, hipMalloc(&N->Ys, sizeof(float) * b * N->O));
    RA_HIP(ctx, hipMalloc(&N->dY, sizeof(float) * b * N->O));
    RA_HIP(ctx, hipMalloc(&N->dA, sizeof(float) * b * N->H));
    RA_HIP(ctx, hipMalloc(&N->dB, sizeof(float) * b * N->H));
    N->cap = batch;
    return RA_OK;
}

// forward into Ys (standardised outputs); activations kept for backward
ra_status forward_std(ra_mlp* N, int B, const float* X)
{
    ra_ctx* ctx = N->ctx;
    hipStream_t st = ctx->stream;
    const float* xm = N->norm;
    const float* xs = N->norm + N->D;
    const int64_t tot = (int64_t)B * N->D;
    k_standardize<<<grid_for(tot), 256, 0, st>>>(X, xm, xs, tot, N->D, N->Xs);
    const float* P = N->params;
    // H1 = relu(Xs W1^T + b1)
    gemm(st, B, N->H, N->D, N->Xs, N->D, 1, P + N->oW1, 1, N->D, N->H1, N->H, P + N->ob1, 1);
    gemm(st, B, N->H, N->H, N->H1, N->H, 1, P + N->oW2, 1, N->H, N->H2, N->H, P + N->ob2, 1);
    gemm(st, B, N->O, N->H, N->H2, N->H, 1, P + N->oW3, 1, N->H, N->Ys, N->O, P + N->ob3, 0);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

// loss and gradients into N->grads
ra_status backward(ra_mlp* N, int B, const float* Ty)
{
    ra_ctx* ctx = N->ctx;
    hipStream_t st = ctx->stream;
    const float* ym = N->norm + 2 * N->D;
    const float* ysd = ym + N->O;
    const float* P = N->params;
    float* G = N->grads;
    const int D = N->D, H = N->H, O = N->O;
    k_mse<<<1, 256, 0, st>>>(N->Ys, Ty, ym, ysd, B, O, N->dY, N->dloss);
    // layer 3: dW3 = dY^T H2, db3 = colsum dY, dH2 = dY W3
    gemm(st, O, H, B, N->dY, 1, O, N->H2, H, 1, G + N->oW3, H, nullptr, 0);
    k_colsum<<<(O + 255) / 256, 256, 0, st>>>(N->dY, B, O, G + N->ob3);
    gemm(st, B, H, O, N->dY, O, 1, P + N->oW3, H, 1, N->dA, H, nullptr, 0);
    k_relu_back<<<grid_for((int64_t)B * H), 256, 0, st>>>(N->dA, N->H2, (int64_t)B * H);
    // layer 2
    gemm(st, H, H, B, N->dA, 1, H, N->H1, H, 1, G + N->oW2, H, nullptr, 0);
    k_colsum<<<(H + 255) / 256, 256, 0, st>>>(N->dA, B, H, G + N->ob2);
    gemm(st, B, H, H, N->dA, H, 1, P + N->oW2, H, 1, N->dB, H, nullptr, 0);
    k_relu_back<<<grid_for((int64_t)B * H), 256, 0, st>>>(N->dB, N->H1, (int64_t)B * H);
    // layer 1
    gemm(st, H, D, B, N->dB, 1, H, N->Xs, D, 1, G + N->oW1, D, nullptr, 0);
    k_colsum<<<(H + 255) / 256, 256, 0, st>>>(N->dB, B, H, G + N->ob1);
    RA_HIP(ctx, hipGetLastError());
    RA_HIP(ctx, hipMemcpyAsync(N->hloss, N->dloss, sizeof(double), hipMemcpyDeviceToHost, st));
    return RA_OK;
}

ra_status check_batch(ra_ctx* ctx, ra_mlp* N, int batch)
{
    if (!N || N->ctx != ctx) return fail(ctx, RA_EINVAL, "network is NULL or from another context");
    if (batch < 1 || batch > (1 << 20)) return fail(ctx, RA_EINVAL, "batch must be in [1, 2^20]");
    return RA_OK;
}

// splitmix64 + Box-Muller: He-normal weights
uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double unit(uint64_t& s) { return ((double)(splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

}  // namespace

namespace ra {

// Features of a problem into the device array feat (8 m + 16 floats).
ra_status features_into(ra_problem* P, float* feat)
{
    ra_ctx* ctx = P->ctx;
    if (!ctx->feat_ws) RA_HIP(ctx, hipMalloc(&ctx->feat_ws, FEAT_WS_BYTES));
    char* ws = static_cast<char*>(ctx->feat_ws);
    unsigned* keys = reinterpret_cast<unsigned*>(ws);
    int* cnts = reinterpret_cast<int*>(ws + FEAT_KEYS_BYTES);
    const int S = (int)std::min<int64_t>(P->n, FEAT_SAMPLE);
    const int nb = (S + FEAT_GATHER_THREADS - 1) / FEAT_GATHER_THREADS;
    k_feat_gather<<<nb, FEAT_GATHER_THREADS, 0, ctx->stream>>>(
        static_cast<const float*>(P->T), static_cast<const float2*>(P->prm), P->n, P->m, keys,
        cnts);
    k_feat_select<<<P->m + 1, 1024, 0, ctx->stream>>>(keys, cnts, P->n, P->m, P->Rdev,
                                                      feat);
    RA_HIP(ctx, hipGetLastError());
    return RA_OK;
}

// Predicted starting prices of P (host, m values).
ra_status predict_prices(ra_mlp* N, ra_problem* P, std::vector<double>& p0)
{
    ra_ctx* ctx = N->ctx;
    if (ensure_cap(N, 1) != RA_OK) return RA_ENOMEM;
    ra_status s = features_into(P, N->feat);
    if (s != RA_OK) return s;
    float* Y = N->feat + N->D;
    const size_t lds = sizeof(float) * ((size_t)N->D + 2 * (size_t)N->H);
    if (N->O <= N->D && lds <= 48 * 1024) {
        // the one-block forward writes the log-prices to pinned host memory
        // and raises a flag there, which the host polls
        __atomic_store_n(N->hflag, 0u, __ATOMIC_RELEASE);
        k_forward1<<<1, 1024, lds, ctx->stream>>>(N->params, N->oW1, N->ob1, N->oW2, N->ob2,
                                                  N->oW3, N->ob3, N->norm, N->D, N->H, N->O,
                                                  N->feat, N->hy, N->hflag);
        RA_HIP(ctx, hipGetLastError());
        s = wait_flag(ctx, N->hflag);
        if (s != RA_OK) return s;
    } else {
        s = forward_std(N, 1, N->feat);
        if (s != RA_OK) return s;
        const float* ym = N->norm + 2 * N->D;
        k_destandardize<<<1, 256, 0, ctx->stream>>>(N->Ys, ym, ym + N->O, N->O, N->O, Y);
        RA_HIP(ctx, hipMemcpyAsync(N->hy, Y, sizeof(float) * N->O, hipMemcpyDeviceToHost,
                                   ctx->stream));
        RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    p0.resize(N->O);
    for (int j = 0; j < N->O; ++j) p0[j] = std::exp((double)N->hy[j]);
    return RA_OK;
}

int mlp_out_dim(const ra_mlp* N) { return N->O; }
int mlp_in_dim(const ra_mlp* N) { return N->D; }

}  // namespace ra

extern "C" {

ra_status ra_features(ra_ctx* ctx, const ra_problem* prob, float* feat)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!prob || prob->ctx != ctx) return fail(ctx, RA_EINVAL, "problem is NULL or from another context");
    if (!feat) return fail(ctx, RA_EINVAL, "feat is required");
    if (prob->dt != 0 || prob->m > 64)
        return fail(ctx, RA_EUNSUPPORTED, "features need an FP32 problem with m <= 64");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    ra_status s = ra::features_into(const_cast<ra_problem*>(prob), feat);
    if (s != RA_OK) return s;
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return RA_OK;
}

ra_status ra_mlp_create(ra_ctx* ctx, int32_t in_dim, int32_t hidden, int32_t out_dim,
                        uint64_t seed, ra_mlp** out)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!out) return fail(ctx, RA_EINVAL, "out is NULL");
    if (in_dim < 1 || hidden < 1 || out_dim < 1 || in_dim > 65536 || hidden > 65536 ||
        out_dim > 65536)
        return fail(ctx, RA_EINVAL, "network sizes must be in [1, 65536]");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    ra_mlp* N = new (std::nothrow) ra_mlp();
    if (!N) return fail(ctx, RA_ENOMEM, "host allocation failed");
    N->ctx = ctx;
    N->D = in_dim;
    N->H = hidden;
    N->O = out_dim;
    const int64_t D = in_dim, H = hidden, O = out_dim;
    N->oW1 = 0;
    N->ob1 = N->oW1 + H * D;
    N->oW2 = N->ob1 + H;
    N->ob2 = N->oW2 + H * H;
    N->oW3 = N->ob2 + H;
    N->ob3 = N->oW3 + O * H;
    N->np = N->ob3 + O;
    auto bad = [&](hipError_t e) {
        ra_mlp_destroy(N);
        return fail(ctx, e == hipErrorOutOfMemory ? RA_ENOMEM : RA_EDEVICE, "ra_mlp_create: %s",
                    hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipMalloc(&N->params, sizeof(float) * N->np)) != hipSuccess) return bad(e);
    if ((e = hipMalloc(&N->grads, sizeof(float) * N->np)) != hipSuccess) return bad(e);
    if ((e = hipMalloc(&N->adam_m, sizeof(float) * N->np)) != hipSuccess) return bad(e);
    if ((e = hipMalloc(&N->adam_v, sizeof(float) * N->np)) != hipSuccess) return bad(e);
    if ((e = hipMalloc(&N->norm, sizeof(float) * 2 * (D + O))) != hipSuccess) return bad(e);
    if ((e = hipMalloc(&N->dloss, sizeof(double))) != hipSuccess) return bad(e);
    if ((e = hipMalloc(&N->feat, sizeof(float) * (D + O))) != hipSuccess) return bad(e);
    if ((e = hipHostMalloc((void**)&N->hloss, sizeof(double), hipHostMallocDefault)) != hipSuccess)
        return bad(e);
    if ((e = hipHostMalloc((void**)&N->hy, sizeof(float) * O, hipHostMallocCoherent)) != hipSuccess)
        return bad(e);
    if ((e = hipHostMalloc((void**)&N->hflag, sizeof(unsigned), hipHostMallocCoherent)) !=
        hipSuccess)
        return bad(e);
    std::vector<float> host(N->np, 0.f);
    uint64_t s = seed;
    auto fill = [&](int64_t off, int64_t rows, int64_t fan_in) {
        const double sd = std::sqrt(2.0 / (double)fan_in);
        for (int64_t k = 0; k < rows * fan_in; ++k) {
            const double u1 = unit(s), u2 = unit(s);
            host[off + k] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
        }
    };
    fill(N->oW1, H, D);
    fill(N->oW2, H, H);
    fill(N->oW3, O, H);
    N->hnorm.assign(2 * (D + O), 0.f);
    for (int64_t j = 0; j < D; ++j) N->hnorm[D + j] = 1.f;
    for (int64_t j = 0; j < O; ++j) N->hnorm[2 * D + O + j] = 1.f;
    std::vector<float> zeros(N->np, 0.f);
    if ((e = hipMemcpy(N->params, host.data(), sizeof(float) * N->np, hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
    if ((e = hipMemcpy(N->adam_m, zeros.data(), sizeof(float) * N->np, hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
    if ((e = hipMemcpy(N->adam_v, zeros.data(), sizeof(float) * N->np, hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
    if ((e = hipMemcpy(N->norm, N->hnorm.data(), sizeof(float) * N->hnorm.size(), hipMemcpyHostToDevice)) != hipSuccess) return bad(e);
    *out = N;
    return RA_OK;
}

ra_status ra_mlp_destroy(ra_mlp* N)
{
    if (!N) return RA_OK;
    if (N->ctx) {
        (void)hipSetDevice(N->ctx->dev);
        (void)hipStreamSynchronize(N->ctx->stream);
    }
    (void)hipFree(N->params);
    (void)hipFree(N->grads);
    (void)hipFree(N->adam_m);
    (void)hipFree(N->adam_v);
    (void)hipFree(N->norm);
    (void)hipFree(N->dloss);
    (void)hipFree(N->feat);
    (void)hipFree(N->Xs);
    (void)hipFree(N->H1);
    (void)hipFree(N->H2);
    (void)hipFree(N->Ys);
    (void)hipFree(N->dY);
    (void)hipFree(N->dA);
    (void)hipFree(N->dB);
    if (N->hloss) (void)hipHostFree(N->hloss);
    if (N->hy) (void)hipHostFree(N->hy);
    if (N->hflag) (void)hipHostFree(N->hflag);
    delete N;
    return RA_OK;
}

ra_status ra_mlp_num_params(const ra_mlp* N, int64_t* count)
{
    if (!N || !count) return RA_EINVAL;
    *count = N->np;
    return RA_OK;
}

ra_status ra_mlp_get_params(ra_mlp* N, float* host)
{
    if (!N || !host) return RA_EINVAL;
    ra_ctx* ctx = N->ctx;
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    RA_HIP(ctx, hipMemcpy(host, N->params, sizeof(float) * N->np, hipMemcpyDeviceToHost));
    return RA_OK;
}

ra_status ra_mlp_set_params(ra_mlp* N, const float* host)
{
    if (!N || !host) return RA_EINVAL;
    ra_ctx* ctx = N->ctx;
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    RA_HIP(ctx, hipMemcpy(N->params, host, sizeof(float) * N->np, hipMemcpyHostToDevice));
    return RA_OK;
}

ra_status ra_mlp_set_normalization(ra_mlp* N, const float* x_mean, const float* x_std,
                                   const float* y_mean, const float* y_std)
{
    if (!N || !x_mean || !x_std || !y_mean || !y_std) return RA_EINVAL;
    ra_ctx* ctx = N->ctx;
    for (int j = 0; j < N->D; ++j)
        if (!(x_std[j] > 0.f) || !std::isfinite(x_std[j]) || !std::isfinite(x_mean[j]))
            return fail(ctx, RA_EINVAL, "x_std[%d] must be > 0 and finite", j);
    for (int j = 0; j < N->O; ++j)
        if (!(y_std[j] > 0.f) || !std::isfinite(y_std[j]) || !std::isfinite(y_mean[j]))
            return fail(ctx, RA_EINVAL, "y_std[%d] must be > 0 and finite", j);
    std::memcpy(N->hnorm.data(), x_mean, sizeof(float) * N->D);
    std::memcpy(N->hnorm.data() + N->D, x_std, sizeof(float) * N->D);
    std::memcpy(N->hnorm.data() + 2 * N->D, y_mean, sizeof(float) * N->O);
    std::memcpy(N->hnorm.data() + 2 * N->D + N->O, y_std, sizeof(float) * N->O);
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    RA_HIP(ctx, hipMemcpy(N->norm, N->hnorm.data(), sizeof(float) * N->hnorm.size(),
                          hipMemcpyHostToDevice));
    return RA_OK;
}

ra_status ra_mlp_forward(ra_ctx* ctx, ra_mlp* N, int32_t batch, const float* X, float* Y)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    ra_status s = check_batch(ctx, N, batch);
    if (s != RA_OK) return s;
    if (!X || !Y) return fail(ctx, RA_EINVAL, "X and Y are required");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    if (ensure_cap(N, batch) != RA_OK) return RA_ENOMEM;
    s = forward_std(N, batch, X);
    if (s != RA_OK) return s;
    const float* ym = N->norm + 2 * N->D;
    const int64_t tot = (int64_t)batch * N->O;
    k_destandardize<<<grid_for(tot), 256, 0, ctx->stream>>>(N->Ys, ym, ym + N->O, tot, N->O, Y);
    RA_HIP(ctx, hipGetLastError());
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return RA_OK;
}

ra_status ra_mlp_gradients(ra_ctx* ctx, ra_mlp* N, int32_t batch, const float* X,
                           const float* Ty, float* grad_host, double* loss)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    ra_status s = check_batch(ctx, N, batch);
    if (s != RA_OK) return s;
    if (!X || !Ty) return fail(ctx, RA_EINVAL, "X and Ty are required");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    if (ensure_cap(N, batch) != RA_OK) return RA_ENOMEM;
    if ((s = forward_std(N, batch, X)) != RA_OK) return s;
    if ((s = backward(N, batch, Ty)) != RA_OK) return s;
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (grad_host)
        RA_HIP(ctx, hipMemcpy(grad_host, N->grads, sizeof(float) * N->np, hipMemcpyDeviceToHost));
    if (loss) *loss = *N->hloss;
    return RA_OK;
}

ra_status ra_mlp_train_step(ra_ctx* ctx, ra_mlp* N, int32_t batch, const float* X,
                            const float* Ty, float lr, double* loss)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    ra_status s = check_batch(ctx, N, batch);
    if (s != RA_OK) return s;
    if (!X || !Ty || !(lr > 0.f)) return fail(ctx, RA_EINVAL, "X, Ty and lr > 0 are required");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    if (ensure_cap(N, batch) != RA_OK) return RA_ENOMEM;
    if ((s = forward_std(N, batch, X)) != RA_OK) return s;
    if ((s = backward(N, batch, Ty)) != RA_OK) return s;
    N->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const double lr_t = lr * std::sqrt(1.0 - std::pow(b2, (double)N->step)) /
                        (1.0 - std::pow(b1, (double)N->step));
    k_adam<<<grid_for(N->np), 256, 0, ctx->stream>>>(N->params, N->grads, N->adam_m, N->adam_v,
                                                     N->np, (float)lr_t, (float)b1, (float)b2,
                                                     1e-8f);
    RA_HIP(ctx, hipGetLastError());
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (loss) *loss = *N->hloss;
    return RA_OK;
}

ra_status ra_mlp_save(const ra_mlp* N, const char* path)
{
    if (!N || !path) return RA_EINVAL;
    ra_ctx* ctx = N->ctx;
    std::vector<float> host(N->np);
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    RA_HIP(ctx, hipStreamSynchronize(ctx->stream));
    RA_HIP(ctx, hipMemcpy(host.data(), N->params, sizeof(float) * N->np, hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(ctx, RA_EINVAL, "cannot open %s", path);
    const char magic[8] = {'R', 'A', 'M', 'L', 'P', '0', '0', '1'};
    const int32_t dims[3] = {N->D, N->H, N->O};
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(dims, 4, 3, f) == 3 &&
              std::fwrite(N->hnorm.data(), 4, N->hnorm.size(), f) == N->hnorm.size() &&
              std::fwrite(host.data(), 4, host.size(), f) == host.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? RA_OK : fail(ctx, RA_EDEVICE, "writing %s failed", path);
}

ra_status ra_mlp_load(ra_ctx* ctx, const char* path, ra_mlp** out)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!path || !out) return fail(ctx, RA_EINVAL, "path and out are required");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(ctx, RA_EINVAL, "cannot open %s", path);
    char magic[8];
    int32_t dims[3];
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "RAMLP001", 8) != 0 ||
        std::fread(dims, 4, 3, f) != 3) {
        std::fclose(f);
        return fail(ctx, RA_EINVAL, "%s is not a saved network", path);
    }
    ra_mlp* N = nullptr;
    ra_status s = ra_mlp_create(ctx, dims[0], dims[1], dims[2], 0, &N);
    if (s != RA_OK) {
        std::fclose(f);
        return s;
    }
    std::vector<float> norm(N->hnorm.size()), host(N->np);
    const bool ok = std::fread(norm.data(), 4, norm.size(), f) == norm.size() &&
                    std::fread(host.data(), 4, host.size(), f) == host.size();
    std::fclose(f);
    if (!ok) {
        ra_mlp_destroy(N);
        return fail(ctx, RA_EINVAL, "%s is truncated", path);
    }
    const int D = N->D, O = N->O;
    s = ra_mlp_set_normalization(N, norm.data(), norm.data() + D, norm.data() + 2 * D,
                                 norm.data() + 2 * D + O);
    if (s == RA_OK) s = ra_mlp_set_params(N, host.data());
    if (s != RA_OK) {
        ra_mlp_destroy(N);
        return s;
    }
    *out = N;
    return RA_OK;
}

}  // extern "C"
