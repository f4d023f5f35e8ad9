// Streaming-read probe: the attainable read bandwidth of this device for a
// buffer, to set the dual kernel's roofline fraction against a measured
// ceiling as well as the published peak.  Every 16 bytes are loaded once
// with non-temporal loads and summed; the sum is stored only if it equals an
// impossible value, which keeps the loads without writing.
#include "ra_internal.hpp"
#include "resalloc.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace {

typedef float probe_f4 __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) k_stream_read(const probe_f4* __restrict__ a, int64_t n4,
                                                     float* __restrict__ sink)
{
    float s = 0.f;
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) {
        const probe_f4 v = __builtin_nontemporal_load(a + i);
        s += (v.x + v.y) + (v.z + v.w);
    }
    if (s == -1234.5f) sink[0] = s;
}

// First-vertex scan probe (§4.1: the first envelope vertex is the
// resource with the largest a_ij / p_j), to compare two mappings of the
// scan onto a wavefront over the same LDS-staged 64-row tiles of an n x 64
// matrix: one lane per job scanning its whole row, or G lanes per job each
// scanning a contiguous 64/G part, joined by a shuffle argmax (lower index
// on equal keys).  Both store each job's vertex.
constexpr int PM = 64, PS = PM + 4;  // row length, padded LDS stride

struct ProbeInv {
    float inv[PM];
};

__device__ __forceinline__ void probe_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the 64 x 64 tile of rows row0.. as 1024 16-byte chunks, 16 per lane
__device__ __forceinline__ void probe_stage(const float* T, int64_t row0, float* tl, int lane)
{
    const probe_f4* src = reinterpret_cast<const probe_f4*>(T + row0 * PM);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int ch = lane + 64 * k;
        *reinterpret_cast<probe_f4*>(tl + (ch >> 4) * PS + 4 * (ch & 15)) =
            __builtin_nontemporal_load(src + ch);
    }
}

template <int G>
__global__ void __launch_bounds__(256) k_scan_probe(const float* __restrict__ T, int64_t ntiles,
                                                    ProbeInv pi, int16_t* __restrict__ j1)
{
    __shared__ __attribute__((aligned(16))) float tile[4][64 * PS];
    __shared__ float inv[PM];
    if (threadIdx.x < PM) inv[threadIdx.x] = pi.inv[threadIdx.x];
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int sub = lane % G, jl = lane / G;
    float* tl = tile[wv];
    for (int64_t t = (int64_t)blockIdx.x * 4 + wv; t < ntiles; t += (int64_t)gridDim.x * 4) {
        probe_stage(T, t * 64, tl, lane);
        probe_wave_sync();
#pragma unroll
        for (int step = 0; step < G; ++step) {
            const int job = step * (64 / G) + jl;
            const float* row = tl + job * PS;
            float best = 0.f;
            int jb = -1;
#pragma unroll
            for (int k = 0; k < PM / G; ++k) {
                const int j = sub * (PM / G) + k;
                const float key = row[j] * (G == 1 ? pi.inv[j] : inv[j]);
                const bool b = key > best;
                best = b ? key : best;
                jb = b ? j : jb;
            }
#pragma unroll
            for (int off = 1; off < G; off <<= 1) {
                const float ob = __shfl_xor(best, off);
                const int oj = __shfl_xor(jb, off);
                const bool take = (ob > best) || (ob == best && oj >= 0 && (jb < 0 || oj < jb));
                best = take ? ob : best;
                jb = take ? oj : jb;
            }
            if (sub == 0) j1[t * 64 + job] = (int16_t)jb;
        }
        probe_wave_sync();
    }
}

}  // namespace

using ra::fail;

extern "C" ra_status ra_probe_first_vertex_ms(ra_ctx* ctx, const float* T, int64_t n,
                                              const double* p, int32_t lanes_per_job,
                                              int32_t reps, int16_t* j1, double* ms)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!T || !p || !j1 || !ms || n < 64 || n % 64 != 0 || reps < 1 ||
        reinterpret_cast<uintptr_t>(T) % 16 != 0)
        return fail(ctx, RA_EINVAL, "T (16-byte aligned), n (a positive multiple of 64), p, j1, "
                                    "reps >= 1 and ms are required");
    if (!(lanes_per_job == 1 || lanes_per_job == 2 || lanes_per_job == 4 || lanes_per_job == 8 ||
          lanes_per_job == 16))
        return fail(ctx, RA_EINVAL, "lanes_per_job must be 1, 2, 4, 8 or 16");
    ProbeInv pi;
    for (int j = 0; j < PM; ++j) {
        if (!(p[j] > 0.0) || !std::isfinite(p[j]))
            return fail(ctx, RA_EINVAL, "p[%d] = %g must be positive and finite", j, p[j]);
        pi.inv[j] = 1.0f / (float)p[j];
    }
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    hipStream_t st = ctx->stream;
    const int64_t ntiles = n / 64;
    const int grid = ctx->cus * 2;
    auto launch = [&]() {
        switch (lanes_per_job) {
        case 1: k_scan_probe<1><<<grid, 256, 0, st>>>(T, ntiles, pi, j1); break;
        case 2: k_scan_probe<2><<<grid, 256, 0, st>>>(T, ntiles, pi, j1); break;
        case 4: k_scan_probe<4><<<grid, 256, 0, st>>>(T, ntiles, pi, j1); break;
        case 8: k_scan_probe<8><<<grid, 256, 0, st>>>(T, ntiles, pi, j1); break;
        default: k_scan_probe<16><<<grid, 256, 0, st>>>(T, ntiles, pi, j1); break;
        }
        return hipGetLastError();
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(ctx, RA_EDEVICE, "first-vertex probe: %s", hipGetErrorString(e));
    *ms = (double)t / reps;
    return RA_OK;
}

extern "C" ra_status ra_stream_read_ms(ra_ctx* ctx, const void* buf, int64_t bytes, int32_t reps,
                                       double* ms)
{
    if (!ctx || ctx->closed) return RA_EINVAL;
    if (!buf || !ms || bytes <= 0 || bytes % 16 != 0 || reps < 1 ||
        reinterpret_cast<uintptr_t>(buf) % 16 != 0)
        return fail(ctx, RA_EINVAL, "buf (16-byte aligned), bytes (> 0, multiple of 16), reps >= 1 and ms are required");
    RA_HIP(ctx, hipSetDevice(ctx->dev));
    hipStream_t st = ctx->stream;
    float* sink = nullptr;
    RA_HIP(ctx, hipMalloc(&sink, sizeof(float)));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const int grid = ctx->cus * 8;
    const int64_t n4 = bytes / 16;
    const auto* a = static_cast<const probe_f4*>(buf);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
        k_stream_read<<<grid, 256, 0, st>>>(a, n4, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) {
        k_stream_read<<<grid, 256, 0, st>>>(a, n4, sink);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    if (e != hipSuccess) return fail(ctx, RA_EDEVICE, "stream read probe: %s", hipGetErrorString(e));
    *ms = (double)t / reps;
    return RA_OK;
}
