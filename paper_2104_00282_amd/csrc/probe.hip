// Streaming-read probe: the attainable read bandwidth of this device for a
// buffer, to set the dual kernel's roofline fraction against a measured
// ceiling as well as the published peak.  Every 16 bytes are loaded once
// with non-temporal loads and summed; the sum is stored only if it equals an
// impossible value, which keeps the loads without writing.
#include "ra_internal.hpp"
#include "resalloc.h"

#include <hip/hip_runtime.h>

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

}  // namespace

using ra::fail;

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
