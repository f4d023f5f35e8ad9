// Column sum of block partials in a fixed order, shared by the plain column
// reduction and the device price loop so that both give the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ra {

// Sum of column j of an nb x ncols row-major array: thread t of a 256-thread
// block adds rows t, t + 256, ...; a tree over the threads follows.  Every
// thread of the block must call it; the sum is returned to thread 0.
__device__ __forceinline__ double column_sum(const double* __restrict__ partial, int nb,
                                             int ncols, int j, double* red)
{
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partial[(int64_t)b * ncols + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    return red[0];
}

}  // namespace ra
