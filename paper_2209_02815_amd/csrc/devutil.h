// Small device helpers shared by the h1w kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace h1w {

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Sum over a 64-lane wavefront; lane 0 holds the result. Fixed order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Sum over a block of NT threads (NT multiple of 64); thread 0 holds the result.
// sh must hold NT/64 doubles. Deterministic for a fixed launch shape.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) r += sh[w];
    }
    __syncthreads();
    return r;
}

}  // namespace h1w
