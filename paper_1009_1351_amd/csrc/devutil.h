// Small device helpers: deterministic block reductions and launch checks.
#pragma once
#include <hip/hip_runtime.h>

namespace tnlm {

constexpr int kBlock = 256;

// Sum of one double per thread over a 256-thread block, fixed tree order.
// Every thread returns the total. Uses 256 doubles of shared memory.
__device__ inline double block_sum_256(double v, double *sh) {
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    sh[t] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// Sum of partials[0..n) in a fixed order (strided per-thread sums, then the
// block tree). Identical in every block that calls it with the same input.
__device__ inline double block_sum_array(const double *partials, int n, double *sh) {
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    double acc = 0.0;
    for (int k = t; k < n; k += kBlock) acc += partials[k];
    return block_sum_256(acc, sh);
}

__device__ inline bool skip_now(const int *skip) { return skip != nullptr && *skip != 0; }

// Values the caller knows to be equal in every lane of the wave (block
// indices, slice descriptors), moved to scalar registers.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ const float *wave_uniform(const float *p) {
    const unsigned long long u = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (const float *)(((unsigned long long)hi << 32) | lo);
}

}  // namespace tnlm
