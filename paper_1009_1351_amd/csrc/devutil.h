// Small device helpers: deterministic block reductions and launch checks.
#pragma once
#include <hip/hip_runtime.h>

namespace tnlm {

constexpr int kBlock = 256;

// Sum of one double per thread over a 256-thread block, in a fixed order.
// Every thread returns the total; all threads must call it. Uses the first 4
// doubles of sh.
__device__ inline double block_sum_256(double v, double *sh) {
    static_assert(kBlock == 256, "four waves");
    // butterfly within the wave: both lanes of a pair form the same sum, so
    // every lane ends with the same value, in a fixed order; then the four
    // waves' sums in a fixed order
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    if ((t & 63) == 0) sh[t >> 6] = v;
    __syncthreads();
    const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
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
