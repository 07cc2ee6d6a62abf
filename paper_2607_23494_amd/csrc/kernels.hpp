// Small utility kernels shared by the translation units.
#pragma once

#include "common.hpp"

namespace hermes {

// Fill with a value.  Used instead of hipMemsetAsync so that work captured
// into a HIP graph contains kernels only.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill(T* __restrict__ p, int64_t n, T v) {
    const int64_t stride = int64_t(gridDim.x) * kThreads;
    for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) p[i] = v;
}

template <typename T>
inline void launch_fill(T* p, int64_t n, T v, hipStream_t stream) {
    if (n <= 0) return;
    const int64_t want = (n + kThreads - 1) / kThreads;
    const int blocks = int(want < 4096 ? want : 4096);
    hipLaunchKernelGGL((k_fill<T>), dim3(blocks), dim3(kThreads), 0, stream, p, n, v);
}

// Order the LDS accesses of one wavefront: its lanes' earlier writes are
// visible to its later reads (a wavefront's LDS operations complete in
// order; the fences keep the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Block-wide float64 sum; every thread passes its value, thread 0 gets the
// total.  `scratch` holds kThreads doubles.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    scratch[threadIdx.x] = v;
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) scratch[threadIdx.x] += scratch[threadIdx.x + s];
        __syncthreads();
    }
    const double r = scratch[0];
    __syncthreads();
    return r;
}

}  // namespace hermes
