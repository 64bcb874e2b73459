// Device helpers shared by the exx kernels (k_exx.hip, k_scatter.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

// k mod N in [0, N) for any k
__device__ __forceinline__ int wrap_idx(int k, int N) {
    int m = k % N;
    return m < 0 ? m + N : m;
}

// orbital value from an FP64 or FP32 array
__device__ __forceinline__ double load_phi(const void* phi, int f32, size_t off) {
    return f32 ? (double)(((const float*)phi)[off]) : ((const double*)phi)[off];
}
