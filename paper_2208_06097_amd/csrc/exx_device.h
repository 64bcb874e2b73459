// Device helpers shared by the exx kernels (k_exx.hip, k_scatter.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

// k mod N in [0, N) for any k
__device__ __forceinline__ int wrap_idx(int k, int N) {
    int m = k % N;
    return m < 0 ? m + N : m;
}

// A pointer read from device memory (a cell record) is generic to the
// compiler, and loads through it become flat loads, which also count on the
// scalar-load counter and so serialize behind scalar loads; the arrays these
// pointers address are always in global memory.
template <typename T>
using global_ptr = __attribute__((address_space(1))) const T*;
template <typename T>
__device__ __forceinline__ global_ptr<T> as_global(const T* p) {
    return (global_ptr<T>)p;
}

// orbital value from an FP64 or FP32 array
__device__ __forceinline__ double load_phi(const void* phi, int f32, size_t off) {
    return f32 ? (double)as_global((const float*)phi)[off] : as_global((const double*)phi)[off];
}

// Multipole potential (Eq. 10) at displacement d from the pair's monomial
// coefficients cf: 84 of them, for dx^a dy^b dz^c with a + b + c <= 6, a the
// outer index, then b, then c.  The degree-l part P_l is homogeneous, so
// sum_l P_l(d) |d|^-(2l+1) = P(d / |d|^2) / |d| with P the whole polynomial:
// one evaluation at the inverted point, no split by degree and few registers.
__device__ __forceinline__ double me_inverted_potential(const double* __restrict__ cf, double dx, double dy, double dz) {
    const double r2inv = 1.0 / (dx * dx + dy * dy + dz * dz);
    const double u = dx * r2inv, v = dy * r2inv, w = dz * r2inv;
    double s = 0.0, ua = 1.0;
    int t = 0;
#pragma unroll
    for (int a = 0; a <= 6; ++a) {
        double vb = ua;
#pragma unroll
        for (int b = 0; b <= 6 - a; ++b) {
            double m = vb;
#pragma unroll
            for (int c = 0; c <= 6 - a - b; ++c) {
                s += cf[t++] * m;
                m *= w;
            }
            vb *= v;
        }
        ua *= u;
    }
    return s * sqrt(r2inv);
}
