// Epsilon-driven domains (Eq. 16) and absolute-overlap pair screening
// (Eq. 17): the two grid reductions they need.
//
//   k_eps_marginals  m[o][a][k] = sum over the plane perpendicular to axis a
//                    at index k of |phi_o|^2 (one workgroup per entry);
//   k_eps_overlap    S_p = dV sum over pair p's box of |phi_i phi_j|
//                    (one workgroup per candidate pair, wrapped indices).
//
// The interval search, the box intersections and the screening decision are
// host work (sea_api.hip); every sum here accumulates in FP64.
#include "sea_internal.h"

namespace {

constexpr int EP_BS = 256;

__device__ __forceinline__ double ld_phi(const void* phi, int f32, size_t off) {
    return f32 ? (double)(((const float*)phi)[off]) : ((const double*)phi)[off];
}

__device__ __forceinline__ int wrap_i(int k, int N) {
    int m = k % N;
    return m < 0 ? m + N : m;
}

__device__ __forceinline__ double block_sum_d(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < EP_BS / 64; ++w) t += red[w];
    return t;  // valid in thread 0
}

// grid (max N, 3, n_occ)
__global__ __launch_bounds__(EP_BS) void k_eps_marginals(const void* __restrict__ phi, int f32, int N0, int N1, int N2,
                                                         int nmax, double* __restrict__ m) {
    __shared__ double red[EP_BS / 64];
    const int k = blockIdx.x, a = blockIdx.y, o = blockIdx.z;
    const int Na = a == 0 ? N0 : (a == 1 ? N1 : N2);
    if (k >= Na) return;
    const size_t Ng = (size_t)N0 * N1 * N2;
    const size_t base = (size_t)o * Ng;
    // the plane's two free axes: (u, v) with u fastest in memory
    const int Nu = a == 0 ? N1 : N0, Nv = a == 2 ? N1 : N2;
    const long n = (long)Nu * Nv;
    double s = 0.0;
    for (long t = threadIdx.x; t < n; t += EP_BS) {
        const int u = (int)(t % Nu), v = (int)(t / Nu);
        size_t g;
        if (a == 0) g = ((size_t)v * N1 + u) * N0 + k;        // (y, z) free, x = k
        else if (a == 1) g = ((size_t)v * N1 + k) * N0 + u;   // (x, z) free, y = k
        else g = ((size_t)k * N1 + v) * N0 + u;               // (x, y) free, z = k
        const double f = ld_phi(phi, f32, base + g);
        s += f * f;
    }
    s = block_sum_d(s, red);
    if (threadIdx.x == 0) m[((size_t)o * 3 + a) * nmax + k] = s;
}

// one workgroup per candidate pair
__global__ __launch_bounds__(EP_BS) void k_eps_overlap(const void* __restrict__ phi, int f32, int N0, int N1, int N2,
                                                       double dV, const sea_pair* __restrict__ pairs,
                                                       double* __restrict__ S) {
    __shared__ double red[EP_BS / 64];
    const sea_pair P = pairs[blockIdx.x];
    const size_t Ng = (size_t)N0 * N1 * N2;
    const size_t oi = (size_t)P.i * Ng, oj = (size_t)P.j * Ng;
    const long n = (long)P.n[0] * P.n[1] * P.n[2];
    double s = 0.0;
    for (long t = threadIdx.x; t < n; t += EP_BS) {
        const int x = (int)(t % P.n[0]), y = (int)((t / P.n[0]) % P.n[1]), z = (int)(t / ((long)P.n[0] * P.n[1]));
        const size_t g = ((size_t)wrap_i(P.lo[2] + z, N2) * N1 + wrap_i(P.lo[1] + y, N1)) * N0 + wrap_i(P.lo[0] + x, N0);
        s += fabs(ld_phi(phi, f32, oi + g) * ld_phi(phi, f32, oj + g));
    }
    s = block_sum_d(s, red);
    if (threadIdx.x == 0) S[blockIdx.x] = dV * s;
}

}  // namespace

hipError_t launch_eps_marginals(const void* phi, int f32, const int* N, int n_occ, int nmax, double* m,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_eps_marginals, dim3(nmax, 3, n_occ), dim3(EP_BS), 0, s, phi, f32, N[0], N[1], N[2], nmax, m);
    return hipGetLastError();
}

hipError_t launch_eps_overlap(const void* phi, int f32, const int* N, double dV, const sea_pair* pairs, int n_pairs,
                              double* S, hipStream_t s) {
    if (n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eps_overlap, dim3(n_pairs), dim3(EP_BS), 0, s, phi, f32, N[0], N[1], N[2], dV, pairs, S);
    return hipGetLastError();
}
