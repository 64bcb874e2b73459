// ACE kernels (Eq. 18, App. A) on the small matrix: symmetrization,
// Cholesky, triangular inverse and the energy's sum of squares.  The
// tall-skinny products over the grid are in k_ace_mfma.hip.
//
// All orbital arrays are orbital-major (rows of length n_grid).
#include "sea_internal.h"
#include "k_ace.h"

namespace {

// ---------------------------------------------------------------------------
// small-matrix kernels (one workgroup)

__global__ void k_symmetrize(const double* __restrict__ M, int n, double* __restrict__ Mb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int i = t / n, j = t % n;
    Mb[t] = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
}

constexpr int CH_BS = 1024;

// Wave-wide sum (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Left-looking Cholesky (lower, row-major) of A into L, one workgroup of 16
// wavefronts: for column j, wavefront 0 forms the pivot from row j, then the
// 16 wavefronts take the rows below it in turn, each row's dot product over
// k < j split across the 64 lanes.  flag[0] = 1-based index of the first
// non-positive pivot, 0 on success.
__global__ __launch_bounds__(CH_BS) void k_cholesky(const double* __restrict__ A, int n, double* __restrict__ L,
                                                    int* __restrict__ flag) {
    __shared__ double piv;
    __shared__ int bad;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = threadIdx.x; t < n * n; t += CH_BS) L[t] = 0.0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (wave == 0) {
            double s = 0.0;
            for (int k = lane; k < j; k += 64) s += L[(size_t)j * n + k] * L[(size_t)j * n + k];
            s = wave_sum(s);
            if (lane == 0) {
                const double d = A[(size_t)j * n + j] - s;
                if (d > 0.0) {
                    piv = sqrt(d);
                    L[(size_t)j * n + j] = piv;
                } else {
                    bad = j + 1;
                }
            }
        }
        __syncthreads();
        if (bad) break;
        const double ljj = piv;
        for (int i = j + 1 + wave; i < n; i += CH_BS / 64) {
            double s = 0.0;
            for (int k = lane; k < j; k += 64) s += L[(size_t)i * n + k] * L[(size_t)j * n + k];
            s = wave_sum(s);
            if (lane == 0) L[(size_t)i * n + j] = (A[(size_t)i * n + j] - s) / ljj;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) flag[0] = bad;
}

// X = L^{-1} (lower): workgroup c (one wavefront) forms column c by forward
// substitution, x_i = (delta_ic - sum_{c<=k<i} L[i][k] x_k) / L[i][i], with
// the column kept in LDS and each dot product split across the lanes.
constexpr int TR_MAX = 4096;
__global__ __launch_bounds__(64) void k_trtri_lower(const double* __restrict__ L, int n, double* __restrict__ X) {
    __shared__ double x[TR_MAX];
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
    for (int i = lane; i < c; i += 64) X[(size_t)i * n + c] = 0.0;
    for (int i = c; i < n; ++i) {
        double s = 0.0;
        for (int k = c + lane; k < i; k += 64) s += L[(size_t)i * n + k] * x[k];
        s = wave_sum(s);
        const double xi = ((i == c ? 1.0 : 0.0) - s) / L[(size_t)i * n + i];
        if (lane == 0) {
            x[i] = xi;
            X[(size_t)i * n + c] = xi;
        }
        __syncthreads();
    }
}

constexpr int SQ_BS = 256;

__global__ __launch_bounds__(SQ_BS) void k_neg_sum_squares(const double* __restrict__ S, int mn, double* out) {
    __shared__ double red[SQ_BS / 64];
    double s = 0.0;
    for (int t = threadIdx.x; t < mn; t += SQ_BS) s += S[t] * S[t];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < SQ_BS / 64; ++w) t += red[w];
        out[0] = -t;
    }
}

}  // namespace

// ---------------------------------------------------------------------------

hipError_t ace_symmetrize(const double* M, int n, double* Mb, hipStream_t s) {
    hipLaunchKernelGGL(k_symmetrize, dim3((n * n + 255) / 256), dim3(256), 0, s, M, n, Mb);
    return hipGetLastError();
}

hipError_t ace_cholesky(const double* A, int n, double* L, int* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(CH_BS), 0, s, A, n, L, flag);
    return hipGetLastError();
}

hipError_t ace_trtri(const double* L, int n, double* X, hipStream_t s) {
    if (n > TR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_trtri_lower, dim3(n), dim3(64), 0, s, L, n, X);
    return hipGetLastError();
}

hipError_t ace_neg_sum_squares(const double* S, int mn, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_neg_sum_squares, dim3(1), dim3(SQ_BS), 0, s, S, mn, out);
    return hipGetLastError();
}
