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

// Left-looking unblocked Cholesky (lower, row-major) of A into L; flag[0] =
// 1-based index of the first non-positive pivot, 0 on success.
__global__ __launch_bounds__(CH_BS) void k_cholesky(const double* __restrict__ A, int n, double* __restrict__ L,
                                                    int* __restrict__ flag) {
    __shared__ double red[CH_BS / 64 + 1];
    __shared__ int bad;
    for (int t = threadIdx.x; t < n * n; t += CH_BS) L[t] = 0.0;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = threadIdx.x; k < j; k += CH_BS) s += L[(size_t)j * n + k] * L[(size_t)j * n + k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = 0.0;
            for (int w = 0; w < CH_BS / 64; ++w) t += red[w];
            const double d = A[(size_t)j * n + j] - t;
            if (!(d > 0.0)) {
                bad = j + 1;
            } else {
                L[(size_t)j * n + j] = sqrt(d);
            }
        }
        __syncthreads();
        if (bad) break;
        const double ljj = L[(size_t)j * n + j];
        for (int i = j + 1 + threadIdx.x; i < n; i += CH_BS) {
            double t = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) t -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = t / ljj;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) flag[0] = bad;
}

// X = L^{-1} (lower), one thread per column, forward substitution.
__global__ void k_trtri_lower(const double* __restrict__ L, int n, double* __restrict__ X) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    for (int i = 0; i < c; ++i) X[(size_t)i * n + c] = 0.0;
    for (int i = c; i < n; ++i) {
        double t = (i == c) ? 1.0 : 0.0;
        for (int k = c; k < i; ++k) t -= L[(size_t)i * n + k] * X[(size_t)k * n + c];
        X[(size_t)i * n + c] = t / L[(size_t)i * n + i];
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
    hipLaunchKernelGGL(k_trtri_lower, dim3((n + 63) / 64), dim3(64), 0, s, L, n, X);
    return hipGetLastError();
}

hipError_t ace_neg_sum_squares(const double* S, int mn, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_neg_sum_squares, dim3(1), dim3(SQ_BS), 0, s, S, mn, out);
    return hipGetLastError();
}
