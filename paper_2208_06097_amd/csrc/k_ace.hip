// ACE kernels (Eq. 18-19, App. A): tall-skinny products over the grid,
// symmetrization, Cholesky and triangular inverse of the small matrix.
//
// All orbital arrays are orbital-major (rows of length n_grid).
#include "sea_internal.h"
#include "k_ace.h"

namespace {

template <typename T>
__device__ __forceinline__ double to_d(T v) { return (double)v; }

// ---------------------------------------------------------------------------
// C_part[s] = A B^T over the s-th slice of the long dimension.
// A: m x K row-major (lda = K), B: n x K row-major.

constexpr int NT_BM = 64, NT_BN = 64, NT_BK = 16, NT_BS = 256;

template <typename TA, typename TB>
__global__ __launch_bounds__(NT_BS) void k_gemm_nt_splitk(const TA* __restrict__ A, const TB* __restrict__ B,
                                                          int m, int n, long K, long kslice,
                                                          double* __restrict__ part) {
    __shared__ double As[NT_BK][NT_BM + 1];
    __shared__ double Bs[NT_BK][NT_BN + 1];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int j0 = blockIdx.x * NT_BN, i0 = blockIdx.y * NT_BM;
    const long kb = (long)blockIdx.z * kslice;
    const long ke = min(K, kb + kslice);
    double acc[4][4] = {};
    for (long k0 = kb; k0 < ke; k0 += NT_BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 16 * q;
            const long k = k0 + tx;
            As[tx][r] = (i0 + r < m && k < ke) ? to_d(A[(size_t)(i0 + r) * K + k]) : 0.0;
            Bs[tx][r] = (j0 + r < n && k < ke) ? to_d(B[(size_t)(j0 + r) * K + k]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < NT_BK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[kk][ty + 16 * q];
                b[q] = Bs[kk][tx + 16 * q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
        }
        __syncthreads();
    }
    double* P = part + (size_t)blockIdx.z * m * n;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + ty + 16 * p, j = j0 + tx + 16 * q;
            if (i < m && j < n) P[(size_t)i * n + j] = acc[p][q];
        }
}

__global__ void k_splitk_reduce(const double* __restrict__ part, int splits, int mn, double alpha,
                                double* __restrict__ C) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mn) return;
    double s = 0.0;
    for (int q = 0; q < splits; ++q) s += part[(size_t)q * mn + t];
    C[t] = alpha * s;
}

// ---------------------------------------------------------------------------
// C[i][g] = alpha * sum_k A(i,k) B[k][g], K small; A(i,k) = A[i*sai + k*sak].

constexpr int NN_BM = 64, NN_BN = 64, NN_BK = 16, NN_BS = 256;

template <typename TB, typename TC>
__global__ __launch_bounds__(NN_BS) void k_gemm_nn_smallk(const double* __restrict__ A, long sai, long sak,
                                                          const TB* __restrict__ B, int m, int K, long ncol,
                                                          double alpha, TC* __restrict__ C) {
    __shared__ double As[NN_BK][NN_BM + 1];
    __shared__ double Bs[NN_BK][NN_BN];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const long g0 = (long)blockIdx.x * NN_BN;
    const int i0 = blockIdx.y * NN_BM;
    double acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += NN_BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = ty + 16 * q;
            As[tx][r] = (i0 + r < m && k0 + tx < K) ? A[(i0 + r) * sai + (k0 + tx) * sak] : 0.0;
            // B tile: 16 rows of 64 columns, coalesced along g
            const int lid = threadIdx.x + NN_BS * q;
            const int kr = lid / NN_BN, gc = lid % NN_BN;
            Bs[kr][gc] = (k0 + kr < K && g0 + gc < ncol) ? to_d(B[(size_t)(k0 + kr) * ncol + g0 + gc]) : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < NN_BK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[kk][ty + 16 * q];
                b[q] = Bs[kk][tx + 16 * q];
            }
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
        }
        __syncthreads();
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = i0 + ty + 16 * p;
            const long g = g0 + tx + 16 * q;
            if (i < m && g < ncol) C[(size_t)i * ncol + g] = (TC)(alpha * acc[p][q]);
        }
}

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

int ace_splits(long K, int m, int n) {
    const long tiles = (long)((m + NT_BM - 1) / NT_BM) * ((n + NT_BN - 1) / NT_BN);
    long s = (2048 + tiles - 1) / tiles;
    const long maxs = (K + 4095) / 4096;
    if (s > maxs) s = maxs;
    if (s < 1) s = 1;
    return (int)s;
}

template <typename TA, typename TB>
hipError_t ace_gemm_nt(const TA* A, const TB* B, int m, int n, long K, double alpha, double* part, double* C,
                       hipStream_t s) {
    const int splits = ace_splits(K, m, n);
    long kslice = (K + splits - 1) / splits;
    kslice = (kslice + NT_BK - 1) / NT_BK * NT_BK;
    dim3 grid((n + NT_BN - 1) / NT_BN, (m + NT_BM - 1) / NT_BM, splits);
    hipLaunchKernelGGL((k_gemm_nt_splitk<TA, TB>), grid, dim3(NT_BS), 0, s, A, B, m, n, K, kslice, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int mn = m * n;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((mn + 255) / 256), dim3(256), 0, s, part, splits, mn, alpha, C);
    return hipGetLastError();
}

template <typename TB, typename TC>
hipError_t ace_gemm_nn(const double* A, long sai, long sak, const TB* B, int m, int K, long ncol, double alpha, TC* C,
                       hipStream_t s) {
    dim3 grid((unsigned)((ncol + NN_BN - 1) / NN_BN), (m + NN_BM - 1) / NN_BM);
    hipLaunchKernelGGL((k_gemm_nn_smallk<TB, TC>), grid, dim3(NN_BS), 0, s, A, sai, sak, B, m, K, ncol, alpha, C);
    return hipGetLastError();
}

template hipError_t ace_gemm_nt<double, double>(const double*, const double*, int, int, long, double, double*,
                                                double*, hipStream_t);
template hipError_t ace_gemm_nn<double, double>(const double*, long, long, const double*, int, int, long, double,
                                                double*, hipStream_t);
template hipError_t ace_gemm_nn<double, float>(const double*, long, long, const double*, int, int, long, double,
                                               float*, hipStream_t);
template hipError_t ace_gemm_nn<float, float>(const double*, long, long, const float*, int, int, long, double,
                                              float*, hipStream_t);
template hipError_t ace_gemm_nt<float, float>(const float*, const float*, int, int, long, double, double*, double*,
                                              hipStream_t);
template hipError_t ace_gemm_nt<double, float>(const double*, const float*, int, int, long, double, double*, double*,
                                               hipStream_t);

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
