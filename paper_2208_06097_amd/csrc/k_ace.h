// Launchers of the ACE kernels (k_ace.hip).
#pragma once

#include <hip/hip_runtime.h>

int ace_splits(long K, int m, int n);

// C (m x n) = alpha * A B^T, A: m x K, B: n x K (row-major); part holds
// ace_splits(K,m,n) * m * n doubles.
template <typename TA, typename TB>
hipError_t ace_gemm_nt(const TA* A, const TB* B, int m, int n, long K, double alpha, double* part, double* C,
                       hipStream_t s);

// C (m x ncol) = alpha * A B, A(i,k) = A[i*sai + k*sak] (m x K, FP64), B: K x ncol.
template <typename TB, typename TC>
hipError_t ace_gemm_nn(const double* A, long sai, long sak, const TB* B, int m, int K, long ncol, double alpha, TC* C,
                       hipStream_t s);

hipError_t ace_symmetrize(const double* M, int n, double* Mb, hipStream_t s);
hipError_t ace_cholesky(const double* A, int n, double* L, int* flag, hipStream_t s);
hipError_t ace_trtri(const double* L, int n, double* X, hipStream_t s);
hipError_t ace_neg_sum_squares(const double* S, int mn, double* out, hipStream_t s);
