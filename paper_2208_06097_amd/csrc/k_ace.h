// Launchers of the ACE kernels (k_ace.hip).
#pragma once

#include <hip/hip_runtime.h>

hipError_t ace_symmetrize(const double* M, int n, double* Mb, hipStream_t s);
hipError_t ace_cholesky(const double* A, int n, double* L, int* flag, hipStream_t s);
hipError_t ace_trtri(const double* L, int n, double* X, hipStream_t s);
hipError_t ace_neg_sum_squares(const double* S, int mn, double* out, hipStream_t s);
// Symmetric eigendecomposition (parallel Jacobi, one workgroup): A is
// overwritten, V gets the eigenvectors in columns, lam the eigenvalues.
hipError_t ace_eig(double* A, int n, double* V, double* lam, hipStream_t s);
// T = (Q |Lambda|^{-1/2})^T, null directions dropped.
hipError_t ace_eig_transform(const double* Q, const double* lam, int n, double* T, hipStream_t s);
hipError_t ace_transpose(const double* X, int n, double* Y, hipStream_t s);

// Matrix-core versions (k_ace_mfma.hip).  KIND selects the operand type:
// FP64 (FP64 accumulation), FP32 or BF16 (FP32 accumulation within a K
// slice, FP64 across slices).  BF16 arrays are uint16_t bit patterns.
enum { ACE_F64 = 0, ACE_F32 = 1, ACE_BF16 = 2 };
// K slices of a long-K product (max_splits > 0 caps them)
int ace_mfma_splits(long K, int m, int n, int max_splits = 0);
// C (m x n) = alpha A B^T over K; part holds ace_mfma_splits(K,m,n,max_splits) * m * n doubles.
template <int KIND, typename TA, typename TB>
hipError_t ace_mm_nt(const TA* A, const TB* B, int m, int n, long K, double alpha, double* part, double* C,
                     hipStream_t s, int max_splits = 0);
// C (m x ncol) = alpha A B, A(i,k) = A[i*sai + k*sak] (m x K, FP64), B: K x ncol.
template <int KIND, typename TB, typename TC>
hipError_t ace_mm_nn(const double* A, long sai, long sak, const TB* B, int m, int K, long ncol, double alpha, TC* C,
                     hipStream_t s);
