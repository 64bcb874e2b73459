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

// Blocked right-looking Cholesky (lower, row-major) of A into L, in place
// in L, blocks of CB: for each block column kb, one workgroup factors the
// diagonal block in LDS (column by column), a grid of workgroups solves the
// panel below it against that factor (a wavefront per row, forward
// substitution with the row's entries on the lanes), and a grid of
// 64 x 64 tiles subtracts the panel's rank-CB product from the lower
// trailing matrix.  flag[0] = 1-based index of the first non-positive
// pivot, 0 on success; every kernel stops once it is set.
constexpr int CB = 64;

__global__ __launch_bounds__(256) void k_chol_init(const double* __restrict__ A, int n, double* __restrict__ L,
                                                   int* __restrict__ flag) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t == 0) flag[0] = 0;
    if (t >= (size_t)n * n) return;
    const int i = (int)(t / n), j = (int)(t % n);
    L[t] = j <= i ? A[t] : 0.0;
}

__global__ __launch_bounds__(CH_BS) void k_chol_diag(int n, int kb, double* __restrict__ L, int* __restrict__ flag) {
    __shared__ double D[CB][CB + 1];
    __shared__ int bad;
    if (flag[0]) return;
    const int nb = min(CB, n - kb);
    for (int t = threadIdx.x; t < CB * CB; t += CH_BS) {
        const int r = t / CB, c = t % CB;
        D[r][c] = (r < nb && c <= r) ? L[(size_t)(kb + r) * n + kb + c] : 0.0;
    }
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
        if (threadIdx.x == 0) {
            const double d = D[j][j];
            if (d > 0.0) D[j][j] = sqrt(d);
            else bad = kb + j + 1;
        }
        __syncthreads();
        if (bad) break;
        const double djj = D[j][j];
        for (int r = j + 1 + threadIdx.x; r < nb; r += CH_BS) D[r][j] /= djj;
        __syncthreads();
        const int m = nb - j - 1;   // trailing lower triangle of the block
        for (int t = threadIdx.x; t < m * m; t += CH_BS) {
            const int r = j + 1 + t / m, c = j + 1 + t % m;
            if (c <= r) D[r][c] -= D[r][j] * D[c][j];
        }
        __syncthreads();
    }
    if (bad) {
        if (threadIdx.x == 0) flag[0] = bad;
        return;
    }
    for (int t = threadIdx.x; t < nb * nb; t += CH_BS) {
        const int r = t / nb, c = t % nb;
        if (c <= r) L[(size_t)(kb + r) * n + kb + c] = D[r][c];
    }
}

// rows kb + CB + 16 blockIdx.x + wave: L[i][kb..kb+CB) <- (that row) L11^-T
__global__ __launch_bounds__(CH_BS) void k_chol_trsm(int n, int kb, double* __restrict__ L, const int* __restrict__ flag) {
    __shared__ double D[CB][CB + 1];
    if (flag[0]) return;
    for (int t = threadIdx.x; t < CB * CB; t += CH_BS) {
        const int r = t / CB, c = t % CB;
        D[r][c] = c <= r ? L[(size_t)(kb + r) * n + kb + c] : 0.0;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = kb + CB + blockIdx.x * (CH_BS / 64) + wave;
    if (i >= n) return;
    double* row = L + (size_t)i * n + kb;
    double a = row[lane];
    for (int k = 0; k < CB; ++k) {
        const double yk = __shfl(a, k, 64) / D[k][k];
        if (lane == k) a = yk;
        else if (lane > k) a -= D[lane][k] * yk;
    }
    row[lane] = a;
}

// lower 64 x 64 tiles (ti >= tc) of the trailing matrix from kb + CB on:
// L[i][c] -= sum_m L[i][kb+m] L[c][kb+m]
__global__ __launch_bounds__(256) void k_chol_syrk(int n, int kb, double* __restrict__ L, const int* __restrict__ flag) {
    __shared__ double Pi[CB][CB + 1], Pc[CB][CB + 1];
    if (flag[0]) return;
    int ti = 0, rem = blockIdx.x;
    while (rem > ti) {
        rem -= ti + 1;
        ++ti;
    }
    const int tc = rem;
    const int r0 = kb + CB + ti * CB, c0 = kb + CB + tc * CB;
    for (int t = threadIdx.x; t < CB * CB; t += 256) {
        const int r = t / CB, m = t % CB;
        Pi[r][m] = r0 + r < n ? L[(size_t)(r0 + r) * n + kb + m] : 0.0;
        Pc[r][m] = c0 + r < n ? L[(size_t)(c0 + r) * n + kb + m] : 0.0;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < CB * CB; t += 256) {
        const int r = t / CB, c = t % CB;
        const int i = r0 + r, j = c0 + c;
        if (i >= n || j > i) continue;
        double s = 0.0;
#pragma unroll 8
        for (int m = 0; m < CB; ++m) s += Pi[r][m] * Pc[c][m];
        L[(size_t)i * n + j] -= s;
    }
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

// Symmetric eigendecomposition A = Q diag(lambda) Q^T (App. A) by parallel
// cyclic Jacobi in one workgroup: each round rotates n/2 disjoint (p, q)
// planes chosen by a round-robin tournament (index 0 fixed, the others
// rotating), so every pair of indices meets once per sweep; rows, then
// columns and the eigenvector matrix are updated in separate phases.  The
// rotation zeroing A[p][q] uses t = tan(angle) = sgn(th)/(|th| + sqrt(th^2
// + 1)), th = (A[q][q] - A[p][p]) / (2 A[p][q]).  Sweeps stop when the
// off-diagonal Frobenius norm is below 1e-15 of the whole, or after 40.
// A (n x n, overwritten), V (n x n, eigenvectors in columns), lam (n).
constexpr int JB_BS = 1024;
constexpr int JB_MAXP = 2048;   // pairs per round (n <= 4096)

__global__ __launch_bounds__(JB_BS) void k_jacobi_eig(double* __restrict__ A, int n, double* __restrict__ V,
                                                      double* __restrict__ lam) {
    __shared__ double cs[JB_MAXP], sn[JB_MAXP];
    __shared__ int pp[JB_MAXP], qq[JB_MAXP];
    __shared__ double red[JB_BS / 64];
    __shared__ int done;
    const int m = n + (n & 1);      // even count; index n (if any) is a dummy
    const int np = m / 2;
    for (int t = threadIdx.x; t < n * n; t += JB_BS) V[t] = (t / n == t % n) ? 1.0 : 0.0;
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        // convergence test on the off-diagonal part
        double off = 0.0, tot = 0.0;
        for (int t = threadIdx.x; t < n * n; t += JB_BS) {
            const double v = A[t] * A[t];
            tot += v;
            if (t / n != t % n) off += v;
        }
        off = wave_sum(off);
        tot = wave_sum(tot);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = off;
        __syncthreads();
        if (threadIdx.x == 0) {
            double o2 = 0.0;
            for (int w = 0; w < JB_BS / 64; ++w) o2 += red[w];
            red[0] = o2;
        }
        __syncthreads();
        const double offs = red[0];
        __syncthreads();
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t2 = 0.0;
            for (int w = 0; w < JB_BS / 64; ++w) t2 += red[w];
            done = !(offs > 1e-30 * t2);
        }
        __syncthreads();
        if (done) break;
        for (int r = 0; r < m - 1; ++r) {
            for (int k = threadIdx.x; k < np; k += JB_BS) {
                auto idx = [&](int t) { return t == 0 ? 0 : ((t - 1 + r) % (m - 1)) + 1; };
                int p = idx(k), q = idx(m - 1 - k);
                if (p > q) { const int tmp = p; p = q; q = tmp; }
                double c = 1.0, sv = 0.0;
                if (q < n) {
                    const double apq = A[(size_t)p * n + q];
                    if (apq != 0.0) {
                        const double th = (A[(size_t)q * n + q] - A[(size_t)p * n + p]) / (2.0 * apq);
                        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sv = t * c;
                    }
                }
                cs[k] = c;
                sn[k] = sv;
                pp[k] = p;
                qq[k] = q;
            }
            __syncthreads();
            // rows p, q <- P^T A
            for (int t = threadIdx.x; t < np * n; t += JB_BS) {
                const int k = t / n, j = t % n;
                const int p = pp[k], q = qq[k];
                if (q >= n || sn[k] == 0.0) continue;
                const double a = A[(size_t)p * n + j], b = A[(size_t)q * n + j];
                A[(size_t)p * n + j] = cs[k] * a - sn[k] * b;
                A[(size_t)q * n + j] = sn[k] * a + cs[k] * b;
            }
            __syncthreads();
            // columns p, q <- A P and V P
            for (int t = threadIdx.x; t < np * n; t += JB_BS) {
                const int k = t / n, i = t % n;
                const int p = pp[k], q = qq[k];
                if (q >= n || sn[k] == 0.0) continue;
                const double a = A[(size_t)i * n + p], b = A[(size_t)i * n + q];
                A[(size_t)i * n + p] = cs[k] * a - sn[k] * b;
                A[(size_t)i * n + q] = sn[k] * a + cs[k] * b;
                const double va = V[(size_t)i * n + p], vb = V[(size_t)i * n + q];
                V[(size_t)i * n + p] = cs[k] * va - sn[k] * vb;
                V[(size_t)i * n + q] = sn[k] * va + cs[k] * vb;
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += JB_BS) lam[i] = A[(size_t)i * n + i];
}

__global__ void k_transpose(const double* __restrict__ X, int n, double* __restrict__ Y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    Y[(size_t)(t % n) * n + t / n] = X[t];
}

// T[k][i] = Q[i][k] / sqrt(|lambda_k|) (zero for |lambda_k| <= 1e-14 max|lambda|),
// the map W -> zeta = W Q |Lambda|^{-1/2} in the layout of the xi product.
__global__ void k_eig_transform(const double* __restrict__ Q, const double* __restrict__ lam, int n,
                                double* __restrict__ T) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * n) return;
    const int k = t / n, i = t % n;
    double lmax = 0.0;
    for (int q = 0; q < n; ++q) lmax = fmax(lmax, fabs(lam[q]));
    const double l = fabs(lam[k]);
    T[t] = l > 1e-14 * lmax ? Q[(size_t)i * n + k] / sqrt(l) : 0.0;
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
    hipLaunchKernelGGL(k_chol_init, dim3((unsigned)(((size_t)n * n + 255) / 256)), dim3(256), 0, s, A, n, L, flag);
    for (int kb = 0; kb < n; kb += CB) {
        hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(CH_BS), 0, s, n, kb, L, flag);
        const int m = n - kb - CB;
        if (m <= 0) break;
        hipLaunchKernelGGL(k_chol_trsm, dim3((m + CH_BS / 64 - 1) / (CH_BS / 64)), dim3(CH_BS), 0, s, n, kb, L, flag);
        const int T = (m + CB - 1) / CB;
        hipLaunchKernelGGL(k_chol_syrk, dim3(T * (T + 1) / 2), dim3(256), 0, s, n, kb, L, flag);
    }
    return hipGetLastError();
}

hipError_t ace_trtri(const double* L, int n, double* X, hipStream_t s) {
    if (n > TR_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_trtri_lower, dim3(n), dim3(64), 0, s, L, n, X);
    return hipGetLastError();
}

hipError_t ace_eig(double* A, int n, double* V, double* lam, hipStream_t s) {
    if (n > 2 * JB_MAXP) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_jacobi_eig, dim3(1), dim3(JB_BS), 0, s, A, n, V, lam);
    return hipGetLastError();
}

hipError_t ace_transpose(const double* X, int n, double* Y, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose, dim3((n * n + 255) / 256), dim3(256), 0, s, X, n, Y);
    return hipGetLastError();
}

hipError_t ace_eig_transform(const double* Q, const double* lam, int n, double* T, hipStream_t s) {
    hipLaunchKernelGGL(k_eig_transform, dim3((n * n + 255) / 256), dim3(256), 0, s, Q, lam, n, T);
    return hipGetLastError();
}

hipError_t ace_neg_sum_squares(const double* S, int mn, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_neg_sum_squares, dim3(1), dim3(SQ_BS), 0, s, S, mn, out);
    return hipGetLastError();
}
