// SCDM column selection (Sec. II.A, Eq. 1): the pivots of a column-pivoted QR
// of Phi^T (n_occ x Ng), in FP64.
//
// Pivot k is the column of Phi^T whose part orthogonal to the columns already
// chosen is longest.  With q_0..q_{k-1} the orthonormal directions of the
// chosen columns, that squared length is nrm_j = |a_j|^2 - sum_l (q_l . a_j)^2.
// Keeping every nrm_j current would read all of Phi^T once per pivot; instead
// pivots are chosen in rounds:
//
//   * at the start of a round every nrm_j is exact; its largest column is the
//     next pivot (no question of staleness);
//   * the columns whose nrm_j lies within a few octaves of that maximum (at
//     most SC_TMAX of them, picked by a histogram of the norms' bit patterns)
//     become candidates: their n_occ-vectors are copied out and their norms
//     are kept current pivot by pivot;
//   * a later pivot of the round is the best candidate as long as its norm
//     strictly exceeds tau, the largest round-start norm of any
//     non-candidate (norms only shrink, so no outside column can beat it);
//     otherwise the round ends, all nrm_j take the round's q's in one pass
//     over Phi^T, and the next round starts.
//
// The result is the greedy choice itself (up to rounding), with one pass
// over Phi^T per round instead of per pivot.  The new direction q_k is the
// pivot column orthogonalized against q_0..q_{k-1} by classical Gram-Schmidt
// applied twice.
#include "k_scdm.h"

namespace {

constexpr int SC_BS = 256;       // block of the grid-wide kernels
constexpr int SC_IT = 32;        // i-tile of the q block staged in LDS
constexpr int SC_PICK = 1024;    // block of the pick kernel
constexpr int SC_NB = 4096;      // histogram bins: 64 per octave of nrm_j / max

struct __align__(16) ScdmState {
    int k;              // pivots chosen so far
    int k0;             // first pivot of the current round
    int stop;           // the current round has ended
    int fail;           // 1-based step whose residual vanished (rank), 0 = none
    int ncand;          // candidates of the current round
    int bstar;          // last histogram bin taken into the candidate set (-1: none)
    long long gidx;     // column of the largest nrm_j at the round start
    double gmax;        // that nrm_j
    unsigned long long tau_bits;   // largest nrm_j outside the candidates (bits)
    double nrm0;        // largest initial column norm^2
};

__device__ __forceinline__ int bin_of(double v, double gmax) {
    // nonnegative doubles order like their bit patterns; 2^46 in the pattern
    // is 1/64 of an octave
    const unsigned long long d =
        (unsigned long long)__double_as_longlong(gmax) - (unsigned long long)__double_as_longlong(v);
    const unsigned long long b = d >> 46;
    return b >= (unsigned long long)SC_NB ? SC_NB - 1 : (int)b;
}

// (value, index) maximum with the smaller index on equal values
__device__ __forceinline__ bool better(double v, long long j, double bv, long long bj) {
    return v > bv || (v == bv && j < bj);
}

__device__ __forceinline__ void wave_argmax(double& v, long long& j) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_down(v, off, 64);
        const long long oj = __shfl_down(j, off, 64);
        if (better(ov, oj, v, j)) {
            v = ov;
            j = oj;
        }
    }
}

template <int BS>
__device__ void block_argmax(double& v, long long& j, double* sv, long long* sj) {
    wave_argmax(v, j);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sv[w] = v;
        sj[w] = j;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int t = 1; t < BS / 64; ++t)
            if (better(sv[t], sj[t], v, j)) {
                v = sv[t];
                j = sj[t];
            }
    }
}

template <int BS>
__device__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int u = 0; u < BS / 64; ++u) t += red[u];
    return t;   // every thread
}

template <typename T>
__device__ __forceinline__ double ld(const T* p, size_t o) {
    return (double)p[o];
}

// nrm_j = |a_j|^2 (INIT) or nrm_j -= sum_{l<b} (q_l . a_j)^2 for the b
// directions Qr (rows of n doubles); chosen pivots (nrm_j < 0) stay
// negative.  Per block: the largest nrm_j and its column.
template <typename T, bool INIT>
__global__ __launch_bounds__(SC_BS) void k_scdm_update(const T* __restrict__ phi, long Ng, int n,
                                                      const double* __restrict__ Qr, int b,
                                                      double* __restrict__ nrm, double* __restrict__ pv,
                                                      long long* __restrict__ pj) {
    __shared__ double qs[SC_IT][SC_RB];
    __shared__ double sv[SC_BS / 64];
    __shared__ long long sj[SC_BS / 64];
    const long j = (long)blockIdx.x * SC_BS + threadIdx.x;
    const bool live = j < Ng;
    const long jj = live ? j : 0;
    double acc[SC_RB];
#pragma unroll
    for (int l = 0; l < SC_RB; ++l) acc[l] = 0.0;
    double ss = 0.0;
    for (int i0 = 0; i0 < n; i0 += SC_IT) {
        const int iend = min(SC_IT, n - i0);
        if (!INIT) {
            __syncthreads();
            for (int t = threadIdx.x; t < SC_IT * SC_RB; t += SC_BS) {
                const int ii = t / SC_RB, l = t % SC_RB;
                qs[ii][l] = (l < b && ii < iend) ? Qr[(size_t)l * n + i0 + ii] : 0.0;
            }
            __syncthreads();
        }
        int ii = 0;
        for (; ii + 8 <= iend; ii += 8) {
            double a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) a[u] = ld(phi, (size_t)(i0 + ii + u) * Ng + jj);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (INIT) {
                    ss += a[u] * a[u];
                } else {
#pragma unroll
                    for (int l = 0; l < SC_RB; ++l) acc[l] += qs[ii + u][l] * a[u];
                }
            }
        }
        for (; ii < iend; ++ii) {
            const double a = ld(phi, (size_t)(i0 + ii) * Ng + jj);
            if (INIT) {
                ss += a * a;
            } else {
#pragma unroll
                for (int l = 0; l < SC_RB; ++l) acc[l] += qs[ii][l] * a;
            }
        }
    }
    double v = -1.0;
    if (live) {
        if (INIT) {
            v = ss;
        } else {
            v = nrm[j];
            if (v >= 0.0) {
                double d = 0.0;
#pragma unroll
                for (int l = 0; l < SC_RB; ++l) d += acc[l] * acc[l];
                v -= d;
                if (!(v >= 0.0)) v = -0.5;   // numerically inside the span
            }
        }
        nrm[j] = v;
    }
    long long bj = live ? j : (long long)Ng;
    block_argmax<SC_BS>(v, bj, sv, sj);
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = v;
        pj[blockIdx.x] = bj;
    }
}

// Round start: the largest nrm_j over the update partials; counters cleared.
__global__ __launch_bounds__(SC_PICK) void k_scdm_round_start(const double* __restrict__ pv,
                                                            const long long* __restrict__ pj, int np,
                                                            ScdmState* __restrict__ st,
                                                            unsigned* __restrict__ hist, int first) {
    __shared__ double sv[SC_PICK / 64];
    __shared__ long long sj[SC_PICK / 64];
    double v = -2.0;
    long long j = 0x7fffffffffffffffll;
    for (int t = threadIdx.x; t < np; t += SC_PICK)
        if (better(pv[t], pj[t], v, j)) {
            v = pv[t];
            j = pj[t];
        }
    block_argmax<SC_PICK>(v, j, sv, sj);
    for (int t = threadIdx.x; t < SC_NB; t += SC_PICK) hist[t] = 0u;
    if (threadIdx.x == 0) {
        if (first) {
            st->k = 0;
            st->fail = 0;
            st->nrm0 = v;
        }
        st->k0 = st->k;
        st->gmax = v;
        st->gidx = j;
        st->ncand = 0;
        st->tau_bits = 0ull;
        // no positive norm left: the remaining columns lie in the span
        st->stop = (v > 1e-26 * st->nrm0) ? 0 : 1;
        if (st->stop && !st->fail) st->fail = st->k + 1;
    }
}

// Histogram of the positive norms by bin_of.
__global__ __launch_bounds__(SC_BS) void k_scdm_hist(const double* __restrict__ nrm, long Ng,
                                                   const ScdmState* __restrict__ st, unsigned* __restrict__ hist) {
    __shared__ unsigned h[SC_NB];
    for (int t = threadIdx.x; t < SC_NB; t += SC_BS) h[t] = 0u;
    __syncthreads();
    const double gmax = st->gmax;
    const bool run = !st->stop;
    if (run)
        for (long j = (long)blockIdx.x * SC_BS + threadIdx.x; j < Ng; j += (long)gridDim.x * SC_BS) {
            const double v = nrm[j];
            if (v > 0.0) atomicAdd(&h[bin_of(v, gmax)], 1u);
        }
    __syncthreads();
    if (run)
        for (int t = threadIdx.x; t < SC_NB; t += SC_BS)
            if (h[t]) atomicAdd(&hist[t], h[t]);
}

// bstar = the last bin whose cumulative count stays within SC_TMAX.
__global__ __launch_bounds__(SC_PICK) void k_scdm_select(const unsigned* __restrict__ hist,
                                                       ScdmState* __restrict__ st) {
    constexpr int PER = SC_NB / SC_PICK;
    __shared__ unsigned scan[SC_PICK];
    __shared__ int best[SC_PICK / 64];
    unsigned loc[PER];
    unsigned s = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        loc[u] = hist[threadIdx.x * PER + u];
        s += loc[u];
    }
    scan[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < SC_PICK; off <<= 1) {
        const unsigned add = threadIdx.x >= (unsigned)off ? scan[threadIdx.x - off] : 0u;
        __syncthreads();
        scan[threadIdx.x] += add;
        __syncthreads();
    }
    unsigned cum = scan[threadIdx.x] - s;   // exclusive prefix
    int b = -1;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        cum += loc[u];
        if (cum <= (unsigned)SC_TMAX) b = threadIdx.x * PER + u;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) b = max(b, __shfl_down(b, off, 64));
    if ((threadIdx.x & 63) == 0) best[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = -1;
        for (int w = 0; w < SC_PICK / 64; ++w) m = max(m, best[w]);
        if (!st->stop) st->bstar = m;
    }
}

// Candidates: positive norms in bins <= bstar, plus the round's first pivot.
// tau = the largest positive norm of the rest.
__global__ __launch_bounds__(SC_BS) void k_scdm_gather(const double* __restrict__ nrm, long Ng,
                                                     ScdmState* __restrict__ st, int* __restrict__ cidx,
                                                     double* __restrict__ cval) {
    if (st->stop) return;
    const double gmax = st->gmax;
    const int bstar = st->bstar;
    const long long gidx = st->gidx;
    const int lane = threadIdx.x & 63;
    unsigned long long tb = 0ull;
    for (long base = (long)blockIdx.x * SC_BS; base < Ng; base += (long)gridDim.x * SC_BS) {
        const long j = base + threadIdx.x;
        const double v = j < Ng ? nrm[j] : -1.0;
        bool cand = false;
        if (v > 0.0) {
            cand = bin_of(v, gmax) <= bstar || j == gidx;
            if (!cand) tb = max(tb, (unsigned long long)__double_as_longlong(v));
        }
        const unsigned long long m = __ballot(cand);
        if (m) {
            int pos0 = 0;
            if (lane == 0) pos0 = atomicAdd(&st->ncand, __popcll(m));
            pos0 = __shfl(pos0, 0, 64);
            if (cand) {
                const int pos = pos0 + __popcll(m & ((1ull << lane) - 1ull));
                if (pos < SC_TMAX + 1) {
                    cidx[pos] = (int)j;
                    cval[pos] = v;
                }
            }
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_down(tb, off, 64);
        tb = o > tb ? o : tb;
    }
    if (lane == 0 && tb) atomicMax(&st->tau_bits, tb);
}

// cvec[t][i] = Phi^T(i, cidx[t]) for the candidates.
template <typename T>
__global__ __launch_bounds__(SC_BS) void k_scdm_cand_vec(const T* __restrict__ phi, long Ng, int n,
                                                       const ScdmState* __restrict__ st,
                                                       const int* __restrict__ cidx, double* __restrict__ cvec) {
    if (st->stop) return;
    const int t = blockIdx.y;
    if (t >= min(st->ncand, SC_TMAX + 1)) return;
    const int i = blockIdx.x * SC_BS + threadIdx.x;
    if (i < n) cvec[(size_t)t * n + i] = ld(phi, (size_t)i * Ng + cidx[t]);
}

// One pivot: the round's first is the largest exact norm; later ones the
// best candidate if it beats tau, else the round ends.  The pivot column is
// orthogonalized against Q (classical Gram-Schmidt, twice) and normalized
// into row k of Q.
template <typename T>
__global__ __launch_bounds__(SC_PICK) void k_scdm_pick(const T* __restrict__ phi, long Ng, int n,
                                                     ScdmState* __restrict__ st, const double* __restrict__ dv,
                                                     const long long* __restrict__ dj, int nd,
                                                     double* __restrict__ Q, int* __restrict__ piv,
                                                     double* __restrict__ rdiag, double* __restrict__ nrm) {
    __shared__ double r[SC_NMAX];
    __shared__ double d[SC_NMAX];
    __shared__ double sv[SC_PICK / 64];
    __shared__ long long sj[SC_PICK / 64];
    __shared__ long long cj;
    __shared__ int go;
    const int k = st->k;
    if (st->stop || k >= n) {
        if (threadIdx.x == 0) st->stop = 1;
        return;
    }
    if (k == st->k0) {
        if (threadIdx.x == 0) {
            cj = st->gidx;
            go = 1;
        }
    } else {
        double v = -2.0;
        long long j = 0x7fffffffffffffffll;
        for (int t = threadIdx.x; t < nd; t += SC_PICK)
            if (better(dv[t], dj[t], v, j)) {
                v = dv[t];
                j = dj[t];
            }
        block_argmax<SC_PICK>(v, j, sv, sj);
        if (threadIdx.x == 0) {
            const double tau = __longlong_as_double((long long)st->tau_bits);
            go = v > tau && v > 0.0;
            cj = j;
            if (!go) st->stop = 1;
        }
    }
    __syncthreads();
    if (!go) return;
    const long long c = cj;
    for (int i = threadIdx.x; i < n; i += SC_PICK) r[i] = ld(phi, (size_t)i * Ng + c);
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int pass = 0; pass < 2; ++pass) {
        for (int l = w; l < k; l += SC_PICK / 64) {
            const double* q = Q + (size_t)l * n;
            double s = 0.0;
            for (int i = lane; i < n; i += 64) s += q[i] * r[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
            if (lane == 0) d[l] = s;
        }
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += SC_PICK) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) s += d[l] * Q[(size_t)l * n + i];
            r[i] -= s;
        }
        __syncthreads();
    }
    double ss = 0.0;
    for (int i = threadIdx.x; i < n; i += SC_PICK) ss += r[i] * r[i];
    ss = block_sum<SC_PICK>(ss, sv);
    if (!(ss > 1e-26 * st->nrm0)) {
        if (threadIdx.x == 0) {
            st->fail = k + 1;
            st->stop = 1;
        }
        return;
    }
    const double rn = sqrt(ss), inv = 1.0 / rn;
    for (int i = threadIdx.x; i < n; i += SC_PICK) Q[(size_t)k * n + i] = r[i] * inv;
    if (threadIdx.x == 0) {
        piv[k] = (int)c;
        rdiag[k] = rn;
        nrm[c] = -1.0;
        st->k = k + 1;
    }
}

// Candidates take the newest direction q_{k-1}: one wave per candidate.
// Per block: the best remaining candidate (value, column).
__global__ __launch_bounds__(SC_BS) void k_scdm_down(int n, const ScdmState* __restrict__ st,
                                                   const int* __restrict__ cidx, double* __restrict__ cval,
                                                   const double* __restrict__ cvec, const double* __restrict__ Q,
                                                   const double* __restrict__ nrm, double* __restrict__ dv,
                                                   long long* __restrict__ dj) {
    __shared__ double sv[SC_BS / 64];
    __shared__ long long sj[SC_BS / 64];
    if (st->stop) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int t = blockIdx.x * (SC_BS / 64) + w;
    const int nc = min(st->ncand, SC_TMAX + 1);
    const double* q = Q + (size_t)(st->k - 1) * n;
    double v = -2.0;
    long long j = 0x7fffffffffffffffll;
    if (t < nc) {
        v = cval[t];
        j = cidx[t];
        if (v >= 0.0 && nrm[j] < 0.0) v = -1.0;   // chosen as a pivot
        if (v >= 0.0) {
            const double* a = cvec + (size_t)t * n;
            double s = 0.0;
            for (int i = lane; i < n; i += 64) s += a[i] * q[i];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
            v -= s * s;
            if (!(v >= 0.0)) v = -0.5;
        }
        if (lane == 0) cval[t] = v;
    }
    block_argmax<SC_BS>(v, j, sv, sj);
    if (threadIdx.x == 0) {
        dv[blockIdx.x] = v;
        dj[blockIdx.x] = j;
    }
}

// G[a][i] = Phi^T(i, piv[a])
template <typename T>
__global__ __launch_bounds__(SC_BS) void k_scdm_pivot_rows(const T* __restrict__ phi, long Ng, int n,
                                                         const int* __restrict__ piv, double* __restrict__ G) {
    const int a = blockIdx.y;
    const int i = blockIdx.x * SC_BS + threadIdx.x;
    if (i < n) G[(size_t)a * n + i] = ld(phi, (size_t)i * Ng + piv[a]);
}

// Newton-Schulz steps for the polar factor (see scdm_polar_*): one workgroup.
constexpr int NS_BS = 1024;

// Y = G / |G|_F
__global__ __launch_bounds__(NS_BS) void k_ns_scale(const double* __restrict__ G, int n, double* __restrict__ Y) {
    __shared__ double red[NS_BS / 64];
    const long nn = (long)n * n;
    double s = 0.0;
    for (long t = threadIdx.x; t < nn; t += NS_BS) s += G[t] * G[t];
    s = block_sum<NS_BS>(s, red);
    const double inv = 1.0 / sqrt(s);
    for (long t = threadIdx.x; t < nn; t += NS_BS) Y[t] = G[t] * inv;
}

// S <- 1.5 I - 0.5 S, err = |S - I|_F^2 of the incoming S
__global__ __launch_bounds__(NS_BS) void k_ns_mid(double* __restrict__ S, int n, double* __restrict__ err) {
    __shared__ double red[NS_BS / 64];
    const long nn = (long)n * n;
    double e = 0.0;
    for (long t = threadIdx.x; t < nn; t += NS_BS) {
        const bool diag = (t / n) == (t % n);
        const double v = S[t];
        const double d = diag ? v - 1.0 : v;
        e += d * d;
        S[t] = (diag ? 1.5 : 0.0) - 0.5 * v;
    }
    e = block_sum<NS_BS>(e, red);
    if (threadIdx.x == 0) *err = e;
}

}  // namespace

hipError_t scdm_ns_scale(const double* G, int n, double* Y, hipStream_t s) {
    hipLaunchKernelGGL(k_ns_scale, dim3(1), dim3(NS_BS), 0, s, G, n, Y);
    return hipGetLastError();
}

hipError_t scdm_ns_mid(double* S, int n, double* err, hipStream_t s) {
    hipLaunchKernelGGL(k_ns_mid, dim3(1), dim3(NS_BS), 0, s, S, n, err);
    return hipGetLastError();
}

ScdmLayout scdm_layout(long Ng, int n) {
    ScdmLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~(size_t)255;
        return o;
    };
    const long nub = (Ng + SC_BS - 1) / SC_BS;
    const int ndb = (SC_TMAX + 1 + SC_BS / 64 - 1) / (SC_BS / 64);
    L.n_upd_blocks = nub;
    L.n_down_blocks = ndb;
    L.state = take(sizeof(ScdmState));
    L.nrm = take((size_t)Ng * sizeof(double));
    L.upv = take((size_t)nub * sizeof(double));
    L.upj = take((size_t)nub * sizeof(long long));
    L.hist = take(SC_NB * sizeof(unsigned));
    L.cidx = take((SC_TMAX + 1) * sizeof(int));
    L.cval = take((SC_TMAX + 1) * sizeof(double));
    L.cvec = take((size_t)(SC_TMAX + 1) * n * sizeof(double));
    L.dv = take((size_t)ndb * sizeof(double));
    L.dj = take((size_t)ndb * sizeof(long long));
    L.Q = take((size_t)n * n * sizeof(double));
    L.piv = take((size_t)n * sizeof(int));
    L.rdiag = take((size_t)n * sizeof(double));
    L.total = off;
    return L;
}

size_t scdm_state_bytes() { return sizeof(ScdmState); }

hipError_t scdm_init(const void* phi, int f32, long Ng, int n, char* ws, const ScdmLayout& L, hipStream_t s) {
    double* nrm = (double*)(ws + L.nrm);
    double* upv = (double*)(ws + L.upv);
    long long* upj = (long long*)(ws + L.upj);
    const unsigned nb = (unsigned)L.n_upd_blocks;
    if (f32)
        hipLaunchKernelGGL((k_scdm_update<float, true>), dim3(nb), dim3(SC_BS), 0, s, (const float*)phi, Ng, n,
                           (const double*)nullptr, 0, nrm, upv, upj);
    else
        hipLaunchKernelGGL((k_scdm_update<double, true>), dim3(nb), dim3(SC_BS), 0, s, (const double*)phi, Ng, n,
                           (const double*)nullptr, 0, nrm, upv, upj);
    return hipGetLastError();
}

hipError_t scdm_update(const void* phi, int f32, long Ng, int n, int k0, int b, char* ws, const ScdmLayout& L,
                       hipStream_t s) {
    double* nrm = (double*)(ws + L.nrm);
    double* upv = (double*)(ws + L.upv);
    long long* upj = (long long*)(ws + L.upj);
    const double* Qr = (const double*)(ws + L.Q) + (size_t)k0 * n;
    const unsigned nb = (unsigned)L.n_upd_blocks;
    if (b < 0 || b > SC_RB) return hipErrorInvalidValue;
    if (f32)
        hipLaunchKernelGGL((k_scdm_update<float, false>), dim3(nb), dim3(SC_BS), 0, s, (const float*)phi, Ng, n, Qr,
                           b, nrm, upv, upj);
    else
        hipLaunchKernelGGL((k_scdm_update<double, false>), dim3(nb), dim3(SC_BS), 0, s, (const double*)phi, Ng, n,
                           Qr, b, nrm, upv, upj);
    return hipGetLastError();
}

hipError_t scdm_round(const void* phi, int f32, long Ng, int n, int first, char* ws, const ScdmLayout& L,
                      hipStream_t s) {
    ScdmState* st = (ScdmState*)(ws + L.state);
    double* nrm = (double*)(ws + L.nrm);
    unsigned* hist = (unsigned*)(ws + L.hist);
    int* cidx = (int*)(ws + L.cidx);
    double* cval = (double*)(ws + L.cval);
    double* cvec = (double*)(ws + L.cvec);
    double* dv = (double*)(ws + L.dv);
    long long* dj = (long long*)(ws + L.dj);
    double* Q = (double*)(ws + L.Q);
    int* piv = (int*)(ws + L.piv);
    double* rdiag = (double*)(ws + L.rdiag);
    hipLaunchKernelGGL(k_scdm_round_start, dim3(1), dim3(SC_PICK), 0, s, (const double*)(ws + L.upv),
                       (const long long*)(ws + L.upj), (int)L.n_upd_blocks, st, hist, first);
    const long gb = (Ng + SC_BS - 1) / SC_BS;
    const unsigned g = (unsigned)(gb < 2048 ? gb : 2048);
    hipLaunchKernelGGL(k_scdm_hist, dim3(g), dim3(SC_BS), 0, s, (const double*)nrm, Ng, (const ScdmState*)st, hist);
    hipLaunchKernelGGL(k_scdm_select, dim3(1), dim3(SC_PICK), 0, s, (const unsigned*)hist, st);
    hipLaunchKernelGGL(k_scdm_gather, dim3(g), dim3(SC_BS), 0, s, (const double*)nrm, Ng, st, cidx, cval);
    const dim3 cg((n + SC_BS - 1) / SC_BS, SC_TMAX + 1);
    if (f32)
        hipLaunchKernelGGL((k_scdm_cand_vec<float>), cg, dim3(SC_BS), 0, s, (const float*)phi, Ng, n,
                           (const ScdmState*)st, (const int*)cidx, cvec);
    else
        hipLaunchKernelGGL((k_scdm_cand_vec<double>), cg, dim3(SC_BS), 0, s, (const double*)phi, Ng, n,
                           (const ScdmState*)st, (const int*)cidx, cvec);
    const int nd = (int)L.n_down_blocks;
    for (int step = 0; step < SC_RB; ++step) {
        if (f32)
            hipLaunchKernelGGL((k_scdm_pick<float>), dim3(1), dim3(SC_PICK), 0, s, (const float*)phi, Ng, n, st,
                               (const double*)dv, (const long long*)dj, nd, Q, piv, rdiag, nrm);
        else
            hipLaunchKernelGGL((k_scdm_pick<double>), dim3(1), dim3(SC_PICK), 0, s, (const double*)phi, Ng, n, st,
                               (const double*)dv, (const long long*)dj, nd, Q, piv, rdiag, nrm);
        hipLaunchKernelGGL(k_scdm_down, dim3(nd), dim3(SC_BS), 0, s, n, (const ScdmState*)st, (const int*)cidx, cval,
                           (const double*)cvec, (const double*)Q, (const double*)nrm, dv, dj);
    }
    return hipGetLastError();
}

hipError_t scdm_pivot_rows(const void* phi, int f32, long Ng, int n, const int* piv, double* G, hipStream_t s) {
    const dim3 g((n + SC_BS - 1) / SC_BS, n);
    if (f32)
        hipLaunchKernelGGL((k_scdm_pivot_rows<float>), g, dim3(SC_BS), 0, s, (const float*)phi, Ng, n, piv, G);
    else
        hipLaunchKernelGGL((k_scdm_pivot_rows<double>), g, dim3(SC_BS), 0, s, (const double*)phi, Ng, n, piv, G);
    return hipGetLastError();
}

// Host view of the state fields the round loop needs.
hipError_t scdm_read_state(const char* ws, const ScdmLayout& L, int* k, int* fail, hipStream_t s) {
    ScdmState h;
    hipError_t e = hipMemcpyAsync(&h, ws + L.state, sizeof(h), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *k = h.k;
    *fail = h.fail;
    return hipSuccess;
}
