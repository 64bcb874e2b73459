// ACE products on the matrix cores (Eq. 18-19): the two shapes of the ACE
// build and apply, for FP64, FP32 and BF16 operands.
//
//   NT (long K):  C = alpha A B^T, A: m x K, B: n x K, K = grid points.
//                 Split over K; every workgroup writes an FP64 partial
//                 m x n block of its K slice and a second kernel sums the
//                 slices in FP64 (M = dV Phi^T W, dV xi^T psi, dV Phi^T xi).
//   NN (small K): C = alpha A B, A: m x K (FP64, small), B: K x ncol,
//                 ncol = grid points (xi = L^-1 W, K psi = -C^T xi).
//
// Operand kinds: FP64 -> v_mfma_f64_16x16x4f64 (FP64 accumulation);
// FP32 -> v_mfma_f32_16x16x4f32 and BF16 -> v_mfma_f32_16x16x32_bf16, both
// with FP32 accumulation inside a workgroup's K range.  Inputs of another
// type are rounded to the operand kind while they are staged in LDS.
//
// Tiling: 256 threads, a 128 x 128 output block, four wavefronts of 64 x 64
// (4 x 4 tiles of 16 x 16), K staged 32 at a time as [row][k] in LDS.
// Operand lanes: A row = lane % 16, B column = lane % 16, k block = lane / 16.
// Result lanes: column = lane % 16; the row of item v is 4 (lane / 16) + v
// for the FP32-accumulating instructions and lane / 16 + 4 v for the FP64
// one (measured on gfx950).
#include <type_traits>

#include "k_ace.h"
#include "sea_internal.h"

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 128, BN = 128, NT = 256;
// Workgroups are handed to the 8 XCDs (each with its own L2) in turn.  The
// workgroups that read the same operand tiles (NT: the output tiles of one
// K slice; NN: the row blocks of one column tile of the grid-point operand)
// are given consecutive places in one XCD's sequence, so that they run there
// together and the second read of a tile comes from that L2.
constexpr int ACE_XCD = 8;
__host__ __device__ inline long xcd_grid(long groups, int per_group) {
    return (groups + ACE_XCD - 1) / ACE_XCD * ACE_XCD * per_group;
}
// workgroup k -> (group, member): group g's members on XCD g % ACE_XCD
__device__ __forceinline__ void xcd_block(int per_group, long& group, int& member) {
    const long k = blockIdx.x, x = k % ACE_XCD, mseq = k / ACE_XCD;
    member = (int)(mseq % per_group);
    group = (mseq / per_group) * ACE_XCD + x;
}

__device__ __forceinline__ float bf_to_f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f_to_bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// value of a stored element as float/double
template <typename T>
__device__ __forceinline__ double as_d(T v) { return (double)v; }
template <>
__device__ __forceinline__ double as_d<uint16_t>(uint16_t v) { return (double)bf_to_f(v); }
template <typename T>
__device__ __forceinline__ float as_f(T v) { return (float)v; }
template <>
__device__ __forceinline__ float as_f<uint16_t>(uint16_t v) { return bf_to_f(v); }

// per-kind operand element, LDS row pitch, accumulator and one MFMA k-step
template <int KIND>
struct Kind;
template <>
struct Kind<ACE_F64> {
    using E = double;
    using Acc = f64x4;
    // K staged 16 at a time: the next stage's loads held in registers stay
    // at 16 doubles per thread (with 128 accumulator registers per lane)
    static constexpr int KT = 16;
    static constexpr int PITCH = KT + 1;
    static constexpr int KSTEP = 4;
    // output item v of lane-group g holds tile row g + 4 v (FP64 layout)
    __device__ static int row(int g, int v) { return g + 4 * v; }
    template <typename T>
    __device__ static E cvt(T v) { return as_d(v); }
    __device__ static Acc mma(const E* a, const E* b, int g, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a[g], b[g], c, 0, 0, 0);
    }
};
template <>
struct Kind<ACE_F32> {
    using E = float;
    using Acc = f32x4;
    static constexpr int KT = 32;
    static constexpr int PITCH = KT + 1;
    static constexpr int KSTEP = 4;
    // output item v of lane-group g holds tile row 4 g + v
    __device__ static int row(int g, int v) { return 4 * g + v; }
    template <typename T>
    __device__ static E cvt(T v) { return as_f(v); }
    __device__ static Acc mma(const E* a, const E* b, int g, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a[g], b[g], c, 0, 0, 0);
    }
};
template <>
struct Kind<ACE_BF16> {
    using E = uint16_t;
    using Acc = f32x4;
    static constexpr int KT = 32;
    static constexpr int PITCH = KT + 8;  // 16-byte aligned rows
    static constexpr int KSTEP = 32;
    __device__ static int row(int g, int v) { return 4 * g + v; }
    template <typename T>
    __device__ static E cvt(T v) {
        if constexpr (std::is_same<T, uint16_t>::value) return v;  // already BF16 bits
        else return f_to_bf(as_f(v));
    }
    __device__ static Acc mma(const E* a, const E* b, int g, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(*reinterpret_cast<const bf16x8*>(a + 8 * g),
                                                       *reinterpret_cast<const bf16x8*>(b + 8 * g), c, 0, 0, 0);
    }
};

// Multiply the staged tiles: wave (wm, wn) = (wave / 2, wave % 2) owns rows
// wm*64.., cols wn*64..
template <int KIND>
__device__ __forceinline__ void tile_step(const typename Kind<KIND>::E* As, const typename Kind<KIND>::E* Bs, int kk,
                                          typename Kind<KIND>::Acc (&acc)[4][4]) {
    using K = Kind<KIND>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const typename K::E* a = As + (wm * 64 + p * 16 + r) * K::PITCH + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const typename K::E* b = Bs + (wn * 64 + q * 16 + r) * K::PITCH + kk;
            acc[p][q] = K::mma(a, b, g, acc[p][q]);
        }
    }
}

// FEW: two k steps at a time, so that only their operands (4 A and 4 B per
// step) are LDS reads in flight, which saves registers for occupancy; else
// the whole stage unrolled (measured faster where occupancy does not change)
template <int KIND, bool FEW>
__device__ __forceinline__ void tile_mma(const typename Kind<KIND>::E* As, const typename Kind<KIND>::E* Bs,
                                         typename Kind<KIND>::Acc (&acc)[4][4]) {
    using K = Kind<KIND>;
    if constexpr (FEW) {
#pragma unroll 2
        for (int kk = 0; kk < K::KT; kk += K::KSTEP) tile_step<KIND>(As, Bs, kk, acc);
    } else {
#pragma unroll
        for (int kk = 0; kk < K::KT; kk += K::KSTEP) tile_step<KIND>(As, Bs, kk, acc);
    }
}

template <int KIND, typename TA, typename TB>
__global__ __launch_bounds__(NT) void k_nt_mfma(const TA* __restrict__ A, const TB* __restrict__ B, int m, int n,
                                                long K, long kslice, int splits, double* __restrict__ part) {
    using Kd = Kind<KIND>;
    using E = typename Kd::E;
    constexpr int KT = Kd::KT;
    __shared__ __attribute__((aligned(16))) E As[BM * Kd::PITCH];
    __shared__ __attribute__((aligned(16))) E Bs[BN * Kd::PITCH];
    // group: K slice; member: output tile
    const int tn = (n + BN - 1) / BN, tm = (m + BM - 1) / BM;
    long slice;
    int tile;
    xcd_block(tn * tm, slice, tile);
    if (slice >= splits) return;   // padding of the last XCD round (an empty slice still writes its zeros)
    const long kb = slice * kslice;
    const int j0 = (tile % tn) * BN, i0 = (tile / tn) * BM;
    const long ke = min(K, kb + kslice);
    typename Kd::Acc acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = typename Kd::Acc{0, 0, 0, 0};
    // Software pipeline: the global loads of the next K stage are in flight
    // (in registers) while the current stage is multiplied out of LDS.
    // Stage element e of thread t: row (t + NT e) / KT, k (t + NT e) % KT;
    // 32 consecutive threads read 32 consecutive k of one row.
    constexpr int PER = BM * KT / NT;
    TA ra[PER];
    TB rb[PER];
    // element offsets within a stage are below BM K < 2^31 (checked at
    // launch): one uniform 64-bit base per stage and a 32-bit offset per
    // element, shared by A and B, instead of a 64-bit address per element
    const int Ki = (int)K;
    auto load = [&](long k0) {
        const TA* __restrict__ Ab = A + (size_t)i0 * K + k0;
        const TB* __restrict__ Bb = B + (size_t)j0 * K + k0;
        const int kl = (int)(ke - k0);   // k of this stage below kl
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + NT * e;
            const int rr = idx / KT, kk = idx % KT;
            const int off = rr * Ki + kk;
            ra[e] = (i0 + rr < m && kk < kl) ? Ab[off] : TA(0);
            rb[e] = (j0 + rr < n && kk < kl) ? Bb[off] : TB(0);
        }
    };
    if (kb < ke) load(kb);
    for (long k0 = kb; k0 < ke; k0 += KT) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + NT * e;
            const int rr = idx / KT, kk = idx % KT;
            As[rr * Kd::PITCH + kk] = Kd::cvt(ra[e]);
            Bs[rr * Kd::PITCH + kk] = Kd::cvt(rb[e]);
        }
        __syncthreads();
        if (k0 + KT < ke) load(k0 + KT);
        tile_mma<KIND, KIND == ACE_F64>(As, Bs, acc);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    double* P = part + (size_t)slice * m * n;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wm * 64 + p * 16 + Kd::row(lane >> 4, v);
                const int j = j0 + wn * 64 + q * 16 + (lane & 15);
                if (i < m && j < n) P[(size_t)i * n + j] = (double)acc[p][q][v];
            }
}

__global__ void k_slice_sum(const double* __restrict__ part, int splits, int mn, double alpha,
                            double* __restrict__ C) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= mn) return;
    double s = 0.0;
    for (int q = 0; q < splits; ++q) s += part[(size_t)q * mn + t];
    C[t] = alpha * s;
}

template <typename T>
__device__ __forceinline__ T store_as(double v);
template <>
__device__ __forceinline__ double store_as<double>(double v) { return v; }
template <>
__device__ __forceinline__ float store_as<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ uint16_t store_as<uint16_t>(double v) { return f_to_bf((float)v); }

template <int KIND, typename TB, typename TC>
__global__ __launch_bounds__(NT) void k_nn_mfma(const double* __restrict__ A, long sai, long sak,
                                                const TB* __restrict__ B, int m, int K, long ncol, double alpha,
                                                TC* __restrict__ C) {
    using Kd = Kind<KIND>;
    using E = typename Kd::E;
    constexpr int KT = Kd::KT;
    __shared__ __attribute__((aligned(16))) E As[BM * Kd::PITCH];
    __shared__ __attribute__((aligned(16))) E Bs[BN * Kd::PITCH];
    // group: column tile of B; member: row block
    long jt;
    int ib;
    xcd_block((m + BM - 1) / BM, jt, ib);
    const long j0 = jt * BN;
    if (j0 >= ncol) return;   // padding of the last XCD round
    const int i0 = ib * BM;
    typename Kd::Acc acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = typename Kd::Acc{0, 0, 0, 0};
    // Same pipeline as the NT kernel.  A (small, cache-resident): row
    // idx / KT, k idx % KT; B: 128 consecutive threads read one grid row.
    constexpr int PER = BM * KT / NT;
    double ra[PER];
    TB rb[PER];
    auto load = [&](int k0) {
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + NT * e;
            const int rr = idx / KT, kk = idx % KT;
            ra[e] = (i0 + rr < m && k0 + kk < K) ? A[(i0 + rr) * sai + (long)(k0 + kk) * sak] : 0.0;
            const int jj = idx % BN, kr = idx / BN;
            const long j = j0 + jj;
            rb[e] = (j < ncol && k0 + kr < K) ? B[(size_t)(k0 + kr) * ncol + j] : TB(0);
        }
    };
    load(0);
    for (int k0 = 0; k0 < K; k0 += KT) {
        __syncthreads();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + NT * e;
            As[(idx / KT) * Kd::PITCH + idx % KT] = Kd::cvt(ra[e]);
            Bs[(idx % BN) * Kd::PITCH + idx / BN] = Kd::cvt(rb[e]);
        }
        __syncthreads();
        if (k0 + KT < K) load(k0 + KT);
        tile_mma<KIND, std::is_same<TB, double>::value>(As, Bs, acc);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = i0 + wm * 64 + p * 16 + Kd::row(lane >> 4, v);
                const long j = j0 + wn * 64 + q * 16 + (lane & 15);
                if (i < m && j < ncol) C[(size_t)i * ncol + j] = store_as<TC>(alpha * (double)acc[p][q][v]);
            }
}

}  // namespace

int ace_mfma_splits(long K, int m, int n, int max_splits) {
    const long tiles = (long)((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    long s = (1024 + tiles - 1) / tiles;
    const long maxs = (K + 2047) / 2048;
    if (s > maxs) s = maxs;
    if (max_splits > 0 && s > max_splits) s = max_splits;
    if (s < 1) s = 1;
    return (int)s;
}

template <int KIND, typename TA, typename TB>
hipError_t ace_mm_nt(const TA* A, const TB* B, int m, int n, long K, double alpha, double* part, double* C,
                     hipStream_t s, int max_splits) {
    if ((long)BM * K >= 0x7fffffffL) return hipErrorInvalidValue;   // 32-bit element offsets of a stage
    const int splits = ace_mfma_splits(K, m, n, max_splits);
    long kslice = (K + splits - 1) / splits;
    kslice = (kslice + Kind<KIND>::KT - 1) / Kind<KIND>::KT * Kind<KIND>::KT;
    const long nb = xcd_grid(splits, ((n + BN - 1) / BN) * ((m + BM - 1) / BM));
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_nt_mfma<KIND, TA, TB>), dim3((unsigned)nb), dim3(NT), 0, s, A, B, m, n, K, kslice, splits,
                       part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int mn = m * n;
    hipLaunchKernelGGL(k_slice_sum, dim3((mn + 255) / 256), dim3(256), 0, s, part, splits, mn, alpha, C);
    return hipGetLastError();
}

template <int KIND, typename TB, typename TC>
hipError_t ace_mm_nn(const double* A, long sai, long sak, const TB* B, int m, int K, long ncol, double alpha, TC* C,
                     hipStream_t s) {
    const long nb = xcd_grid((ncol + BN - 1) / BN, (m + BM - 1) / BM);
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_nn_mfma<KIND, TB, TC>), dim3((unsigned)nb), dim3(NT), 0, s, A, sai, sak, B, m, K, ncol, alpha,
                       C);
    return hipGetLastError();
}

#define NT_INST(KIND, TA, TB) \
    template hipError_t ace_mm_nt<KIND, TA, TB>(const TA*, const TB*, int, int, long, double, double*, double*, \
                                                hipStream_t, int);
#define NN_INST(KIND, TB, TC)                                                                                      \
    template hipError_t ace_mm_nn<KIND, TB, TC>(const double*, long, long, const TB*, int, int, long, double, TC*, \
                                                hipStream_t);
// M and the energy (FP64 operands; xi converted exactly), dV xi^T psi per ace_dtype
NT_INST(ACE_F64, double, double)
NT_INST(ACE_F64, double, float)
NT_INST(ACE_F64, double, uint16_t)
NT_INST(ACE_F32, float, float)
NT_INST(ACE_BF16, uint16_t, uint16_t)
// xi = L^-1 W and K psi = -C^T xi per ace_dtype
NN_INST(ACE_F64, double, double)
NN_INST(ACE_F32, double, float)
NN_INST(ACE_F32, float, float)
NN_INST(ACE_BF16, double, uint16_t)
NN_INST(ACE_BF16, uint16_t, float)
