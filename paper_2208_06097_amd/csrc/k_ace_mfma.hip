// ACE products on the matrix cores (Eq. 18-19): the two shapes of the ACE
// build and apply, for FP64, FP32 and BF16 operands.
//
//   NT (long K):  C = alpha A B^T, A: m x K, B: n x K, K = grid points.
//                 Split over K; every workgroup writes an FP64 partial
//                 m x n block of its K slice and a second kernel sums the
//                 slices in FP64 (M = dV Phi^T W, dV xi^T psi, dV Phi^T xi).
//   NN (small K): C = alpha A B, A: m x K (FP64, small), B: K x ncol,
//                 ncol = grid points (xi = L^-1 W, K psi = -C^T xi).
//                 Persistent workgroups walk the column tiles with the
//                 next tile's first K stage loaded during the last stage.
//
// Operand kinds: FP64 -> v_mfma_f64_16x16x4f64 (FP64 accumulation);
// FP32 -> v_mfma_f32_16x16x4f32 and BF16 -> v_mfma_f32_16x16x32_bf16, both
// with FP32 accumulation inside a workgroup's K range.  Inputs of another
// type are rounded to the operand kind while they are staged in LDS.
//
// Tiling: 256 threads, a 128 x 128 output block, four wavefronts of 64 x 64
// (4 x 4 tiles of 16 x 16), K staged as [row][k] in LDS (FP64 16 at a time,
// FP32 32 at a time in the NT product and 16 in the NN one, BF16 32).
// Operand lanes: A row = lane % 16, B column = lane % 16, k block = lane / 16.
// Result lanes: column = lane % 16; the row of item v is 4 (lane / 16) + v
// for the FP32-accumulating instructions and lane / 16 + 4 v for the FP64
// one (measured on gfx950).
#include <algorithm>
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
template <int KIND, int PITCH = Kind<KIND>::PITCH>
__device__ __forceinline__ void tile_step(const typename Kind<KIND>::E* As, const typename Kind<KIND>::E* Bs, int kk,
                                          typename Kind<KIND>::Acc (&acc)[4][4]) {
    using K = Kind<KIND>;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const typename K::E* a = As + (wm * 64 + p * 16 + r) * PITCH + kk;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const typename K::E* b = Bs + (wn * 64 + q * 16 + r) * PITCH + kk;
            acc[p][q] = K::mma(a, b, g, acc[p][q]);
        }
    }
}

// FEW: two k steps at a time, so that only their operands (4 A and 4 B per
// step) are LDS reads in flight, which saves registers for occupancy; else
// the whole stage unrolled (measured faster where occupancy does not change).
// KT, PITCH: the stage depth and LDS row pitch, if not the kind's own.
template <int KIND, bool FEW, int KT = Kind<KIND>::KT, int PITCH = Kind<KIND>::PITCH>
__device__ __forceinline__ void tile_mma(const typename Kind<KIND>::E* As, const typename Kind<KIND>::E* Bs,
                                         typename Kind<KIND>::Acc (&acc)[4][4]) {
    using K = Kind<KIND>;
    if constexpr (FEW) {
#pragma unroll 2
        for (int kk = 0; kk < KT; kk += K::KSTEP) tile_step<KIND, PITCH>(As, Bs, kk, acc);
    } else {
#pragma unroll
        for (int kk = 0; kk < KT; kk += K::KSTEP) tile_step<KIND, PITCH>(As, Bs, kk, acc);
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

// Persistent: `slots` workgroups per (XCD, row block), all resident at once.
// Workgroup k runs on XCD x = k % 8; with q = k / 8 it takes row block
// q % (row blocks) and slot s = q / (row blocks), and walks the column tiles
// jt = (s + i slots) 8 + x, i = 0, 1, ..., so that the row blocks of one
// column tile run together on one XCD (the second read of the tile comes
// from that L2).  The first K stage of the next column tile is loaded
// during the last stage of the current one: the pipeline does not drain
// between tiles (K is short here: the orbital count).
//
// Workgroups per CU asked of the compiler, which then keeps the
// accumulators in VGPRs: FP64 and BF16 two (the FP64 kind otherwise takes
// 194 VGPRs + 128 AGPRs and runs one workgroup per CU; three spill); FP32
// three, with K staged 16 at a time (32 at a time spills at three).
template <int KIND>
constexpr int nn_kt() { return KIND == ACE_F32 ? 16 : Kind<KIND>::KT; }
template <int KIND>
constexpr int nn_pitch() { return nn_kt<KIND>() == Kind<KIND>::KT ? Kind<KIND>::PITCH : nn_kt<KIND>() + 1; }
template <int KIND>
constexpr int nn_minb() { return KIND == ACE_F32 ? 3 : 2; }
template <int KIND, typename TB, typename TC>
__global__ __launch_bounds__(NT, nn_minb<KIND>()) void k_nn_mfma(const double* __restrict__ A, long sai, long sak,
                                                const TB* __restrict__ B, int m, int K, long ncol, double alpha,
                                                TC* __restrict__ C, int slots) {
    using Kd = Kind<KIND>;
    using E = typename Kd::E;
    constexpr int KT = nn_kt<KIND>(), PITCH = nn_pitch<KIND>();
    __shared__ __attribute__((aligned(16))) E As[BM * PITCH];
    __shared__ __attribute__((aligned(16))) E Bs[BN * PITCH];
    const int per = (m + BM - 1) / BM;
    const int x = blockIdx.x % ACE_XCD, mseq = blockIdx.x / ACE_XCD;
    const int i0 = (mseq % per) * BM;
    const long ntile = (ncol + BN - 1) / BN, jstep = (long)slots * ACE_XCD;
    long jt = (long)(mseq / per) * ACE_XCD + x;
    if (jt >= ntile) return;
    const int nst = K > 0 ? (K + KT - 1) / KT : 1;   // K = 0: one stage of zeros
    typename Kd::Acc acc[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = typename Kd::Acc{0, 0, 0, 0};
    // Same stage layout as the NT kernel.  A (small, cache-resident): row
    // idx / KT, k idx % KT; B: 128 consecutive threads read one grid row.
    constexpr int PER = BM * KT / NT;
    double ra[PER];
    TB rb[PER];
    // Element e of a thread: A row rr0 + e NT/KT, k kk; B row kr0 + e NT/BN,
    // column jj.  Its address is a uniform base for (stage, e) plus a 32-bit
    // offset of the thread's own (the same for every e); the thread index is
    // taken opaque in each call, so that nothing of it is held in registers
    // across the tile loop.
    auto load = [&](long j0, int k0) {
        int t = threadIdx.x;
        asm volatile("" : "+v"(t));
        const int rr0 = t / KT, kk = t % KT, kr0 = t / BN, jj = t % BN;
        const int oa = rr0 * (int)sai + kk * (int)sak, ob = kr0 * (int)ncol + jj;
        const int kl = K - k0, il = m - i0;
        const long jl = ncol - j0;
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const double* __restrict__ Ae = A + i0 * sai + (long)k0 * sak + (long)e * (NT / KT) * sai;
            const TB* __restrict__ Be = B + (size_t)(k0 + e * (NT / BN)) * ncol + j0;
            ra[e] = (rr0 + e * (NT / KT) < il && kk < kl) ? Ae[oa] : 0.0;
            rb[e] = (jj < jl && kr0 + e * (NT / BN) < kl) ? Be[ob] : TB(0);
        }
    };
    const int wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    load(jt * BN, 0);
    for (int st = 0;;) {
        // LDS-only barriers: the loads in flight cross them (their
        // registers are waited for where they are staged)
        lds_sync();
#pragma unroll
        for (int e = 0; e < PER; ++e) {
            const int idx = threadIdx.x + NT * e;
            As[(idx / KT) * PITCH + idx % KT] = Kd::cvt(ra[e]);
            Bs[(idx % BN) * PITCH + idx / BN] = Kd::cvt(rb[e]);
        }
        lds_sync();
        long jn = jt;
        int sn = st + 1;
        if (sn == nst) {
            sn = 0;
            jn = jt + jstep;
        }
        if (jn < ntile) load(jn * BN, sn * KT);
        tile_mma<KIND, std::is_same<TB, double>::value, KT, PITCH>(As, Bs, acc);
        if (sn == 0) {
            int lane = threadIdx.x & 63;
            asm volatile("" : "+v"(lane));
            const int ib = i0 + wm * 64, il = m - ib;
            const long jb = jt * BN + wn * 64, jl = ncol - jb;
            TC* __restrict__ Cb = C + (size_t)ib * ncol + jb;
#pragma unroll
            for (int p = 0; p < 4; ++p)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = p * 16 + Kd::row(lane >> 4, v), j = q * 16 + (lane & 15);
                        if (i < il && j < jl) Cb[(size_t)i * ncol + j] = store_as<TC>(alpha * (double)acc[p][q][v]);
                    }
                    acc[p][q] = typename Kd::Acc{0, 0, 0, 0};
                }
            if (jn >= ntile) break;
        }
        jt = jn;
        st = sn;
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
    if (m <= 0 || ncol <= 0) return hipSuccess;
    // resident workgroups per CU of this instantiation and the CU count,
    // queried once per process (a thread-safe static initialization)
    struct Fill {
        hipError_t err;
        int occ, n_cu;
    };
    static const Fill fill = [] {
        int dev = 0, o = 0, c = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k_nn_mfma<KIND, TB, TC>, NT, 0);
        if (e == hipSuccess && (o < 1 || c < 1)) e = hipErrorInvalidValue;
        return Fill{e, o, c};
    }();
    if (fill.err != hipSuccess) return fill.err;
    const int occ = fill.occ, n_cu = fill.n_cu;
    const int per = (m + BM - 1) / BM;
    const long ntile = (ncol + BN - 1) / BN;
    // as many slots as stay resident (at least one), no more than the tiles need
    long slots = (long)n_cu * occ / ((long)ACE_XCD * per);
    slots = std::max(1L, std::min(slots, (ntile + ACE_XCD - 1) / ACE_XCD));
    const long nb = slots * ACE_XCD * per;
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    // a thread's 32-bit offsets: A rows below NT / KT, k below KT; B rows 0, 1
    constexpr int KT = nn_kt<KIND>();
    if (sai < 0 || sak < 0 || (long)(NT / KT) * sai + (long)KT * sak >= 0x7fffffffL ||
        2 * ncol + BN >= 0x7fffffffL)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_nn_mfma<KIND, TB, TC>), dim3((unsigned)nb), dim3(NT), 0, s, A, sai, sak, B, m, K, ncol, alpha,
                       C, (int)slots);
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
