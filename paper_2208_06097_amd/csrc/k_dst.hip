// Spectral start for the pair Poisson solves (an extension of the CG start
// guess of Eq. 9; the CG still drives every pair to the same true residual).
//
// A is the O(h^12) Laplacian (negated) with zero values beyond the domain.
// The same stencil with odd (instead of zero) continuation beyond each face,
// A_odd, is diagonalized exactly by the type-I discrete sine transform: for
// the mode sin((i+1) theta), theta = pi m / (n+1), one axis contributes
// -(c0 + 2 sum_k ck cos(k theta)) / h^2.  The two differ only where the
// stencil reaches past a face: D = A - A_odd lives on the 5 points next to
// each face.  With x0 the multipole potential of Eq. 10 (the ghost values'
// own expansion, continued inside), the start is
//   x = x0 + A_odd^-1 (b - A x0) = A_odd^-1 (b - D x0),
// whose right-hand side the gather and the boundary kernels form (D x0 needs
// x0 on those points only, which the ghost-value kernels evaluate from the
// same line coefficients).  x leaves a residual many decades below that of
// x0 because x0 already carries the multipole potential that sets the
// boundary values; the CG's exit test then takes the true residual b - A x,
// formed in FP64 by a stencil sweep over the whole domain.
//
// The transform along one axis is a dense product with the symmetric,
// orthogonal matrix S_n[j][k] = sqrt(2/(n+1)) sin(pi (j+1)(k+1)/(n+1))
// (n <= 64 here, so a 64 x 64 product on the matrix cores beats an FFT of
// this length on this part).  Three passes over a pair's array, each one
// read and one write: the forward 2-D transform of every z plane (two
// products in LDS), then along z the forward transform, the division by
// lambda and the inverse transform (S is its own inverse) in one tile, then
// the inverse 2-D transform of every plane into x.  FP64 throughout; pairs
// with an axis longer than 64 keep the multipole start.
#include "sea_internal.h"

namespace {

constexpr int DS_BS = 256;
constexpr int DS_N = 64;        // longest axis handled
constexpr int DS_TC = 64;       // columns per z-line tile
constexpr int DS_OPN = 2048;    // operand table entries per length n
constexpr double kPiD = 3.14159265358979323846;
// second-derivative weights of the O(h^12) central difference (App. C)
constexpr double kW[7] = {-5369.0 / 1800.0, 12.0 / 7.0, -15.0 / 56.0, 10.0 / 189.0,
                          -1.0 / 112.0, 2.0 / 1925.0, -1.0 / 16632.0};

__host__ __device__ constexpr int mu_off(int n) { return (n - 1) * n / 2; }   // sum of m, m < n

// Even/odd split.  With S[j][n-1-k] = (-1)^j S[j][k], the transform of a
// vector a of length n is, for h = floor(n/2),
//   y_{2i}   = sum_{k<h} S[2i][k]   (a_k + a_{n-1-k})  (+ S[2i][h] a_h, n odd)
//   y_{2i+1} = sum_{k<h} S[2i+1][k] (a_k - a_{n-1-k}),
// two products of half the size: half the flops of the dense product.
// The kernels fold a column as p_k = a_k + a_{n-1-k}, m_k = a_k - a_{n-1-k}
// for k < h and p_k = m_k = a_k beyond; the table below is zero where a
// folded entry must not count (k > h; k = h unless n is odd and the row
// even), so both are read with one rule.
//
// Operand table of length n: entry ((par * 2 + b) * 8 + kk) * 64 + lane
// holds S[2 i + par][k] for i = 16 b + lane % 16, k = 4 kk + lane / 16, the
// matrix-core operand of lane `lane` at k step kk for output block b of
// parity par (as A: rows i; as B: columns i; the same lanes either way).
__global__ __launch_bounds__(DS_BS) void k_dst_tables(double* __restrict__ opt, double* __restrict__ mu) {
    const int n = blockIdx.x + 1;
    double* On = opt + (size_t)(n - 1) * DS_OPN;
    const double sc = sqrt(2.0 / (n + 1));
    const int h = n / 2;
    for (int t = threadIdx.x; t < DS_OPN; t += DS_BS) {
        const int par = t >> 10, b = (t >> 9) & 1, kk = (t >> 6) & 7, lane = t & 63;
        const int j = 2 * (16 * b + (lane & 15)) + par, k = 4 * kk + (lane >> 4);
        const bool use = j < n && (k < h || (k == h && (n & 1) && par == 0));
        double v = 0.0;
        if (use) {
            const int m = ((j + 1) * (k + 1)) % (2 * (n + 1));   // argument reduced to [0, 2 pi)
            v = sc * sin(kPiD * (double)m / (double)(n + 1));
        }
        On[t] = v;
    }
    for (int m = threadIdx.x; m < n; m += DS_BS) {
        const double th = kPiD * (double)(m + 1) / (double)(n + 1);
        double s = kW[0];
#pragma unroll
        for (int k = 1; k <= 6; ++k) s += 2.0 * kW[k] * cos(k * th);
        mu[mu_off(n) + m] = -s;
    }
}

struct DstArgs {
    const sea_pair* pairs;
    const DevCell* cells;
    const int* pair_cell;
    size_t stride;
    const double* in;
    double* out;
    const double* opt;
    const double* mu;
    const double* add;    // plane pass: added to `in` on the face points (nullable)
    const int* skip;      // pairs to leave alone (nullable)
};

// Products on the FP64 matrix cores (v_mfma_f64_16x16x4f64), 4 waves per
// workgroup, every product a 64 x 64 (folded: 2 x 32 x 32) one.  Operand
// lanes: row (A) or column (B) = lane % 16, k = lane / 16; result item v of
// a lane is row lane / 16 + 4 v, column lane % 16.  A wave keeps the table
// operands of its output block (both parities, all 8 k steps) in registers
// for the whole kernel, so the products issue no global loads.  One LDS
// array per workgroup holds the tile through every step (in place, with a
// barrier before each overwrite), which lets four workgroups share a CU and
// hide each other's global latency.  Its rows are padded to DP_LD (66
// doubles): every matrix-core operand read below has the row index on the
// lanes, which that pitch spreads over all banks.
typedef double dst_f64x4 __attribute__((ext_vector_type(4)));
constexpr int DP_LD = 66;
constexpr int DP_BS = 256;  // threads per workgroup
constexpr int DP_PT = DS_N * DS_N / DP_BS;   // tile elements per thread

// p, m of the fold at k for the entries a[k], a[n-1-k] of one row
__device__ __forceinline__ void dst_fold(const double* row, int n, int k, double& p, double& m) {
    const double a0 = row[k];
    const int k2 = n - 1 - k;
    const double a1 = k2 > k ? row[k2] : 0.0;
    p = a0 + a1;
    m = a0 - a1;
}

// the operands of output block b (both parities) of length n
__device__ __forceinline__ void dst_ops(const double* opt, int n, int b, int lane, double e[8], double o[8]) {
    const double* t = opt + (size_t)(n - 1) * DS_OPN + lane;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
        e[kk] = t[((0 + b) * 8 + kk) * 64];
        o[kk] = t[((2 + b) * 8 + kk) * 64];
    }
}

// 2-D transform of every z plane of a pair, Y = S_y X S_x (X[y][x], x
// contiguous), written in the plane's layout (the same kernel serves the
// forward and the inverse transform: S is its own inverse).  With `add`,
// the input is in + add on the points within 5 of a face (in elsewhere).  Grid
// (pairs, PG): workgroup y takes planes y, y + PG, ...  The LDS array
// holds X[y][x], then T transposed (T^T[c][y], c = 32 parity + i for the
// x mode 2 i + parity), then Y[j][x].  Wave w: output block w % 2 of the
// transform, row (then column) blocks 2 (w / 2) and 2 (w / 2) + 1.
// Variants (the autotuner picks PG; SQ is chosen from the pairs): PG
// workgroups per pair; SQ: every plane the call transforms is square
// (nx = ny), so one operand set serves both axes (32 fewer registers, four
// workgroups per CU instead of three).
template <int PG, bool SQ>
__global__ __launch_bounds__(DP_BS, SQ ? 4 : 3) void k_dst_plane(DstArgs d) {
    __shared__ double B[DS_N * DP_LD];
    const int pid = blockIdx.x;
    const sea_pair P = d.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    if (nx > DS_N || ny > DS_N || nz > DS_N) return;   // keeps the multipole start
    if ((int)blockIdx.y >= nz || (d.skip && d.skip[pid])) return;   // no plane here, or a pair left alone
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int hb = w & 1, bp = 2 * (w >> 1);
    double ex[8], ox[8];
    dst_ops(d.opt, nx, hb, lane, ex, ox);
    double eyb[SQ ? 1 : 8], oyb[SQ ? 1 : 8];
    if constexpr (!SQ) dst_ops(d.opt, ny, hb, lane, eyb, oyb);
    const double* ey = SQ ? ex : eyb;
    const double* oy = SQ ? ox : oyb;
    // entries outside the ny x nx corner only ever meet zero table entries;
    // they start finite and stay finite
    for (int t = threadIdx.x; t < DS_N * DP_LD; t += DP_BS) B[t] = 0.0;
    const int npl = nx * ny;
    // LDS offset y * DP_LD + x of element e = threadIdx.x + u * DP_BS
    const int x0 = threadIdx.x % nx, y0 = threadIdx.x / nx, sxs = DP_BS % nx, sys = DP_BS / nx;
    auto for_elems = [&](auto&& f) {
        int x = x0, y = y0;
        asm volatile("" : "+v"(x), "+v"(y));   // walked per plane, not precomputed and held
#pragma unroll
        for (int u = 0; u < DP_PT; ++u) {
            const int e = threadIdx.x + u * DP_BS;
            if (e < npl) f(u, e, y * DP_LD + x);
            x += sxs;
            y += sys;
            if (x >= nx) {
                x -= nx;
                ++y;
            }
        }
    };
    const double* in = d.in + (size_t)pid * d.stride;
    double* out = d.out + (size_t)pid * d.stride;
    const double* add = d.add ? d.add + (size_t)pid * d.stride : nullptr;
    for (int z = blockIdx.y; z < nz; z += PG) {
        const size_t zo = (size_t)z * npl;
        int gk = g;
        asm volatile("" : "+v"(gk));   // recompute the fold addresses per plane rather than keep them all live
        double val[DP_PT];
#pragma unroll
        for (int u = 0; u < DP_PT; ++u) {
            const int e = threadIdx.x + u * DP_BS;
            val[u] = e < npl ? in[zo + e] : 0.0;
        }
        if (add) {   // the face correction, its loads in flight with the plane's
            double ad[DP_PT];
#pragma unroll
            for (int u = 0; u < DP_PT; ++u) ad[u] = 0.0;
            const bool zf = near_face(z, nz);
            for_elems([&](int u, int e, int o) {
                const int yy = o / DP_LD, xx = o % DP_LD;
                ad[u] = (zf || near_face(xx, nx) || near_face(yy, ny)) ? add[zo + e] : 0.0;
            });
#pragma unroll
            for (int u = 0; u < DP_PT; ++u) val[u] += ad[u];
        }
        __syncthreads();
        for_elems([&](int u, int, int o) { B[o] = val[u]; });
        __syncthreads();
        // T = X S_x: rows y of blocks bp, bp + 1; x modes of block hb
        dst_f64x4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = dst_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                double p, m;
                dst_fold(B + (16 * (bp + a) + r) * DP_LD, nx, 4 * kk + gk, p, m);
                acc[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(p, ex[kk], acc[a][0], 0, 0, 0);
                acc[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(m, ox[kk], acc[a][1], 0, 0, 0);
                if (a == 1 && (kk & 1)) __builtin_amdgcn_sched_barrier(0);   // bounds the reads in flight
            }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int par = 0; par < 2; ++par)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    B[(32 * par + 16 * hb + r) * DP_LD + 16 * (bp + a) + g + 4 * v] = acc[a][par][v];
        __syncthreads();
        // Y = S_y T: columns c of blocks bp, bp + 1; y modes of block hb
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = dst_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                double p, m;
                dst_fold(B + (16 * (bp + a) + r) * DP_LD, ny, 4 * kk + gk, p, m);
                acc[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ey[kk], p, acc[a][0], 0, 0, 0);
                acc[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(oy[kk], m, acc[a][1], 0, 0, 0);
                if (a == 1 && (kk & 1)) __builtin_amdgcn_sched_barrier(0);
            }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int c = 16 * (bp + a) + r;
            const int xm = 2 * (c & 31) + (c >> 5);
#pragma unroll
            for (int par = 0; par < 2; ++par)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = 2 * (16 * hb + g + 4 * v) + par;
                    if (j < ny && xm < nx) B[j * DP_LD + xm] = acc[a][par][v];
                }
        }
        __syncthreads();
        for_elems([&](int, int e, int o) { out[zo + e] = B[o]; });
    }
}

// Along z for each column (y, x): forward transform, division by the
// eigenvalue of the mode, inverse transform; same layout in and out.  Grid
// (pairs, PG): workgroup y takes 64-column tiles y, y + PG, ...  The
// LDS array holds the tile transposed (column-major: U[c][z]), so that the
// transform along z reads rows.  Wave w: z modes of block w % 2, columns of
// blocks 2 (w / 2) and 2 (w / 2) + 1.
// Variants: PG workgroups per pair; LB: tile values loaded per batch into
// registers before they go to LDS (16: all at once, 8: two batches, fewer
// registers).
template <int PG, int LB>
__global__ __launch_bounds__(DP_BS, 4) void k_dst_zline(DstArgs d) {
    __shared__ double U[DS_TC * DP_LD];
    __shared__ double lxy[DS_TC];   // x and y parts of the eigenvalue of each tile column
    const int pid = blockIdx.x;
    const sea_pair P = d.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    if (nx > DS_N || ny > DS_N || nz > DS_N) return;
    const int ncol = nx * ny;
    if ((int)blockIdx.y * DS_TC >= ncol || (d.skip && d.skip[pid])) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int hb = w & 1, bp = 2 * (w >> 1);
    double ez[8], oz[8];
    dst_ops(d.opt, nz, hb, lane, ez, oz);
    const DevCell& Cl = d.cells[d.pair_cell[pid]];
    const double ihx = 1.0 / (Cl.h[0] * Cl.h[0]), ihy = 1.0 / (Cl.h[1] * Cl.h[1]), ihz = 1.0 / (Cl.h[2] * Cl.h[2]);
    const double* mux = d.mu + mu_off(nx);
    const double* muy = d.mu + mu_off(ny);
    const double lzj = lane < nz ? d.mu[mu_off(nz) + lane] * ihz : 0.0;   // z part for mode j = lane
    const double* in = d.in + (size_t)pid * d.stride;
    double* out = d.out + (size_t)pid * d.stride;
    // load element u of a thread: row a = threadIdx.x / 64 + 4 u, column threadIdx.x % 64
    const int lc = threadIdx.x % DS_TC, la = threadIdx.x / DS_TC;
    for (int c0 = blockIdx.y * DS_TC; c0 < ncol; c0 += PG * DS_TC) {
        int gk = g;
        asm volatile("" : "+v"(gk));   // recompute the fold addresses per tile rather than keep them all live
        const bool cl = c0 + lc < ncol;
        static_assert(DP_PT % LB == 0, "load batches");
        // the first batch's loads are in flight while the workgroup finishes
        // the previous tile (the barrier), the others go straight to LDS
        // 32-bit element offsets walked per tile (not precomputed per load and
        // held across tiles)
        int off = la * ncol + c0 + lc;
        asm volatile("" : "+v"(off));
#pragma unroll
        for (int u0 = 0; u0 < DP_PT; u0 += LB) {
            double val[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int a = la + 4 * (u0 + u);
                val[u] = (cl && a < nz) ? in[off] : 0.0;
                off += 4 * ncol;
            }
            if (u0 == 0) __syncthreads();
#pragma unroll
            for (int u = 0; u < LB; ++u) U[lc * DP_LD + la + 4 * (u0 + u)] = val[u];
        }
        if (threadIdx.x < DS_TC) {
            const int col = c0 + threadIdx.x;
            double l = 0.0;
            if (col < ncol) {
                const int yy = col / nx, xx = col - yy * nx;
                l = muy[yy] * ihy + mux[xx] * ihx;
            }
            lxy[threadIdx.x] = l;
        }
        __syncthreads();
        dst_f64x4 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = dst_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                double p, m;
                dst_fold(U + (16 * (bp + a) + r) * DP_LD, nz, 4 * kk + gk, p, m);
                acc[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ez[kk], p, acc[a][0], 0, 0, 0);
                acc[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(oz[kk], m, acc[a][1], 0, 0, 0);
                if (a == 1 && (kk & 1)) __builtin_amdgcn_sched_barrier(0);
            }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int par = 0; par < 2; ++par)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    U[(16 * (bp + a) + r) * DP_LD + 2 * (16 * hb + g + 4 * v) + par] = acc[a][par][v];
        __syncthreads();
        // divide by the eigenvalue: wave w takes columns w + 4 u, lane the mode j
        if (lane < nz) {
#pragma unroll 2
            for (int u = 0; u < DS_TC / 4; ++u) {
                const int cc = w + 4 * u;
                if (c0 + cc < ncol) U[cc * DP_LD + lane] /= lxy[cc] + lzj;
            }
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][0] = acc[a][1] = dst_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                double p, m;
                dst_fold(U + (16 * (bp + a) + r) * DP_LD, nz, 4 * kk + gk, p, m);
                acc[a][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ez[kk], p, acc[a][0], 0, 0, 0);
                acc[a][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(oz[kk], m, acc[a][1], 0, 0, 0);
                if (a == 1 && (kk & 1)) __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int col = c0 + 16 * (bp + a) + r;
            if (col >= ncol) continue;
#pragma unroll
            for (int par = 0; par < 2; ++par)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = 2 * (16 * hb + g + 4 * v) + par;
                    if (j < nz) out[j * ncol + col] = acc[a][par][v];   // 32-bit offsets (< 64^3)
                }
        }
    }
}

}  // namespace

size_t dst_table_doubles() { return (size_t)DS_N * DS_OPN; }
size_t dst_mu_doubles() { return (size_t)mu_off(DS_N + 1); }

// Compiled variants of the two transform kernels, the autotuner's choices.
namespace {
using DstKernel = void (*)(DstArgs);
struct PlaneVariant {
    const char* name;
    DstKernel gen, sq;   // general planes / every plane square
    int pg;
};
struct ZlineVariant {
    const char* name;
    DstKernel fn;
    int pg;
};
const PlaneVariant kPlaneVariants[] = {
    {"plane-pg16", k_dst_plane<16, false>, k_dst_plane<16, true>, 16},
    {"plane-pg8", k_dst_plane<8, false>, k_dst_plane<8, true>, 8},
    {"plane-pg32", k_dst_plane<32, false>, k_dst_plane<32, true>, 32},
};
const ZlineVariant kZlineVariants[] = {
    {"zline-pg16-lb16", k_dst_zline<16, 16>, 16},
    {"zline-pg16-lb8", k_dst_zline<16, 8>, 16},
    {"zline-pg32-lb16", k_dst_zline<32, 16>, 32},
    {"zline-pg8-lb16", k_dst_zline<8, 16>, 8},
};
constexpr int kNumPlane = sizeof(kPlaneVariants) / sizeof(kPlaneVariants[0]);
constexpr int kNumZline = sizeof(kZlineVariants) / sizeof(kZlineVariants[0]);
}  // namespace

int dst_variant_count() { return kNumPlane + kNumZline; }
int dst_plane_variant_count() { return kNumPlane; }
const char* dst_variant_name(int v) {
    if (v >= 0 && v < kNumPlane) return kPlaneVariants[v].name;
    if (v >= kNumPlane && v < kNumPlane + kNumZline) return kZlineVariants[v - kNumPlane].name;
    return nullptr;
}

namespace {
DstArgs dst_args(const ExxArgs& a, double* tab, double* mu) {
    DstArgs d{};
    d.pairs = a.pairs;
    d.cells = a.cells;
    d.pair_cell = a.pair_cell;
    d.stride = a.stride;
    d.opt = tab;
    d.mu = mu;
    return d;
}
void launch_plane(const DstArgs& d, int n_pairs, int pv, bool square, hipStream_t s) {
    const PlaneVariant& V = kPlaneVariants[pv];
    hipLaunchKernelGGL(square ? V.sq : V.gen, dim3((unsigned)n_pairs, V.pg), dim3(DP_BS), 0, s, d);
}
void launch_zline(const DstArgs& d, int n_pairs, int zv, hipStream_t s) {
    const ZlineVariant& V = kZlineVariants[zv];
    hipLaunchKernelGGL(V.fn, dim3((unsigned)n_pairs, V.pg), dim3(DP_BS), 0, s, d);
}
}  // namespace

hipError_t launch_dst_tables(double* tab, double* mu, hipStream_t s) {
    hipLaunchKernelGGL(k_dst_tables, dim3(DS_N), dim3(DS_BS), 0, s, tab, mu);
    return hipGetLastError();
}

// One transform pass of a variant on every pair (autotuner): pass 0 forward
// planes (in -> out, no face correction), 1 z lines, 2 inverse planes.
hipError_t launch_dst_pass(const ExxArgs& a, int pass, int variant, bool square, const double* in, double* out,
                           double* tab, double* mu, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    DstArgs d = dst_args(a, tab, mu);
    d.in = in;
    d.out = out;
    if (pass == 1) launch_zline(d, a.n_pairs, variant, s);
    else launch_plane(d, a.n_pairs, variant, square, s);
    return hipGetLastError();
}

hipError_t launch_dst_solve(const ExxArgs& a, const double* r, double* z, double* tmp, double* tmp2, double* tab,
                            double* mu, int pv, int zv, bool square, const int* skip, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    if (pv < 0 || pv >= kNumPlane || zv < 0 || zv >= kNumZline) return hipErrorInvalidValue;
    DstArgs d = dst_args(a, tab, mu);
    d.skip = skip;
    d.in = r;
    d.out = tmp;
    launch_plane(d, a.n_pairs, pv, square, s);
    d.in = tmp;
    d.out = tmp2;
    launch_zline(d, a.n_pairs, zv, s);
    d.in = tmp2;
    d.out = z;
    launch_plane(d, a.n_pairs, pv, square, s);
    return hipGetLastError();
}

// x = S^-1 ((S (b + fcorr)) ./ lambda) for every pair whose axes are all <=
// 64 (fcorr added on the face points; it lives in tmp, scratch of the pair
// arrays' size, which the passes then overwrite); r is scratch of the same
// size.  pv, zv: plane and z-line variants; square: every pair the
// transform takes has nx = ny.
hipError_t launch_spectral_start(const ExxArgs& a, double* r, double* tmp, double* tab, double* mu, int pv, int zv,
                                 bool square, hipStream_t s, const std::function<void(int, bool)>& mark) {
    if (a.n_pairs <= 0) return hipSuccess;
    if (pv < 0 || pv >= kNumPlane || zv < 0 || zv >= kNumZline) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dst_tables, dim3(DS_N), dim3(DS_BS), 0, s, tab, mu);
    DstArgs d = dst_args(a, tab, mu);
    // planes forward: b + fcorr (in tmp) -> tmp; z lines forward, divided,
    // inverse: tmp -> r; planes inverse: r -> x
    d.in = a.b;
    d.add = tmp;
    d.out = tmp;
    mark(0, true);
    launch_plane(d, a.n_pairs, pv, square, s);
    mark(0, false);
    d.add = nullptr;
    d.in = tmp;
    d.out = r;
    mark(1, true);
    launch_zline(d, a.n_pairs, zv, s);
    mark(1, false);
    d.in = r;
    d.out = a.v;
    mark(2, true);
    launch_plane(d, a.n_pairs, pv, square, s);
    mark(2, false);
    return hipGetLastError();
}
