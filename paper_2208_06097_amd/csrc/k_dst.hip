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
// (n <= 64 here, so a product on the matrix cores beats an FFT of this
// length on this part), folded by its even/odd symmetry once (any n: two
// 32 x 32 products) or twice (odd n: four 16 x 16 products, half the
// matrix-core work).  Three passes over a pair's array, each one
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
constexpr int DS_OPN2 = 1024;   // second-level operand table entries per odd length n
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
//
// Second-level fold (n odd, N = (n + 1) / 2 <= 32).  With m = k + 1 the even
// modes are y_{2i} = sum_{k < N} p_k S[2i][k] and S[2 (N-1-i)][k] =
// (-1)^(m+1) S[2i][k]; so for i < ceil(N/2) the sum over odd k (E_i) and the
// sum over even k (O_i) give two modes, y_{2i} = E_i + O_i and
// y_{2 (N-1-i)} = O_i - E_i.  The odd modes y_{2i'+1} = sum_{k < N-1} m_k
// S[2i'+1][k] are, up to the scale, a type-I sine transform of length N - 1,
// which folds like the first level: pp_k = m_k + m_{N-2-k} gives the modes
// 4i + 1, mm_k = m_k - m_{N-2-k} the modes 4i + 3.  Four 16 x 16 products
// (K = 16) per 16 lines instead of two 32 x 32: half the matrix-core work.
// Second-level table of odd length n (after the 64 first-level ones): entry
// (q * 4 + kk) * 64 + lane holds, for output index i = lane % 16 and
// k' = 4 kk + lane / 16, the operand of product q (0: E, k = 2k' + 1; 1: O,
// k = 2k'; 2: pp; 3: mm), zero where the term does not count.
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
    if (n & 1) {
        double* O2 = opt + (size_t)DS_N * DS_OPN + (size_t)(n - 1) * DS_OPN2;
        const int N = (n + 1) / 2, Ne = (N + 1) / 2, n2 = N - 1, h2 = n2 / 2;
        for (int t = threadIdx.x; t < DS_OPN2; t += DS_BS) {
            const int q = t >> 8, kk = (t >> 6) & 3, lane = t & 63;
            const int i = lane & 15, kp = 4 * kk + (lane >> 4);
            int m = -1;   // the sine of pi m / (n + 1), m reduced below
            if (q < 2) {
                const int k = 2 * kp + (q == 0 ? 1 : 0);
                if (i < Ne && k <= N - 1) m = (2 * i + 1) * (k + 1);
            } else {
                const int i2 = 2 * i + (q - 2);   // index in the odd part
                const bool kin = kp < h2 || (q == 2 && kp == h2 && (n2 & 1));
                if (i2 <= N - 2 && kin) m = 2 * (i2 + 1) * (kp + 1);
            }
            double v = 0.0;
            if (m >= 0) v = sc * sin(kPiD * (double)(m % (2 * (n + 1))) / (double)(n + 1));
            O2[t] = v;
        }
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
    size_t stride;        // pair layout (b, x, the face corrections)
    size_t pstride;       // the padded intermediates
    const double* in;
    double* out;
    const double* opt;
    const double* mu;
    const double* add;    // plane pass: added to `in` on the face points (nullable, pair layout)
    int in_pad, out_pad;  // plane pitch of in / out: dst_plane_pitch(nx*ny, pad); a plane
                          // pass with out_pad is the forward one (pair layout in, padded
                          // out), without it the inverse (padded in, pair layout out)
    const int* skip;      // pairs to leave alone (nullable)
    int pair0;            // z-line pass: first pair of the launch (long calls run in chunks)
};

// Products on the FP64 matrix cores (v_mfma_f64_16x16x4f64), 4 waves per
// workgroup, every product a 64 x 64 one (folded: 2 x 32 x 32, or for odd
// lengths 4 x 16 x 16).  Operand
// lanes: row (A) or column (B) = lane % 16, k = lane / 16; result item v of
// a lane is row lane / 16 + 4 v, column lane % 16.  A wave keeps the table
// operands of its output block (both parities, all 8 k steps; or the four
// second-level products, all 4 k steps) in registers
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

// the second-level operands of odd length n
__device__ __forceinline__ void dst_ops2(const double* opt, int n, int lane, double t[16]) {
    const double* p = opt + (size_t)DS_N * DS_OPN + (size_t)(n - 1) * DS_OPN2 + lane;
#pragma unroll
    for (int e = 0; e < 16; ++e) t[e] = p[e * 64];
}

// mode of output index i of product group q in the second-level fold
// (0: 2i from E + O; 1: 2 (N-1-i) from O - E; 2: 4i + 1; 3: 4i + 3), -1 if none
__device__ __forceinline__ int dst_mode2(int q, int i, int N) {
    const int Ne = (N + 1) >> 1;
    if (q == 0) return i < Ne ? 2 * i : -1;
    if (q == 1) return (i < Ne && N - 1 - i > i) ? 2 * (N - 1 - i) : -1;
    if (q == 2) return 2 * i <= N - 2 ? 4 * i + 1 : -1;
    return 2 * i + 1 <= N - 2 ? 4 * i + 3 : -1;
}

// value of product group q from the four products
__device__ __forceinline__ double dst_val2(const dst_f64x4 acc[4], int q, int v) {
    return q == 0 ? acc[0][v] + acc[1][v] : (q == 1 ? acc[1][v] - acc[0][v] : acc[q][v]);
}

// The four second-level products of a block of 16 lines (odd length n):
// `row` is this lane's line (lane % 16 of the block) in LDS.  DATA_A: the
// lines are the A operand (result v of a lane: line lane / 16 + 4 v, output
// index lane % 16); else the B operand (output index lane / 16 + 4 v, line
// lane % 16).
template <bool DATA_A>
__device__ __forceinline__ void dst_xform2(const double* row, int n, int g, const double t[16], dst_f64x4 acc[4]) {
    const int N = (n + 1) >> 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = dst_f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        const int kp = 4 * kk + g;
        const int k1 = 2 * kp + 1, k0 = 2 * kp, k2 = N - 2 - kp;
        // first level at k = 2k' + 1 and 2k' (p), and at k' and N - 2 - k' (m;
        // the partner of N - 2 - k' is N + k')
        const double e1 = row[k1] + (n - 1 - k1 > k1 ? row[n - 1 - k1] : 0.0);
        const double e0 = row[k0] + (n - 1 - k0 > k0 ? row[n - 1 - k0] : 0.0);
        const double m0 = row[kp] - (n - 1 - kp > kp ? row[n - 1 - kp] : 0.0);
        const double m2 = k2 > kp ? row[k2] - row[N + kp] : 0.0;
        const double pp = m0 + m2, mm = m0 - m2;
        if constexpr (DATA_A) {
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(e1, t[kk], acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(e0, t[4 + kk], acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(pp, t[8 + kk], acc[2], 0, 0, 0);
            acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(mm, t[12 + kk], acc[3], 0, 0, 0);
        } else {
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(t[kk], e1, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(t[4 + kk], e0, acc[1], 0, 0, 0);
            acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(t[8 + kk], pp, acc[2], 0, 0, 0);
            acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(t[12 + kk], mm, acc[3], 0, 0, 0);
        }
        if (kk & 1) __builtin_amdgcn_sched_barrier(0);   // bounds the reads in flight
    }
}

// 2-D transform of every z plane of a pair, Y = S_y X S_x (X[y][x], x
// contiguous), written in the plane's layout (the same kernel serves the
// forward and the inverse transform: S is its own inverse).  With `add`,
// the input is in + add on the points within 5 of a face (in elsewhere).  Grid
// (pairs, PG): workgroup y takes planes y, y + PG, ...  The LDS array
// holds X[y][x], then T transposed (T^T[c][y]; one level: c = 32 parity +
// i for the x mode 2 i + parity; two levels: c = 16 q + i for mode
// dst_mode2(q, i)), then Y[j][x].  Per axis, one level: wave w takes output
// block w % 2 of row (then column) blocks 2 (w / 2) and 2 (w / 2) + 1; two
// levels (odd length): wave w takes every mode of row (column) block w.
// Variants (the autotuner picks PG; SQ is chosen from the pairs): PG
// workgroups per pair; SQ: every plane the call transforms is square
// (nx = ny), so one operand set serves both axes (32 fewer registers, four
// workgroups per CU instead of three).
// FWD: the forward pass (pair layout in, padded planes out); else the
// inverse (padded in, pair layout out)
template <int PG, bool SQ, bool FWD>
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
    // odd lengths take the second-level fold (wave w: line block w, all
    // modes); even ones the first level alone (wave w: output block hb, line
    // blocks bp, bp + 1).  tx[0..7] / tx[8..15]: the first level's even and
    // odd operands, or the four second-level products' operands.
    const bool fx = nx & 1, fy = ny & 1;
    const int Nx = (nx + 1) >> 1, Ny = (ny + 1) >> 1;
    double tx[16];
    if (fx) dst_ops2(d.opt, nx, lane, tx);
    else dst_ops(d.opt, nx, hb, lane, tx, tx + 8);
    double tyb[SQ ? 1 : 16];
    if constexpr (!SQ) {
        if (fy) dst_ops2(d.opt, ny, lane, tyb);
        else dst_ops(d.opt, ny, hb, lane, tyb, tyb + 8);
    }
    const double* ty = SQ ? tx : tyb;
    const double* ex = tx;
    const double* ox = tx + 8;
    const double* ey = ty;
    const double* oy = ty + 8;
    // x mode of row c of the transposed intermediate
    auto xmode = [&](int c, int Nxk) { return fx ? dst_mode2(c >> 4, c & 15, Nxk) : 2 * (c & 31) + (c >> 5); };
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
    const double* in = d.in + (size_t)pid * (FWD ? d.stride : d.pstride);
    double* out = d.out + (size_t)pid * (FWD ? d.pstride : d.stride);
    const double* add = d.add ? d.add + (size_t)pid * d.stride : nullptr;
    // the face correction of plane zz at this thread's elements (0 elsewhere)
    auto load_add = [&](int zz, double ad[DP_PT]) {
        const size_t zo = (size_t)zz * npl;
        const bool zf = near_face(zz, nz);
        for_elems([&](int u, int e, int o) {
            const int yy = o / DP_LD, xx = o % DP_LD;
            ad[u] = (zf || near_face(xx, nx) || near_face(yy, ny)) ? add[zo + e] : 0.0;
        });
    };
    const int pin = dst_plane_pitch(npl, !FWD), pout = dst_plane_pitch(npl, FWD);
    for (int z = blockIdx.y; z < nz; z += PG) {
        // the plane's uniform bases; elements by 32-bit offsets from them
        const double* __restrict__ inz = in + (size_t)z * pin;
        double* __restrict__ outz = out + (size_t)z * pout;
        int gk = g, Nxk = Nx, Nyk = Ny;
        // recompute the fold addresses and the output modes per plane rather
        // than keep them all live
        asm volatile("" : "+v"(gk), "+s"(Nxk), "+s"(Nyk));
        double val[DP_PT];
#pragma unroll
        for (int u = 0; u < DP_PT; ++u) {
            const int e = threadIdx.x + u * DP_BS;
            val[u] = e < npl ? inz[e] : 0.0;
        }
        if (add) {   // the face correction, its loads in flight with the plane's
            double ad[DP_PT];
#pragma unroll
            for (int u = 0; u < DP_PT; ++u) ad[u] = 0.0;
            load_add(z, ad);
#pragma unroll
            for (int u = 0; u < DP_PT; ++u) val[u] += ad[u];
        }
        lds_sync();
        for_elems([&](int u, int, int o) { B[o] = val[u]; });
        lds_sync();
        // T = X S_x, written transposed (row c: an x mode, see xmode)
        if (fx) {   // rows y of block w, every x mode
            dst_f64x4 acc[4];
            dst_xform2<true>(B + (16 * w + r) * DP_LD, nx, gk, ex, acc);
            lds_sync();
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) B[(16 * q + r) * DP_LD + 16 * w + gk + 4 * v] = dst_val2(acc, q, v);
        } else {    // rows y of blocks bp, bp + 1; x modes of block hb
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
            lds_sync();
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int par = 0; par < 2; ++par)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        B[(32 * par + 16 * hb + r) * DP_LD + 16 * (bp + a) + g + 4 * v] = acc[a][par][v];
        }
        lds_sync();
        // Y = S_y T into B[y mode][x mode]
        if (fy) {   // rows c of block w, every y mode
            dst_f64x4 acc[4];
            dst_xform2<false>(B + (16 * w + r) * DP_LD, ny, gk, ey, acc);
            lds_sync();
            const int xm = xmode(16 * w + r, Nxk);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = dst_mode2(q, gk + 4 * v, Nyk);
                    if (j >= 0 && xm >= 0 && xm < nx) B[j * DP_LD + xm] = dst_val2(acc, q, v);
                }
        } else {    // rows c of blocks bp, bp + 1; y modes of block hb
            dst_f64x4 acc[2][2];
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
            lds_sync();
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int xm = xmode(16 * (bp + a) + r, Nxk);
#pragma unroll
                for (int par = 0; par < 2; ++par)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = 2 * (16 * hb + g + 4 * v) + par;
                        if (j < ny && xm >= 0 && xm < nx) B[j * DP_LD + xm] = acc[a][par][v];
                    }
            }
        }
        lds_sync();
        for_elems([&](int, int e, int o) { outz[e] = B[o]; });
    }
}

// Along z for each column (y, x): forward transform, division by the
// eigenvalue of the mode, inverse transform; same layout in and out.
// One-dimensional grid of PG workgroups per pair, a pair's workgroups
// adjacent: workgroup y of a pair takes 64-column tiles y, y + PG, ..., so
// that the workgroups running together read neighbouring 512-byte pieces of
// each z plane (a tile alone reads one piece per plane, 31 KB apart).  The
// LDS array holds the tile transposed (column-major: U[c][z]), so that the
// transform along z reads rows.
// Variants: PG workgroups per pair; LB: tile values loaded per batch into
// registers before they go to LDS (16: all at once, 8: two batches, fewer
// registers).  F2: the pairs with odd nz, by the second-level fold (the
// others return at once); else the pairs with even nz.
template <int PG, int LB, bool F2>
__global__ __launch_bounds__(DP_BS, 4) void k_dst_zline(DstArgs d) {
    __shared__ double U[DS_TC * DP_LD];
    __shared__ double lxy[DS_TC];   // x and y parts of the eigenvalue of each tile column
    const int pid = d.pair0 + (int)(blockIdx.x / PG), tg = (int)(blockIdx.x % PG);
    const sea_pair P = d.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    if (nx > DS_N || ny > DS_N || nz > DS_N) return;
    const int ncol = nx * ny;
    if (tg * DS_TC >= ncol || (d.skip && d.skip[pid]) || ((nz & 1) != 0) != F2) return;
    const int pin = dst_plane_pitch(ncol, d.in_pad), pout = dst_plane_pitch(ncol, d.out_pad);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int hb = w & 1, bp = 2 * (w >> 1);
    // F2: wave w takes the 16 columns of block w through both transforms and
    // the division with no barrier between them (no other wave touches those
    // LDS rows); else wave w takes z modes of block hb of column blocks bp,
    // bp + 1
    const int Nz = (nz + 1) >> 1;
    double tz[16];
    if constexpr (F2) dst_ops2(d.opt, nz, lane, tz);
    else dst_ops(d.opt, nz, hb, lane, tz, tz + 8);
    const double* ez = tz;
    const double* oz = tz + 8;
    const DevCell& Cl = d.cells[d.pair_cell[pid]];
    const double ihx = 1.0 / (Cl.h[0] * Cl.h[0]), ihy = 1.0 / (Cl.h[1] * Cl.h[1]), ihz = 1.0 / (Cl.h[2] * Cl.h[2]);
    const double* mux = d.mu + mu_off(nx);
    const double* muy = d.mu + mu_off(ny);
    const double lzj = lane < nz ? d.mu[mu_off(nz) + lane] * ihz : 0.0;   // z part for mode j = lane
    __shared__ double lzs[F2 ? DS_N : 1];   // the same by mode, for the second-level fold
    if (F2 && threadIdx.x < DS_N) lzs[threadIdx.x] = lzj;   // (read after the first tile's barrier)
    const double* in = d.in + (size_t)pid * (d.in_pad ? d.pstride : d.stride);
    double* out = d.out + (size_t)pid * (d.out_pad ? d.pstride : d.stride);
    // load element u of a thread: row a = threadIdx.x / 64 + 4 u, column threadIdx.x % 64
    const int lc = threadIdx.x % DS_TC, la = threadIdx.x / DS_TC;
    for (int c0 = tg * DS_TC; c0 < ncol; c0 += PG * DS_TC) {
        int gk = g, Nzk = Nz;
        // recompute the fold addresses and the output modes per tile rather
        // than keep them all live
        asm volatile("" : "+v"(gk), "+s"(Nzk));
        const bool cl = c0 + lc < ncol;
        static_assert(DP_PT % LB == 0, "load batches");
        // the first batch's loads are in flight while the workgroup finishes
        // the previous tile (the barrier), the others go straight to LDS
        // 32-bit element offsets walked per tile (not precomputed per load and
        // held across tiles)
        int off = la * pin + c0 + lc;
        asm volatile("" : "+v"(off));
#pragma unroll
        for (int u0 = 0; u0 < DP_PT; u0 += LB) {
            double val[LB];
#pragma unroll
            for (int u = 0; u < LB; ++u) {
                const int a = la + 4 * (u0 + u);
                val[u] = (cl && a < nz) ? in[off] : 0.0;
                off += 4 * pin;
            }
            if (u0 == 0) lds_sync();
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
        lds_sync();
        if constexpr (F2) {
            // forward, divided by the eigenvalue into the same row (mode j at
            // position j), inverse; the row is this lane's column
            double* row = U + (16 * w + r) * DP_LD;
            dst_f64x4 acc[4];
            dst_xform2<false>(row, nz, gk, ez, acc);
            const double lx = lxy[16 * w + r];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int j = dst_mode2(q, gk + 4 * v, Nzk);
                    if (j >= 0) row[j] = dst_val2(acc, q, v) / (lx + lzs[j]);
                }
            dst_xform2<false>(row, nz, gk, ez, acc);
            const int col = c0 + 16 * w + r;
            if (col < ncol) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int j = dst_mode2(q, gk + 4 * v, Nzk);
                        if (j >= 0) out[j * pout + col] = dst_val2(acc, q, v);   // 32-bit offsets (< 2^31)
                    }
            }
        } else {
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
            lds_sync();
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int par = 0; par < 2; ++par)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        U[(16 * (bp + a) + r) * DP_LD + 2 * (16 * hb + g + 4 * v) + par] = acc[a][par][v];
            lds_sync();
            // divide by the eigenvalue: wave w takes columns w + 4 u, lane the mode j
            if (lane < nz) {
#pragma unroll 2
                for (int u = 0; u < DS_TC / 4; ++u) {
                    const int cc = w + 4 * u;
                    if (c0 + cc < ncol) U[cc * DP_LD + lane] /= lxy[cc] + lzj;
                }
            }
            lds_sync();
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
                        if (j < nz) out[j * pout + col] = acc[a][par][v];   // 32-bit offsets (< 2^31)
                    }
            }
        }
    }
}

}  // namespace

size_t dst_table_doubles() { return (size_t)DS_N * (DS_OPN + DS_OPN2); }
size_t dst_mu_doubles() { return (size_t)mu_off(DS_N + 1); }

// Compiled variants of the two transform kernels, the autotuner's choices.
namespace {
using DstKernel = void (*)(DstArgs);
struct PlaneVariant {
    const char* name;
    DstKernel gen, sq, gen_inv, sq_inv;   // general planes / every plane square; forward, inverse
    int pg;
};
struct ZlineVariant {
    const char* name;
    DstKernel even, odd;   // pairs with even nz / odd nz
    int pg;
};
const PlaneVariant kPlaneVariants[] = {
    {"plane-pg16", k_dst_plane<16, false, true>, k_dst_plane<16, true, true>, k_dst_plane<16, false, false>,
     k_dst_plane<16, true, false>, 16},
    {"plane-pg8", k_dst_plane<8, false, true>, k_dst_plane<8, true, true>, k_dst_plane<8, false, false>,
     k_dst_plane<8, true, false>, 8},
    {"plane-pg32", k_dst_plane<32, false, true>, k_dst_plane<32, true, true>, k_dst_plane<32, false, false>,
     k_dst_plane<32, true, false>, 32},
};
const ZlineVariant kZlineVariants[] = {
    {"zline-pg16-lb16", k_dst_zline<16, 16, false>, k_dst_zline<16, 16, true>, 16},
    {"zline-pg16-lb8", k_dst_zline<16, 8, false>, k_dst_zline<16, 8, true>, 16},
    {"zline-pg32-lb16", k_dst_zline<32, 16, false>, k_dst_zline<32, 16, true>, 32},
    {"zline-pg8-lb16", k_dst_zline<8, 16, false>, k_dst_zline<8, 16, true>, 8},
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
    d.pstride = a.pstride;
    d.opt = tab;
    d.mu = mu;
    return d;
}
void launch_plane(const DstArgs& d, int n_pairs, int pv, int shape, hipStream_t s) {
    const PlaneVariant& V = kPlaneVariants[pv];
    const bool sq = (shape & DST_SQUARE) != 0;
    // the forward pass writes the padded planes, the inverse reads them
    const DstKernel k = d.out_pad ? (sq ? V.sq : V.gen) : (sq ? V.sq_inv : V.gen_inv);
    hipLaunchKernelGGL(k, dim3((unsigned)n_pairs, V.pg), dim3(DP_BS), 0, s, d);
}
void launch_zline(const DstArgs& d, int n_pairs, int zv, int shape, hipStream_t s) {
    const ZlineVariant& V = kZlineVariants[zv];
    // a launch's work-items (pairs x PG x DP_BS) stay below 2^32
    const int chunk = (int)(0xffffffffu / ((unsigned)V.pg * DP_BS));
    for (int p0 = 0; p0 < n_pairs; p0 += chunk) {
        DstArgs dc = d;
        dc.pair0 = p0;
        const int np = n_pairs - p0 < chunk ? n_pairs - p0 : chunk;
        if (shape & DST_ZODD) hipLaunchKernelGGL(V.odd, dim3((unsigned)np * V.pg), dim3(DP_BS), 0, s, dc);
        if (shape & DST_ZEVEN) hipLaunchKernelGGL(V.even, dim3((unsigned)np * V.pg), dim3(DP_BS), 0, s, dc);
    }
}
}  // namespace

hipError_t launch_dst_tables(double* tab, double* mu, hipStream_t s) {
    hipLaunchKernelGGL(k_dst_tables, dim3(DS_N), dim3(DS_BS), 0, s, tab, mu);
    return hipGetLastError();
}

// One transform pass of a variant on every pair (autotuner): pass 0 forward
// planes (in -> out, no face correction), 1 z lines, 2 inverse planes.
hipError_t launch_dst_pass(const ExxArgs& a, int pass, int variant, int shape, const double* in, double* out,
                           double* tab, double* mu, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    DstArgs d = dst_args(a, tab, mu);
    d.in = in;
    d.out = out;
    d.in_pad = pass != 0;   // the layouts of the spectral start's passes
    d.out_pad = pass != 2;
    if (pass == 1) launch_zline(d, a.n_pairs, variant, shape, s);
    else launch_plane(d, a.n_pairs, variant, shape, s);
    return hipGetLastError();
}

hipError_t launch_dst_solve(const ExxArgs& a, const double* r, double* z, double* tmp, double* tmp2, double* tab,
                            double* mu, int pv, int zv, int shape, const int* skip, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    if (pv < 0 || pv >= kNumPlane || zv < 0 || zv >= kNumZline) return hipErrorInvalidValue;
    DstArgs d = dst_args(a, tab, mu);
    d.skip = skip;
    d.in = r;
    d.out = tmp;
    d.out_pad = 1;
    launch_plane(d, a.n_pairs, pv, shape, s);
    d.in = tmp;
    d.out = tmp2;
    d.in_pad = 1;
    launch_zline(d, a.n_pairs, zv, shape, s);
    d.in = tmp2;
    d.out = z;
    d.out_pad = 0;
    launch_plane(d, a.n_pairs, pv, shape, s);
    return hipGetLastError();
}

// x = S^-1 ((S (b + fcorr)) ./ lambda) for every pair whose axes are all <=
// 64 (fcorr added on the face points; it lives in tmp, scratch of the pair
// arrays' size, which the z-line pass then overwrites); r is scratch of the
// same size.  The intermediate arrays have padded planes (whole 128-byte
// lines): the forward planes write r, the z lines r -> tmp, the inverse
// planes tmp -> x.  pv, zv: plane and z-line variants; shape: DST_* bits of the pairs the
// transform takes.
hipError_t launch_spectral_start(const ExxArgs& a, double* r, double* tmp, double* tab, double* mu, int pv, int zv,
                                 int shape, hipStream_t s, const std::function<void(int, bool)>& mark) {
    if (a.n_pairs <= 0) return hipSuccess;
    if (pv < 0 || pv >= kNumPlane || zv < 0 || zv >= kNumZline) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dst_tables, dim3(DS_N), dim3(DS_BS), 0, s, tab, mu);
    DstArgs d = dst_args(a, tab, mu);
    // planes forward: b + fcorr (in tmp) -> r; z lines forward, divided,
    // inverse: r -> tmp; planes inverse: tmp -> x
    d.in = a.b;
    d.add = tmp;
    d.out = r;
    d.out_pad = 1;
    mark(0, true);
    launch_plane(d, a.n_pairs, pv, shape, s);
    mark(0, false);
    d.add = nullptr;
    d.in = r;
    d.out = tmp;
    d.in_pad = 1;
    mark(1, true);
    launch_zline(d, a.n_pairs, zv, shape, s);
    mark(1, false);
    d.in = tmp;
    d.out = a.v;
    d.out_pad = 0;
    mark(2, true);
    launch_plane(d, a.n_pairs, pv, shape, s);
    mark(2, false);
    return hipGetLastError();
}
