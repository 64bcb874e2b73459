// Owner-computes scatter of the exx action for gfx950 (Eq. 13-14): W_o(g)
// is the sum over the pairs of orbital o, in pair order, of v_ij(g) times
// the other orbital, with v_ij the pair potential inside the pair's domain
// and its multipole expansion (Eq. 10) outside it; no atomics, so W is
// bitwise reproducible.  On the way it forms the pair energies of Eq. 8:
// the workgroup of orbital i = min(i, j) multiplies each contribution
// v_ij phi_j at a domain point by phi_i there and sums them per (pair,
// tile), so e_ij = dV sum rho_ij v_ij needs one more orbital load per tile
// point instead of a pass of its own over every pair domain.
#include <algorithm>
#include <type_traits>

#include "exx_device.h"
#include "sea_internal.h"

namespace {

// owner-computes scatter: W_o(g) = sum over o's pairs (pair order) of
//    v_pair(g - lo) phi_other(g), every domain duplicate of g included.

constexpr int SC_BS = 256;
constexpr int SC_MAXE = 128;   // list entries per chunk
constexpr int SC_NM = 84;      // monomial coefficients of a pair's multipole sum

// (orbital, tile) of this workgroup, by the order of the workgroups (the
// schedule; the autotuner's variants).  0: the tiles of one orbital in
// turn; 1: the orbitals of one tile in turn; 2: as 1 within each XCD
// (workgroup k runs on XCD k mod 8), which owns every eighth tile, so that
// the owners of a tile share that XCD's L2 for the partner orbitals and pair
// potentials they read there.  Measured on the 64-molecule cell: 4.80, 6.22
// and 4.56 ms per launch; 0 and 2 are compiled.
constexpr int SC_XCD = 8;

template <int ORDER>
__device__ __forceinline__ void sc_block(int n_tiles, int n_occ, int& o, int& t) {
    const int k = blockIdx.x;
    if constexpr (ORDER == 0) {
        t = k % n_tiles;
        o = k / n_tiles;
    } else if constexpr (ORDER == 1) {
        o = k % n_occ;
        t = k / n_occ;
    } else {
        const int x = k % SC_XCD, m = k / SC_XCD;
        o = m % n_occ;
        t = (m / n_occ) * SC_XCD + x;
    }
}
__host__ inline long sc_grid(int order, int n_tiles, int n_occ) {
    return order == 2 ? (long)((n_tiles + SC_XCD - 1) / SC_XCD) * SC_XCD * n_occ : (long)n_tiles * n_occ;
}

__device__ __forceinline__ bool axis_hits(int t0, int T, int lo, int n, int N) {
    if (n >= N) return true;
    const int s = wrap_idx(t0 - lo, N);
    return s < n || s + T > N;
}

// W gathered per (orbital, tile): every pair of the orbital whose W box
// touches the tile adds v * phi_partner at the tile's points, in pair order.
// The box is the pair's W box for this orbital's side (lo[3], n[3] in the
// pair domain's unwrapped frame); inside the pair's domain v is the solution,
// outside it the multipole potential of the pair (Eq. 10).
// The cell's record comes by value, so its pointers are kernel arguments:
// uniform, and known to the compiler to address global memory.
// GENERAL: some W box reaches beyond its pair's domain (multipole values
// there) or is wider than the cell (points met several times); without it
// every W box is its pair's domain, and the kernel carries neither path (nor
// their registers).  PT: the orbitals' precision.
template <bool GENERAL, typename PT, int ORDER>
__global__ __launch_bounds__(SC_BS) void k_scatter(ExxArgs a, const DevCell C, const int* __restrict__ off_all,
                                                   const int2* __restrict__ ent) {
    __shared__ int list[SC_MAXE];
    // per listed entry: pair, partner orbital, W box (lo, n), domain (lo, n),
    // wide flag, energy slot (-1: this workgroup adds nothing to e_ij)
    __shared__ int meta[SC_MAXE][16];
    // per entry of the orbital's list: the wavefronts' parts of its energy
    // partial, its slot and pair (the list has at most SC_EP_MAXE entries
    // when a.epart is set)
    __shared__ double ep_w[SC_EP_MAXE][SC_BS / 64];
    __shared__ int ep_slot_of[SC_EP_MAXE], ep_pid_of[SC_EP_MAXE];
    // this orbital at the tile's points (energy partials)
    __shared__ double po_s[SC_TZ][SC_BS];
    __shared__ int cnt, wide, n_e;
    const int* off = off_all + C.csr_base;
    double* __restrict__ W = C.W;
    const int tiles_x = (C.N[0] + SC_TX - 1) / SC_TX;
    const int tiles_y = (C.N[1] + SC_TY - 1) / SC_TY;
    const int n_tiles = tiles_x * tiles_y * ((C.N[2] + SC_TZ - 1) / SC_TZ);
    int o, t;
    sc_block<ORDER>(n_tiles, C.n_occ, o, t);
    if (t >= n_tiles) return;
    const int tx0 = (t % tiles_x) * SC_TX;
    const int ty0 = ((t / tiles_x) % tiles_y) * SC_TY;
    const int tz0 = (t / (tiles_x * tiles_y)) * SC_TZ;
    const int tiles[3] = {tiles_x, tiles_y, (C.N[2] + SC_TZ - 1) / SC_TZ};
    const int tc[3] = {t % tiles_x, (t / tiles_x) % tiles_y, t / (tiles_x * tiles_y)};
    const int e0 = off[o], e1 = off[o + 1];
    // energy partials only for lists that fit the per-entry LDS arrays (the
    // host leaves a.epart unset otherwise)
    const bool take_e = a.epart && e1 - e0 <= SC_EP_MAXE;
    if (threadIdx.x == 0) cnt = 0;
    if (take_e)
        for (int q = threadIdx.x; q < e1 - e0; q += SC_BS) ep_slot_of[q] = -1;
    __syncthreads();
    double acc[SC_TX * SC_TY * SC_TZ / SC_BS];
#pragma unroll
    for (int k = 0; k < SC_TX * SC_TY * SC_TZ / SC_BS; ++k) acc[k] = 0.0;
    for (int c0 = e0; c0 < e1; c0 += SC_MAXE) {
        const int c1 = min(e1, c0 + SC_MAXE);
        // ordered compaction by wavefront 0: lane k tests entry c0 + 64 s + k,
        // hits keep their order through the ballot's prefix counts
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            int m = 0, nw = 0, ne = 0;
            for (int b0 = c0; b0 < c1; b0 += 64) {
                const int e = b0 + lane;
                bool hit = false, wd = false;
                int slot = -1;
                if (e < c1) {
                    const int pid = ent[e].x;
                    const sea_pair P = a.pairs[pid];
                    const bool iside = o == P.i;
                    const int* D = a.dbox + 12 * (size_t)pid + (iside ? 0 : 6);
                    hit = axis_hits(tx0, SC_TX, D[0], D[3], C.N[0]) && axis_hits(ty0, SC_TY, D[1], D[4], C.N[1]) &&
                          axis_hits(tz0, SC_TZ, D[2], D[5], C.N[2]);
                    wd = GENERAL && hit && (D[3] > C.N[0] || D[4] > C.N[1] || D[5] > C.N[2]);
                    // the pair's energy partial of this tile: i side, a W box
                    // that holds the domain once, a tile the domain meets
                    if (hit && iside && take_e && ep_takes(P, D, C.N) &&
                        axis_hits(tx0, SC_TX, P.lo[0], P.n[0], C.N[0]) &&
                        axis_hits(ty0, SC_TY, P.lo[1], P.n[1], C.N[1]) &&
                        axis_hits(tz0, SC_TZ, P.lo[2], P.n[2], C.N[2]))
                        slot = ep_slot(P, C.N, tc, tiles);
                }
                const unsigned long long mask = __ballot(hit);
                const unsigned long long below = lane ? (mask << (64 - lane)) : 0ull;
                if (hit) {
                    const int q = m + __popcll(below);
                    const int2 en = ent[e];
                    const sea_pair P = a.pairs[en.x];
                    const int* D = a.dbox + 12 * (size_t)en.x + (o == P.i ? 0 : 6);
                    list[q] = e;
                    meta[q][0] = en.x;
                    meta[q][1] = en.y;
#pragma unroll
                    for (int d = 0; d < 6; ++d) meta[q][2 + d] = D[d];
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        meta[q][8 + d] = P.lo[d];
                        meta[q][11 + d] = P.n[d];
                    }
                    meta[q][14] = wd;
                    meta[q][15] = slot;
                    if (slot >= 0) {
                        ep_slot_of[e - e0] = slot;
                        ep_pid_of[e - e0] = en.x;
                    }
                }
                m += __popcll(mask);
                nw += __popcll(__ballot(wd));
                ne += __popcll(__ballot(slot >= 0));
            }
            if (lane == 0) {
                cnt = m;
                wide = nw;
                n_e = ne;
            }
        }
        __syncthreads();
        const int m = cnt;
        // fast path: this thread's column (gx, gy) and planes tz0 + k; a box no
        // wider than the cell holds each grid point at most once, found from
        // per-pair offsets by compare-and-subtract instead of modulo
        static_assert(SC_TX * SC_TY == SC_BS, "one (x, y) column per thread");
        const int cx = threadIdx.x % SC_TX, cy = threadIdx.x / SC_TX;
        const int gx = tx0 + cx, gy = ty0 + cy;
        const bool colin = gx < C.N[0] && gy < C.N[1];
        {
            const PT* __restrict__ ph = (const PT*)C.phi;
            // this orbital at the column's points (in LDS), for the energy partials
            if (n_e) {
                const size_t gcol = (size_t)o * C.Ng + (size_t)gy * C.N[0] + gx;
                const size_t gplane = (size_t)C.N[0] * C.N[1];
#pragma unroll
                for (int k = 0; k < SC_TZ; ++k)
                    po_s[k][threadIdx.x] = colin ? (double)ph[gcol + (size_t)min(tz0 + k, C.N[2] - 1) * gplane] : 0.0;
            }
            for (int q = 0; q < m; ++q) {
                // the entry's values are the same in every lane: read them into
                // scalar registers, so the per-plane addresses below are a scalar
                // base plus one per-lane offset shared by all planes
                int e[14];
#pragma unroll
                for (int d = 0; d < 14; ++d) e[d] = __builtin_amdgcn_readfirstlane(meta[q][d]);
                if (GENERAL && __builtin_amdgcn_readfirstlane(meta[q][14])) continue;   // general path below
                const int eslot = __builtin_amdgcn_readfirstlane(meta[q][15]);
                const int pid = e[0], oth = e[1];
                const int* D = &e[2];
                const int* plo = &e[8];
                const int* pn = &e[11];
                // box coordinates of the tile corner (uniform), then of this column:
                // gx < N keeps lx below 2N, so one subtraction wraps it
                int lx = wrap_idx(tx0 - D[0], C.N[0]) + cx;
                int ly = wrap_idx(ty0 - D[1], C.N[1]) + cy;
                lx -= (lx >= C.N[0]) ? C.N[0] : 0;
                ly -= (ly >= C.N[1]) ? C.N[1] : 0;
                double ep = 0.0;
                if (colin && lx < D[3] && ly < D[4]) {
                    const int lz0 = wrap_idx(tz0 - D[2], C.N[2]);
                    const int sx = D[0] + lx - plo[0], sy = D[1] + ly - plo[1];
                    const bool in_xy = sx >= 0 && sx < pn[0] && sy >= 0 && sy < pn[1];
                    const double* v = a.v + (size_t)pid * a.stride;
                    const unsigned vcol = in_xy ? (unsigned)(sy * pn[0] + sx) : 0u;
                    const size_t vplane = (size_t)pn[0] * pn[1], gplane = (size_t)C.N[0] * C.N[1];
                    const unsigned gcol = (unsigned)(gy * C.N[0] + gx);
                    const size_t phoff = (size_t)oth * C.Ng;
                    // all loads of the column's points first (independent, in flight
                    // together), then the multipole values of points outside the domain
                    double vv[SC_TZ];
                    PT pv[SC_TZ];   // converted at the product: no wait inside the load sequence
                    int lzs[SC_TZ];
                    bool me[SC_TZ], ins[SC_TZ];
#pragma unroll
                    for (int k = 0; k < SC_TZ; ++k) {
                        const int gz = tz0 + k;
                        int lz = lz0 + k;
                        lz -= (lz >= C.N[2]) ? C.N[2] : 0;
                        lzs[k] = lz;
                        const bool valid = gz < C.N[2] && lz < D[5];
                        const int sz = D[2] + lz - plo[2];
                        const bool zin = valid && sz >= 0 && sz < pn[2];
                        const bool inside = zin && in_xy;
                        ins[k] = inside;
                        me[k] = GENERAL && valid && !inside;
                        if constexpr (std::is_same<PT, float>::value) {
                            // unconditional (a clamped plane is in bounds), so the
                            // widening is not pulled into a branch with its own wait
                            const size_t go = phoff + (size_t)min(gz, C.N[2] - 1) * gplane;
                            pv[k] = ph[go + gcol];
                            pv[k] = valid ? pv[k] : 0.0f;
                        } else {
                            const size_t go = phoff + (size_t)(valid ? gz : 0) * gplane;
                            pv[k] = valid ? ph[go + gcol] : 0.0;
                        }
                        const double* vz = v + (size_t)(zin ? sz : 0) * vplane;
                        vv[k] = inside ? vz[vcol] : 0.0;
                    }
                    bool any_me = false;
#pragma unroll
                    for (int k = 0; k < SC_TZ; ++k) any_me |= me[k];
                    if (GENERAL && any_me) {   // the multipole value outside the domain (W boxes beyond it)
                        const double* cf = a.mpoly + (size_t)pid * SC_NM;
                        const double* org = a.pairs[pid].origin;
#pragma unroll
                        for (int k = 0; k < SC_TZ; ++k)
                            if (me[k])
                                vv[k] = me_inverted_potential(cf, (D[0] + lx) * C.h[0] - org[0],
                                                               (D[1] + ly) * C.h[1] - org[1],
                                                               (D[2] + lzs[k]) * C.h[2] - org[2]);
                    }
#pragma unroll
                    for (int k = 0; k < SC_TZ; ++k) {
                        const double c = vv[k] * (double)pv[k];
                        acc[k] += c;
                        if (ins[k]) ep += po_s[k][threadIdx.x] * c;
                    }
                }
                if (eslot >= 0) {   // uniform: every lane of the workgroup is here
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) ep += __shfl_xor(ep, off, 64);
                    if ((threadIdx.x & 63) == 0) ep_w[list[q] - e0][threadIdx.x >> 6] = ep;
                }
            }
        }
        // general path: boxes wider than the cell (a grid point met several times)
        if (GENERAL && wide)
#pragma unroll
        for (int k = 0; k < SC_TX * SC_TY * SC_TZ / SC_BS; ++k) {
            const int lid = threadIdx.x + k * SC_BS;
            const int gx = tx0 + lid % SC_TX, gy = ty0 + (lid / SC_TX) % SC_TY, gz = tz0 + lid / (SC_TX * SC_TY);
            if (gx >= C.N[0] || gy >= C.N[1] || gz >= C.N[2]) continue;
            const size_t g = ((size_t)gz * C.N[1] + gy) * C.N[0] + gx;
            double s = acc[k];
            for (int q = 0; q < m; ++q) {
                const int2 en = ent[list[q]];
                const sea_pair P = a.pairs[en.x];
                const int* D = a.dbox + 12 * (size_t)en.x + (o == P.i ? 0 : 6);
                if (!(D[3] > C.N[0] || D[4] > C.N[1] || D[5] > C.N[2])) continue;   // fast path above
                const double* v = a.v + (size_t)en.x * a.stride;
                const double* cf = a.mpoly + (size_t)en.x * SC_NM;
                const double ph = load_phi(C.phi, C.phi_f32, (size_t)en.y * C.Ng + g);
                for (int lz = wrap_idx(gz - D[2], C.N[2]); lz < D[5]; lz += C.N[2])
                    for (int ly = wrap_idx(gy - D[1], C.N[1]); ly < D[4]; ly += C.N[1])
                        for (int lx = wrap_idx(gx - D[0], C.N[0]); lx < D[3]; lx += C.N[0]) {
                            const int px = D[0] + lx, py = D[1] + ly, pz = D[2] + lz;  // unwrapped point
                            const int sx = px - P.lo[0], sy = py - P.lo[1], sz = pz - P.lo[2];
                            double val;
                            if (sx >= 0 && sx < P.n[0] && sy >= 0 && sy < P.n[1] && sz >= 0 && sz < P.n[2])
                                val = v[((size_t)sz * P.n[1] + sy) * P.n[0] + sx];
                            else
                                val = me_inverted_potential(cf, px * C.h[0] - P.origin[0],
                                                             py * C.h[1] - P.origin[1], pz * C.h[2] - P.origin[2]);
                            s += val * ph;
                        }
            }
            acc[k] = s;
        }
        __syncthreads();
    }
    // the energy partials: the wavefronts' parts of each entry summed in a
    // fixed order
    if (take_e)
    for (int q = threadIdx.x; q < e1 - e0; q += SC_BS) {
        if (ep_slot_of[q] >= 0) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < SC_BS / 64; ++w) t += ep_w[q][w];
            a.epart[(size_t)ep_pid_of[q] * a.ep_stride + ep_slot_of[q]] = t;
        }
    }
#pragma unroll
    for (int k = 0; k < SC_TX * SC_TY * SC_TZ / SC_BS; ++k) {
        const int lid = threadIdx.x + k * SC_BS;
        const int gx = tx0 + lid % SC_TX, gy = ty0 + (lid / SC_TX) % SC_TY, gz = tz0 + lid / (SC_TX * SC_TY);
        if (gx >= C.N[0] || gy >= C.N[1] || gz >= C.N[2]) continue;
        W[(size_t)o * C.Ng + ((size_t)gz * C.N[1] + gy) * C.N[0] + gx] = acc[k];
    }
}

__global__ __launch_bounds__(256) void k_epart_clear(double* __restrict__ p, size_t n) {
    for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) p[k] = 0.0;
}

}  // namespace

hipError_t launch_epart_clear(const ExxArgs& a, hipStream_t s) {
    const size_t n = (size_t)a.n_pairs * a.ep_stride;
    if (!a.epart || n == 0) return hipSuccess;
    const unsigned nb = (unsigned)std::min<size_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_epart_clear, dim3(nb), dim3(256), 0, s, a.epart, n);
    return hipGetLastError();
}

namespace {
using ScatterKernel = void (*)(ExxArgs, const DevCell, const int*, const int2*);
struct ScatterVariant {
    const char* name;
    int order;
    ScatterKernel k[2][2];   // [general W boxes][FP32 orbitals]
};
template <int ORDER>
ScatterVariant scatter_variant(const char* name) {
    return {name,
            ORDER,
            {{k_scatter<false, double, ORDER>, k_scatter<false, float, ORDER>},
             {k_scatter<true, double, ORDER>, k_scatter<true, float, ORDER>}}};
}
const ScatterVariant kScatterVariants[] = {
    scatter_variant<2>("scatter-xcd-owners"),
    scatter_variant<0>("scatter-orbital-tiles"),
};
constexpr int kNumScatter = sizeof(kScatterVariants) / sizeof(kScatterVariants[0]);
}  // namespace

int scatter_variant_count() { return kNumScatter; }
const char* scatter_variant_name(int v) { return v >= 0 && v < kNumScatter ? kScatterVariants[v].name : nullptr; }

hipError_t launch_scatter(const ExxArgs& a, const DevCell& cell, const int* csr_off, const int2* csr_ent, int variant,
                          hipStream_t s) {
    if (variant < 0 || variant >= kNumScatter) return hipErrorInvalidValue;
    const ScatterVariant& V = kScatterVariants[variant];
    const int* N = cell.N;
    const int tiles = ((N[0] + SC_TX - 1) / SC_TX) * ((N[1] + SC_TY - 1) / SC_TY) * ((N[2] + SC_TZ - 1) / SC_TZ);
    const long nb = sc_grid(V.order, tiles, cell.n_occ);
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(V.k[cell.wbox_general ? 1 : 0][cell.phi_f32 ? 1 : 0], dim3((unsigned)nb), dim3(SC_BS), 0, s, a,
                       cell, csr_off, csr_ent);
    return hipGetLastError();
}

