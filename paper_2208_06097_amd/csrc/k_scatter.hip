// Owner-computes scatter of the exx action for gfx950 (Eq. 15): W_o(g) is
// the sum over the pairs of orbital o, in pair order, of v_ij(g) times the
// other orbital, with v_ij the pair potential inside the pair's domain and
// its multipole expansion (Eq. 10) outside it; no atomics, so W is bitwise
// reproducible.
#include <type_traits>

#include "exx_device.h"
#include "sea_internal.h"

namespace {

// owner-computes scatter: W_o(g) = sum over o's pairs (pair order) of
//    v_pair(g - lo) phi_other(g), every domain duplicate of g included.

constexpr int SC_BS = 256;
constexpr int SC_TX = 64, SC_TY = 4, SC_TZ = 8;
constexpr int SC_MAXE = 128;   // list entries per chunk
constexpr int SC_NM = 84;      // monomial coefficients of a pair's multipole sum

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
__global__ __launch_bounds__(SC_BS) void k_scatter(ExxArgs a, const DevCell C, const int* __restrict__ off_all,
                                                   const int2* __restrict__ ent) {
    __shared__ int list[SC_MAXE];
    // per listed entry: pair, partner orbital, W box (lo, n), domain (lo, n), wide flag
    __shared__ int meta[SC_MAXE][16];
    __shared__ int cnt, wide;
    const int* off = off_all + C.csr_base;
    double* __restrict__ W = C.W;
    const int o = blockIdx.y;
    const int tiles_x = (C.N[0] + SC_TX - 1) / SC_TX;
    const int tiles_y = (C.N[1] + SC_TY - 1) / SC_TY;
    const int t = blockIdx.x;
    const int tx0 = (t % tiles_x) * SC_TX;
    const int ty0 = ((t / tiles_x) % tiles_y) * SC_TY;
    const int tz0 = (t / (tiles_x * tiles_y)) * SC_TZ;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const int e0 = off[o], e1 = off[o + 1];
    double acc[SC_TX * SC_TY * SC_TZ / SC_BS];
#pragma unroll
    for (int k = 0; k < SC_TX * SC_TY * SC_TZ / SC_BS; ++k) acc[k] = 0.0;
    for (int c0 = e0; c0 < e1; c0 += SC_MAXE) {
        const int c1 = min(e1, c0 + SC_MAXE);
        // ordered compaction by wavefront 0: lane k tests entry c0 + 64 s + k,
        // hits keep their order through the ballot's prefix counts
        if (threadIdx.x < 64) {
            const int lane = threadIdx.x;
            int m = 0, nw = 0;
            for (int b0 = c0; b0 < c1; b0 += 64) {
                const int e = b0 + lane;
                bool hit = false, wd = false;
                if (e < c1) {
                    const int pid = ent[e].x;
                    const int* D = a.dbox + 12 * (size_t)pid + (o == a.pairs[pid].i ? 0 : 6);
                    hit = axis_hits(tx0, SC_TX, D[0], D[3], C.N[0]) && axis_hits(ty0, SC_TY, D[1], D[4], C.N[1]) &&
                          axis_hits(tz0, SC_TZ, D[2], D[5], C.N[2]);
                    wd = hit && (D[3] > C.N[0] || D[4] > C.N[1] || D[5] > C.N[2]);
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
                }
                m += __popcll(mask);
                nw += __popcll(__ballot(wd));
            }
            if (lane == 0) {
                cnt = m;
                wide = nw;
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
        // one copy of the loop per orbital precision: no per-point branch on it
        auto fast_entries = [&](auto f32) {
            using PT = typename std::conditional<decltype(f32)::value, float, double>::type;
            const PT* __restrict__ ph = (const PT*)C.phi;
            for (int q = 0; q < m; ++q) {
                // the entry's values are the same in every lane: read them into
                // scalar registers, so the per-plane addresses below are a scalar
                // base plus one per-lane offset shared by all planes
                int e[14];
#pragma unroll
                for (int d = 0; d < 14; ++d) e[d] = __builtin_amdgcn_readfirstlane(meta[q][d]);
                if (__builtin_amdgcn_readfirstlane(meta[q][14])) continue;   // general path below
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
                if (!colin || lx >= D[3] || ly >= D[4]) continue;
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
                bool me[SC_TZ];
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
                    me[k] = valid && !inside;
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
                if (any_me) {   // the multipole value outside the domain (W boxes beyond it)
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
                for (int k = 0; k < SC_TZ; ++k) acc[k] += vv[k] * (double)pv[k];
            }
        };
        if (C.phi_f32) fast_entries(std::true_type());
        else fast_entries(std::false_type());
        // general path: boxes wider than the cell (a grid point met several times)
        if (wide)
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
#pragma unroll
    for (int k = 0; k < SC_TX * SC_TY * SC_TZ / SC_BS; ++k) {
        const int lid = threadIdx.x + k * SC_BS;
        const int gx = tx0 + lid % SC_TX, gy = ty0 + (lid / SC_TX) % SC_TY, gz = tz0 + lid / (SC_TX * SC_TY);
        if (gx >= C.N[0] || gy >= C.N[1] || gz >= C.N[2]) continue;
        W[(size_t)o * C.Ng + ((size_t)gz * C.N[1] + gy) * C.N[0] + gx] = acc[k];
    }
}

}  // namespace

hipError_t launch_scatter(const ExxArgs& a, const DevCell& cell, const int* csr_off, const int2* csr_ent, hipStream_t s) {
    const int* N = cell.N;
    const int tiles = ((N[0] + SC_TX - 1) / SC_TX) * ((N[1] + SC_TY - 1) / SC_TY) * ((N[2] + SC_TZ - 1) / SC_TZ);
    dim3 grid(tiles, cell.n_occ);
    hipLaunchKernelGGL(k_scatter, grid, dim3(SC_BS), 0, s, a, cell, csr_off, csr_ent);
    return hipGetLastError();
}

