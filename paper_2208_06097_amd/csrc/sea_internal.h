// Internal declarations shared by the HIP translation units of libsea.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "sea.h"

#define SEA_LMAX 6
#define SEA_NMOM 49        // (lmax+1)^2 real moments
#define SEA_NACC 52        // moments + s_abs + q + sum |rho| r^2
#define SEA_HALO 6         // stencil radius (half order of the O(h^12) Laplacian)

// Device-side per-pair record written by the solve kernels.
struct DevStat {
    int32_t iters;
    int32_t converged;   // 1 converged, 0 not, -1 nonfinite
    double rel_res;
    double e_ij;
    double s_abs;
    double q;
};
static_assert(sizeof(DevStat) == sizeof(sea_pair_stat), "stat layout");

struct sea_ctx {
    sea_opts opts;
    std::string err;
    int device = 0;
    int n_cu = 256;
    size_t max_lds = 65536;   // LDS bytes one workgroup may allocate
    // stage timing (opts.profile): begin/end events per stage
    hipEvent_t ev[SEA_STAGE_COUNT][2] = {};
    bool ev_used[SEA_STAGE_COUNT] = {};
    bool ev_ready = false;
    const void* nn_state = nullptr;   // attached network (learned start)
    int cg_tuned = -1;                // z-march variant chosen by sea_exx_autotune
    void* noalloc_scratch = nullptr;  // device address of this device's static scratch array
    // sine-transform kernel variants (spectral start): the autotuner's choice
    // and a fixed choice (-1: none; the fixed one wins)
    int dst_plane_tuned = -1, dst_zline_tuned = -1;
    int dst_plane_fixed = -1, dst_zline_fixed = -1;
    int scatter_tuned = -1, scatter_fixed = -1;
    // per-pair residual histories (caller's device buffer; nullptr: off)
    double* hist = nullptr;
    int hist_len = 0;
};

// Looks up, once per device, the device address of the static scratch array
// of the allocation-free entry point (sea_noalloc.hip); call with `dev`
// current.  nullptr if the lookup failed.
void* noalloc_scratch_setup(int dev);

// Records the begin/end event of a stage when profiling is on.
struct StageTimer {
    sea_ctx* ctx;
    int stage;
    hipStream_t s;
    StageTimer(sea_ctx* c, int st, hipStream_t str) : ctx(c), stage(st), s(str) {
        if (ctx->opts.profile && ctx->ev_ready) {
            (void)hipEventRecord(ctx->ev[stage][0], s);
            ctx->ev_used[stage] = true;
        }
    }
    ~StageTimer() {
        if (ctx->opts.profile && ctx->ev_ready) (void)hipEventRecord(ctx->ev[stage][1], s);
    }
};

// Byte layout of the exx workspace (offsets from the workspace base).
struct ExxLayout {
    size_t pairs, pair_cell, order, dbox, cells, partial, mom, b, v, bres, slots, stats, csr_off, csr_ent, scal, counter;
    size_t nnx, nny, nnact, dst_tmp, dst_tab, dst_mu, rnorm, racah_tab, mpoly, epart, cg_r, cg_p, cg_z, cg_part,
        cg_rho, cg_done, cg_active, total;
    int nmax;
    int ep_stride;        // pair-energy partial slots per pair (scatter)
    int n_chunks;
    int n_zchunks;
    int n_slots;
    size_t stride;        // doubles per pair-domain array (max interior size)
    size_t pstride;       // doubles per pair of the sine-transform intermediates (padded planes)
    size_t slot_stride;   // elements per CG slot array
};


// One cell of a (possibly batched) call: orbitals, grid, outputs, and the
// contiguous range of the global pair list that belongs to it.
struct DevCell {
    const void* phi;      // n_occ x Ng, double or float
    int phi_f32;
    int n_occ;
    int N[3];
    double h[3];
    double dV;
    size_t Ng;
    double* W;            // n_occ x Ng (nullptr: no scatter)
    double* exx;          // device scalar (nullable)
    int pair_begin, pair_end;
    int csr_base;         // offset of this cell's orbital lists in the CSR arrays
    int wbox_general;     // some W box is not its pair's domain, or is wider than the cell
};

// Arguments shared by the exx kernels (passed by value).
struct ExxArgs {
    const sea_pair* pairs;
    int n_pairs;
    const DevCell* cells; // device cell table
    const int* pair_cell; // cell index of every pair
    int n_cells;
    double* partial;      // n_pairs x n_zchunks x GC_N (Cartesian moments per plane chunk)
    int n_chunks;         // point chunks of GM_CHUNK (start-guess and network kernels)
    int n_zchunks;        // plane chunks of GC_ZC (moment gather)
    double* racah_tab;    // SEA_NMOM x 84 monomial coefficients of the Racah harmonics
    double* mpoly;        // n_pairs x 84: the multipole sum's monomial coefficients per pair
    double* mom;          // n_pairs x SEA_NACC (Racah moments, dV applied)
    double* b;            // n_pairs x stride
    double* fcorr;        // spectral start: -D x0 on the face points (the transform's scratch array)
    double* v;            // n_pairs x stride
    size_t stride;
    size_t pstride;       // per pair of the sine-transform intermediates (dst_plane_pitch planes)
    double* slots;        // n_slots x 3 x slot_stride elements (state precision)
    size_t slot_stride;   // elements per slot array (64 x 64 x max nz for the z-march)
    int n_slots;
    DevStat* stats;
    double rel_tol;
    double xc_beta_min;   // paired-update CG: smallest beta for recovering a pending step
    int max_iter;
    int lmax;
    int* queue_ctr;       // persistent-kernel pair counter (zeroed before the CG launch)
    const int* order;     // CG queue order: pair ids by decreasing domain size (nullable)
    const int* dbox;      // per pair 12 ints: boxes where W_i and W_j take the pair
    int x_nonzero;        // v holds a start guess on entry to the CG
    int start_res;        // FP32 z-march: bres already holds b - A x in FP64 (x kept as the FP64 start)
    double* rnorm;        // n_pairs x RZ_TILES x 2: |b|^2, |b - A x|^2 per row tile of the FP64 residual z-march (nullable)
    double* bres;         // n_pairs x stride: b - A x0 when x_nonzero
    int nmax;             // largest domain extent over pairs and axes
    double* epart;        // n_pairs x ep_stride pair-energy partials of the scatter (nullable: e_ij by k_cg_finish)
    int ep_stride;        // partial slots per pair
    // FP64 row-tile CG (one launch per sweep over all pairs)
    double* cg_r;         // n_pairs x stride: residual
    double* cg_p;         // 2 x n_pairs x stride: search direction, by iteration parity
    double* cg_part;      // n_pairs x RZ_TILES x 8 partial sums per row tile (k_cg.hip)
    double* cg_z;         // n_pairs x stride: preconditioned residual (nullable)
    int cg_pre;           // the CG is preconditioned by the sine transform (z = A_odd^-1 r)
    double* cg_rho;       // n_pairs x 2: |r|^2 of the last two iterations
    int* cg_done;         // n_pairs: the pair has stopped (2: by its start); null outside the row-tile CG
    int* cg_active;       // max_iter + 2 counters: pairs still iterating at each iteration; the last, after the init
    int cg_it;            // the iteration a sweep launch performs
    double* hist;         // n_pairs x (hist_len + 1) relative residuals per iteration (nullable)
    int hist_len;
};

// Scatter tiles (k_scatter.hip): 64 x 4 x 8 grid points of one orbital.
constexpr int SC_TX = 64, SC_TY = 4, SC_TZ = 8;
// longest orbital pair list whose pair energies the scatter forms
constexpr int SC_EP_MAXE = 128;

// Pair energies from the scatter.  The workgroup of orbital i of pair
// (i, j) writes one partial of e_ij per scatter tile the pair's domain
// meets.  It can when i's W box holds every domain point once: a box no
// wider than the cell (in the domain's unwrapped frame) that contains the
// domain.  D: lo[3], n[3] of the W box.
__host__ __device__ inline bool ep_takes(const sea_pair& P, const int* D, const int* N) {
    for (int a = 0; a < 3; ++a)
        if (D[3 + a] > N[a] || D[a] > P.lo[a] || P.lo[a] + P.n[a] > D[a] + D[3 + a]) return false;
    return true;
}
// Along an axis the tiles that n consecutive points (cyclically) meet form a
// run from the tile of the first point; its length is at most the number
// of tile boundaries inside the run plus one, plus one more for the cell's
// edge when the last tile is shorter than the others.
__host__ __device__ inline int ep_axis_slots(int n, int T, int tiles) {
    const int s = (T + n - 2) / T + 2;
    return s < tiles ? s : tiles;
}
__host__ __device__ inline int ep_slots(const sea_pair& P, const int* N) {
    const int T[3] = {SC_TX, SC_TY, SC_TZ};
    int s = 1;
    for (int a = 0; a < 3; ++a) s *= ep_axis_slots(P.n[a], T[a], (N[a] + T[a] - 1) / T[a]);
    return s;
}
// slot of tile tc (per-axis tile coordinates; `tiles` per axis) in pair P's run
__host__ __device__ inline int ep_slot(const sea_pair& P, const int* N, const int* tc, const int* tiles) {
    const int T[3] = {SC_TX, SC_TY, SC_TZ};
    int slot = 0;
    for (int a = 2; a >= 0; --a) {
        int w = P.lo[a] % N[a];
        w += w < 0 ? N[a] : 0;
        int r = tc[a] - w / T[a];
        r += r < 0 ? tiles[a] : 0;
        const int sa = ep_axis_slots(P.n[a], T[a], tiles[a]);
        if (r >= sa) return -1;
        slot = slot * sa + r;
    }
    return slot;
}

// (x, y, z) of a linear index over an nx x ny box (x fastest), advanced by a
// fixed stride with carries instead of integer divisions.
struct BoxWalk {
    int x, y, z, sx, sy, nx, ny;
    __device__ BoxWalk(int id, int stride, int nx_, int ny_) : nx(nx_), ny(ny_) {
        x = id % nx;
        const int r = id / nx;
        y = r % ny;
        z = r / ny;
        sx = stride % nx;
        sy = stride / nx;
    }
    __device__ __forceinline__ void next() {
        x += sx;
        y += sy;
        if (x >= nx) {
            x -= nx;
            ++y;
        }
        while (y >= ny) {
            y -= ny;
            ++z;
        }
    }
};

// m mod N for m a few cells away from [0, N), without a division
__device__ __forceinline__ int wrap_near(int m, int N) {
    while (m < 0) m += N;
    while (m >= N) m -= N;
    return m;
}

// Moment gather: planes per workgroup and doubles per chunk record.
constexpr int GC_ZC = 16;
constexpr int GC_N = 88;
constexpr int GC_TAB = SEA_NMOM * 84;

// Kernel launchers (k_exx.hip).  All enqueue on `s`.
int exx_n_chunks(long n_int_max);
hipError_t launch_gather_moments(const ExxArgs& a, hipStream_t s);
hipError_t launch_moments_final(const ExxArgs& a, double* Q_orth, hipStream_t s);
// The ghost values (Eq. 10) folded into b along x, then y, then z; with
// `face` (spectral start) also -D x0 into a.fcorr on the face points of the
// pairs the sine transform takes, x0 the multipole potential there.
hipError_t launch_boundary_fold(const ExxArgs& a, int nz_max, hipStream_t s, bool face = false);
hipError_t launch_cg(const ExxArgs& a, hipStream_t s);
hipError_t launch_me_guess(const ExxArgs& a, hipStream_t s);
// Spectral start: the whole multipole start into x for the pairs the sine
// transform skips (an axis beyond 64 points)
hipError_t launch_me_big(const ExxArgs& a, int nz_max, hipStream_t s);
constexpr double kPi = 3.14159265358979323846;
hipError_t launch_nn_sample(const ExxArgs& a, int D, float* out, double* s_out, int mode, hipStream_t s);
hipError_t launch_nn_apply(const ExxArgs& a, int D, const float* y32, hipStream_t s);
hipError_t launch_start_residual(const ExxArgs& a, hipStream_t s);
// b - A x in FP64 by z-march (cubic grids, nx, ny <= 64), in two launches:
// the norms |b|^2 and |b - A x|^2 per pair into a.rnorm (nothing else
// written), then (with `write`) b - A x into bres for the pairs whose start
// does not meet the FP32 z-march CG's exit test (the others are left alone).
constexpr int RZ_TILES = 4;   // row tiles of 16 rows per pair (row-tile march, k_cg.hip)
size_t residual_zm_lds_bytes();
hipError_t launch_residual_zm(const ExxArgs& a, hipStream_t s, bool write = true);
// FP64-state CG by row tiles (cubic grids, nx, ny <= 64): r = b - A x0 (or
// b with x = 0), p = r and the norms' partials; then per iteration a.cg_it
// sweep A (stop test; p = r + beta p; <p, A p>) and sweep B (x += alpha p,
// r -= alpha A p, |r|^2); after the last iteration the true residual's
// norms (launch_residual_zm) go into each pair's rel_res.
hipError_t launch_cg64_init(const ExxArgs& a, hipStream_t s);
hipError_t launch_cg64_sweep(const ExxArgs& a, int sweep, hipStream_t s);
hipError_t launch_cg64_exit(const ExxArgs& a, hipStream_t s);
// <r, z> partials of the preconditioned form (after z = A_odd^-1 r)
hipError_t launch_cg64_dot(const ExxArgs& a, hipStream_t s);
// z = A_odd^-1 r for the pairs not marked in `skip` (the three transform
// passes with the context's variants; tmp, tmp2 scratch of the pair arrays' size)
hipError_t launch_dst_solve(const ExxArgs& a, const double* r, double* z, double* tmp, double* tmp2, double* tab,
                            double* mu, int pv, int zv, int shape, const int* skip, hipStream_t s);
hipError_t launch_fill_int(int* p, size_t n, hipStream_t s);
// p[0 .. n) = NaN (the residual histories' empty entries)
hipError_t launch_fill_nan(double* p, size_t n, hipStream_t s);
// Shape bits of the pairs the sine transform takes: every one has nx = ny;
// some has an odd nz; some has an even nz (the z-line kernels of each kind
// launched only when needed).
enum { DST_SQUARE = 1, DST_ZODD = 2, DST_ZEVEN = 4 };
// Plane pitch (doubles) of the sine-transform passes' intermediate arrays:
// each z plane of nx*ny points padded to whole 128-byte lines (pad = 1), or
// the pair layout itself (pad = 0).  The intermediates' per-pair stride
// (pstride) leaves room for nz padded planes.
__host__ __device__ inline int dst_plane_pitch(int npl, int pad) { return pad ? (npl + 15) & ~15 : npl; }
// Spectral start (k_dst.hip): x = A_odd^-1 (b + a.fcorr on the face points)
// for the pairs with every axis <= 64 (a.fcorr is tmp, scratch of the pair
// arrays' size; r scratch of the same size).
size_t dst_table_doubles();
size_t dst_mu_doubles();
// pv, zv: variants of the plane and z-line kernels (0 <= pv <
// dst_plane_variant_count(), 0 <= zv < dst_variant_count() - that); shape:
// DST_* bits of the pairs the transform takes.  `mark(pass, true)` /
// `mark(pass, false)` bracket each of the three transform passes (0 forward
// planes, 1 z lines, 2 inverse planes; stage timing).
hipError_t launch_spectral_start(const ExxArgs& a, double* r, double* tmp, double* tab, double* mu, int pv, int zv,
                                 int shape, hipStream_t s, const std::function<void(int, bool)>& mark);
// transform-kernel variants: plane variants first, then the z-line ones
int dst_variant_count();
int dst_plane_variant_count();
const char* dst_variant_name(int v);
hipError_t launch_dst_tables(double* tab, double* mu, hipStream_t s);
// one pass (0 forward planes, 1 z lines, 2 inverse planes) of a variant on
// every pair, in -> out (autotuner)
hipError_t launch_dst_pass(const ExxArgs& a, int pass, int variant, int shape, const double* in, double* out,
                           double* tab, double* mu, hipStream_t s);
// the pairs the sine transform takes
__host__ __device__ inline bool spectral_pair(const sea_pair& P) { return P.n[0] <= 64 && P.n[1] <= 64 && P.n[2] <= 64; }
// points next to a face that the difference of the zero and the odd
// continuations of the stencil reaches (index i of an axis of n points)
constexpr int FF_W = 5;
__host__ __device__ inline bool near_face(int i, int n) { return i < FF_W || i >= n - FF_W; }
// LDS-only barrier: waits for this thread's LDS traffic, not for global loads
// or stores in flight (which __syncthreads, a workgroup-scope fence, waits
// for), then synchronizes the workgroup.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }
// z-marching CG (k_cg.hip): needs every pair with n[0], n[1] <= 64.
bool cg_zm_fits(const sea_pair* pairs, int n_pairs, const double* h);
size_t cg_zm_lds_bytes(int state_f32);
hipError_t launch_eps_marginals(const void* phi, int f32, const int* N, int n_occ, int nmax, double* m,
                                hipStream_t s);
hipError_t launch_eps_overlap(const void* phi, int f32, const int* N, double dV, const sea_pair* pairs, int n_pairs,
                              double* S, hipStream_t s);
int cg_variant_count();
const char* cg_variant_name(int v);
hipError_t launch_cg_zm(const ExxArgs& a, int variant, hipStream_t s);
hipError_t launch_cg_finish(const ExxArgs& a, hipStream_t s);
// the scatter's compiled schedules (workgroup orders), the autotuner's choices
int scatter_variant_count();
const char* scatter_variant_name(int v);
hipError_t launch_scatter(const ExxArgs& a, const DevCell& cell, const int* csr_off, const int2* csr_ent, int variant,
                          hipStream_t s);
// zeroes a.epart (every slot the scatter does not write must read zero)
hipError_t launch_epart_clear(const ExxArgs& a, hipStream_t s);
hipError_t launch_energy_sum(const ExxArgs& a, double* out_scalars, double* e_dev, hipStream_t s);

// Host evaluation of the solid-harmonic recurrence (orthonormal real form).
void solid_harmonics_orthonormal_host(int lmax, double x, double y, double z, double* out);

// ACE launchers (k_ace.hip).
struct AceWs;
