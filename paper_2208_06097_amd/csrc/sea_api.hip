// C ABI of libsea: argument validation, workspace layout, orchestration of
// the exx kernels on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "nn_internal.h"
#include "host_geometry.h"
#include "sea_internal.h"

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

sea_status fail(sea_ctx* ctx, sea_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
sea_status fail(sea_ctx* ctx, sea_status st, const char* fmt, ...) {
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return st;
}

#define SEA_HIP_CHECK(ctx, expr)                                                                 \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, SEA_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)


sea_status check_opts(sea_ctx* ctx, const sea_opts* o) {
    if (!o) return fail(ctx, SEA_E_ARG, "opts is NULL");
    if (o->fd_half_order != 6) return fail(ctx, SEA_E_ARG, "fd_half_order must be 6 (O(h^12) Laplacian)");
    if (o->lmax < 0 || o->lmax > SEA_LMAX) return fail(ctx, SEA_E_ARG, "lmax must be in 0..%d", SEA_LMAX);
    if (!(o->rel_tol > 0.0) || !std::isfinite(o->rel_tol)) return fail(ctx, SEA_E_ARG, "rel_tol must be > 0");
    if (o->max_iter < 0) return fail(ctx, SEA_E_ARG, "max_iter must be >= 0");
    if (o->stencil_dtype != SEA_F64 && o->stencil_dtype != SEA_F32)
        return fail(ctx, SEA_E_ARG, "stencil_dtype must be SEA_F64 or SEA_F32");
    if (o->ace_dtype != SEA_F64 && o->ace_dtype != SEA_F32 && o->ace_dtype != SEA_BF16)
        return fail(ctx, SEA_E_ARG, "bad ace_dtype");
    if (o->start != SEA_START_ZERO && o->start != SEA_START_MULTIPOLE && o->start != SEA_START_LEARNED &&
        o->start != SEA_START_SPECTRAL)
        return fail(ctx, SEA_E_ARG, "bad start");
    if (o->nn_weight_dtype != SEA_F32 && o->nn_weight_dtype != SEA_BF16)
        return fail(ctx, SEA_E_ARG, "nn_weight_dtype must be SEA_F32 or SEA_BF16");
    if (o->ace_decomp != SEA_DECOMP_CHOLESKY && o->ace_decomp != SEA_DECOMP_EIGEN && o->ace_decomp != SEA_DECOMP_AUTO)
        return fail(ctx, SEA_E_ARG, "bad ace_decomp");
    if (!(o->cg_xc_beta_min >= 0.0) || !std::isfinite(o->cg_xc_beta_min))
        return fail(ctx, SEA_E_ARG, "cg_xc_beta_min must be finite and >= 0");
    if (o->cg_variant < -1 || o->cg_variant >= cg_variant_count())
        return fail(ctx, SEA_E_ARG, "cg_variant must be -1 or 0..%d", cg_variant_count() - 1);
    return SEA_OK;
}

sea_status check_grid(sea_ctx* ctx, const sea_grid* g) {
    if (!g) return fail(ctx, SEA_E_ARG, "grid is NULL");
    for (int a = 0; a < 3; ++a) {
        if (g->n[a] < 1) return fail(ctx, SEA_E_ARG, "grid n[%d] = %d < 1", a, g->n[a]);
        if (!(g->L[a] > 0.0) || !std::isfinite(g->L[a])) return fail(ctx, SEA_E_ARG, "grid L[%d] not positive", a);
    }
    return SEA_OK;
}

sea_status check_pairs(sea_ctx* ctx, int n_occ, int n_pairs, const sea_pair* pairs) {
    if (n_pairs < 0) return fail(ctx, SEA_E_ARG, "n_pairs < 0");
    if (n_pairs > 0 && !pairs) return fail(ctx, SEA_E_ARG, "pairs is NULL");
    for (int k = 0; k < n_pairs; ++k) {
        const sea_pair& p = pairs[k];
        if (p.i < 0 || p.j < p.i || p.j >= n_occ)
            return fail(ctx, SEA_E_ARG, "pair %d: need 0 <= i <= j < n_occ (i=%d j=%d n_occ=%d)", k, p.i, p.j, n_occ);
        for (int a = 0; a < 3; ++a) {
            if (p.n[a] < 1 || p.n[a] > 4096) return fail(ctx, SEA_E_ARG, "pair %d: domain n[%d]=%d out of range", k, a, p.n[a]);
            if (!std::isfinite(p.origin[a])) return fail(ctx, SEA_E_ARG, "pair %d: origin not finite", k);
        }
        if ((long long)p.n[0] * p.n[1] * p.n[2] > (1LL << 30))
            return fail(ctx, SEA_E_ARG, "pair %d: domain too large", k);
    }
    return SEA_OK;
}

}  // namespace

// Host view of the cells of one call: concatenated pairs, the cell of each
// pair, per-cell CSR lists (pair, partner) in pair order, device cell table.
struct CellSet {
    std::vector<sea_cell> cells;
    std::vector<sea_pair> pairs;
    std::vector<int> pair_cell;
    std::vector<int> csr_off;
    std::vector<int2> csr_ent;
    std::vector<DevCell> dev;
    std::vector<int> order;  // CG queue: pair ids by decreasing interior size (ties: id order)
    std::vector<int> dbox;   // 12 per pair: W_i box, W_j box (default: the pair's domain twice)
    bool cubic = true;
    int dst_shape = DST_SQUARE;   // DST_* bits of the pairs the sine transform takes
};

// the sine-transform kernel variants a call uses: the fixed ones, else the
// autotuner's, else the first
static void dst_variants(const sea_ctx* ctx, int& pv, int& zv) {
    const int np = dst_plane_variant_count(), nzv = dst_variant_count() - np;
    pv = ctx->dst_plane_fixed >= 0 ? ctx->dst_plane_fixed : (ctx->dst_plane_tuned >= 0 ? ctx->dst_plane_tuned : 0);
    zv = ctx->dst_zline_fixed >= 0 ? ctx->dst_zline_fixed : (ctx->dst_zline_tuned >= 0 ? ctx->dst_zline_tuned : 0);
    if (pv >= np) pv = 0;
    if (zv >= nzv) zv = 0;
}

// the scatter's schedule: the fixed one, else the autotuner's, else the first
static int scatter_variant(const sea_ctx* ctx) {
    const int v = ctx->scatter_fixed >= 0 ? ctx->scatter_fixed : (ctx->scatter_tuned >= 0 ? ctx->scatter_tuned : 0);
    return v < scatter_variant_count() ? v : 0;
}

static sea_status build_cellset(sea_ctx* ctx, int n_cells, const sea_cell* cells, bool action, CellSet& S) {
    if (n_cells < 1 || !cells) return fail(ctx, SEA_E_ARG, "need n_cells >= 1 and a cell array");
    S = CellSet{};
    S.cells.assign(cells, cells + n_cells);
    int csr_base = 0;
    for (int c = 0; c < n_cells; ++c) {
        const sea_cell& C = cells[c];
        sea_status st = check_grid(ctx, &C.grid);
        if (st != SEA_OK) return st;
        if (C.n_occ < 1) return fail(ctx, SEA_E_ARG, "cell %d: n_occ < 1", c);
        if (!C.phi_dev) return fail(ctx, SEA_E_ARG, "cell %d: phi_dev is NULL", c);
        if (C.phi_dtype != SEA_F64 && C.phi_dtype != SEA_F32)
            return fail(ctx, SEA_E_ARG, "cell %d: phi_dtype must be SEA_F64 or SEA_F32", c);
        if (action && !C.W_dev) return fail(ctx, SEA_E_ARG, "cell %d: W_dev is NULL", c);
        st = check_pairs(ctx, C.n_occ, C.n_pairs, C.pairs_host);
        if (st != SEA_OK) return st;
        DevCell D{};
        D.phi = C.phi_dev;
        D.phi_f32 = C.phi_dtype == SEA_F32;
        D.n_occ = C.n_occ;
        for (int k = 0; k < 3; ++k) {
            D.N[k] = C.grid.n[k];
            D.h[k] = C.grid.L[k] / C.grid.n[k];
        }
        if (D.h[0] != D.h[1] || D.h[0] != D.h[2]) S.cubic = false;
        D.dV = D.h[0] * D.h[1] * D.h[2];
        D.Ng = (size_t)D.N[0] * D.N[1] * D.N[2];
        D.W = C.W_dev;
        D.exx = C.exx_dev;
        D.pair_begin = (int)S.pairs.size();
        D.csr_base = csr_base;
        for (int k = 0; k < C.n_pairs; ++k) {
            const sea_pair& P = C.pairs_host[k];
            S.pairs.push_back(P);
            S.pair_cell.push_back(c);
            for (int side = 0; side < 2; ++side) {  // lo[3] then n[3] per side
                int box[6];
                for (int a2 = 0; a2 < 3; ++a2) {
                    box[a2] = C.dbox_host ? C.dbox_host[12 * k + 6 * side + a2] : P.lo[a2];
                    box[3 + a2] = C.dbox_host ? C.dbox_host[12 * k + 6 * side + 3 + a2] : P.n[a2];
                    if (box[3 + a2] < 1 || box[3 + a2] > 4096 || box[a2] < -(1 << 24) || box[a2] > (1 << 24))
                        return fail(ctx, SEA_E_ARG, "cell %d pair %d: W box out of range", c, k);
                }
                S.dbox.insert(S.dbox.end(), box, box + 6);
                for (int a2 = 0; a2 < 3; ++a2)
                    if (box[a2] != P.lo[a2] || box[3 + a2] != P.n[a2] || box[3 + a2] > D.N[a2]) D.wbox_general = 1;
            }
        }
        D.pair_end = (int)S.pairs.size();
        if (action) {
            std::vector<int> off(C.n_occ + 1, 0);
            for (int k = 0; k < C.n_pairs; ++k) {
                off[C.pairs_host[k].i + 1]++;
                if (C.pairs_host[k].j != C.pairs_host[k].i) off[C.pairs_host[k].j + 1]++;
            }
            for (int o = 0; o < C.n_occ; ++o) off[o + 1] += off[o];
            const int ent0 = (int)S.csr_ent.size();
            S.csr_ent.resize(ent0 + off[C.n_occ]);
            std::vector<int> fill(off.begin(), off.end() - 1);
            for (int k = 0; k < C.n_pairs; ++k) {
                const int gk = D.pair_begin + k;
                S.csr_ent[ent0 + fill[C.pairs_host[k].i]++] = make_int2(gk, C.pairs_host[k].j);
                if (C.pairs_host[k].j != C.pairs_host[k].i)
                    S.csr_ent[ent0 + fill[C.pairs_host[k].j]++] = make_int2(gk, C.pairs_host[k].i);
            }
            for (int o = 0; o <= C.n_occ; ++o) S.csr_off.push_back(ent0 + off[o]);
            csr_base += C.n_occ + 1;
        }
        S.dev.push_back(D);
    }
    if ((long long)S.pairs.size() > (1LL << 30)) return fail(ctx, SEA_E_ARG, "too many pairs");
    for (const auto& p : S.pairs)
        if (spectral_pair(p)) {
            if (p.n[0] != p.n[1]) S.dst_shape &= ~DST_SQUARE;
            S.dst_shape |= (p.n[2] & 1) ? DST_ZODD : DST_ZEVEN;
        }
    // longest-processing-time-first queue for the persistent CG kernels
    S.order.resize(S.pairs.size());
    for (size_t k = 0; k < S.pairs.size(); ++k) S.order[k] = (int)k;
    auto vol = [&](int k) { return (long long)S.pairs[k].n[0] * S.pairs[k].n[1] * S.pairs[k].n[2]; };
    std::stable_sort(S.order.begin(), S.order.end(), [&](int x, int y) { return vol(x) > vol(y); });
    return SEA_OK;
}

// FP64 state on the row-tile CG: cubic grids and pair domains with n[0], n[1] <= 64
static bool cg64_tiled(const sea_ctx* ctx, const CellSet& S) {
    return ctx->opts.stencil_dtype == SEA_F64 && S.cubic && !S.pairs.empty() &&
           cg_zm_fits(S.pairs.data(), (int)S.pairs.size(), nullptr) && residual_zm_lds_bytes() <= ctx->max_lds;
}

// The spectral start continued by the row-tile CG preconditioned with the
// sine transform: cubic grids and every pair taken by the transform
static bool cg64_pcg(const sea_ctx* ctx, const CellSet& S) {
    if (ctx->opts.start != SEA_START_SPECTRAL || !S.cubic || S.pairs.empty() ||
        residual_zm_lds_bytes() > ctx->max_lds)
        return false;
    for (const auto& p : S.pairs)
        if (!spectral_pair(p)) return false;
    return true;
}

// `eager`: a call that runs the sequence at once (not captured in a plan),
// which may take the row-tile CG and its state arrays
ExxLayout exx_layout(const sea_ctx* ctx, const CellSet& S, bool with_v, bool eager = true) {
    ExxLayout L{};
    const int n_pairs = (int)S.pairs.size();
    const sea_pair* pairs = S.pairs.data();
    size_t stride = 1;
    int nz_max = 1, nmax = 1;
    size_t pstride = 1;
    for (int k = 0; k < n_pairs; ++k) {
        const size_t n = (size_t)pairs[k].n[0] * pairs[k].n[1] * pairs[k].n[2];
        if (n > stride) stride = n;
        // the nz planes at the sine-transform passes' padded pitch
        const size_t pn = (size_t)dst_plane_pitch(pairs[k].n[0] * pairs[k].n[1], 1) * pairs[k].n[2];
        if (pn > pstride) pstride = pn;
        nz_max = pairs[k].n[2] > nz_max ? pairs[k].n[2] : nz_max;
        for (int d = 0; d < 3; ++d) nmax = pairs[k].n[d] > nmax ? pairs[k].n[d] : nmax;
    }
    stride = (stride + 31) / 32 * 32;
    L.stride = stride;
    L.pstride = std::max(stride, (pstride + 31) / 32 * 32);
    L.slot_stride = (size_t)64 * 64 * (nz_max + 1);
    if (L.slot_stride < stride) L.slot_stride = stride;
    L.n_chunks = exx_n_chunks((long)stride);
    L.n_zchunks = (nz_max + GC_ZC - 1) / GC_ZC;
    L.n_slots = n_pairs < ctx->n_cu * 4 ? (n_pairs > 0 ? n_pairs : 1) : ctx->n_cu * 4;
    L.nmax = nmax;
    L.ep_stride = 1;
    for (int k = 0; k < n_pairs; ++k) {
        const int ns = ep_slots(pairs[k], S.dev[S.pair_cell[k]].N);
        L.ep_stride = ns > L.ep_stride ? ns : L.ep_stride;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t np = n_pairs > 0 ? n_pairs : 1;
    const size_t nc = S.cells.size();
    L.pairs = take(np * sizeof(sea_pair));
    L.pair_cell = take(np * sizeof(int));
    L.order = take(np * sizeof(int));
    L.dbox = take(np * 12 * sizeof(int));
    L.cells = take(nc * sizeof(DevCell));
    L.partial = take(np * L.n_zchunks * GC_N * sizeof(double));
    L.racah_tab = take(GC_TAB * sizeof(double));
    L.mpoly = take(np * 84 * sizeof(double));
    L.mom = take(np * SEA_NACC * sizeof(double));
    L.b = take(np * stride * sizeof(double));
    L.v = with_v ? take(np * stride * sizeof(double)) : 0;
    // b - A x0 of a start guess: the generic FP64 kernel and the spectral
    // start (the FP32 z-march folds the other guesses into its first FP64
    // residual update)
    const bool spectral = ctx->opts.start == SEA_START_SPECTRAL;
    L.bres = ((ctx->opts.start != SEA_START_ZERO && ctx->opts.stencil_dtype == SEA_F64) || spectral)
                 ? take(np * L.pstride * sizeof(double)) : 0;   // also a sine-transform intermediate
    L.dst_tmp = spectral ? take(np * L.pstride * sizeof(double)) : 0;
    L.dst_tab = spectral ? take(dst_table_doubles() * sizeof(double)) : 0;
    L.dst_mu = spectral ? take(dst_mu_doubles() * sizeof(double)) : 0;
    const bool pcg = eager && cg64_pcg(ctx, S);
    const bool tiled64 = eager && (cg64_tiled(ctx, S) || pcg);
    L.rnorm = (spectral || tiled64) ? take(np * RZ_TILES * 2 * sizeof(double)) : 0;
    L.cg_r = tiled64 ? take(np * stride * sizeof(double)) : 0;
    L.cg_p = tiled64 ? take(2 * np * stride * sizeof(double)) : 0;
    L.cg_part = tiled64 ? take(np * RZ_TILES * 8 * sizeof(double)) : 0;
    L.cg_rho = tiled64 ? take(np * 2 * sizeof(double)) : 0;
    L.cg_done = tiled64 ? take(np * sizeof(int)) : 0;
    L.cg_active = tiled64 ? take(((size_t)ctx->opts.max_iter + 2) * sizeof(int)) : 0;
    L.cg_z = pcg ? take(np * stride * sizeof(double)) : 0;
    L.epart = take(np * (size_t)L.ep_stride * sizeof(double));
    L.slots = take((size_t)L.n_slots * 4 * L.slot_stride * sizeof(double));
    L.stats = take(np * sizeof(DevStat));
    L.csr_off = take((S.csr_off.size() + 1) * sizeof(int));
    L.csr_ent = take((S.csr_ent.size() + 1) * sizeof(int2));
    L.scal = take((3 * nc + 8) * sizeof(double));
    L.counter = take(256);
    if (ctx->opts.start == SEA_START_LEARNED) {
        const size_t d3 = (size_t)kNnGrid * kNnGrid * kNnGrid;
        L.nnx = take(np * d3 * sizeof(float));
        L.nny = take(np * d3 * sizeof(float));
        L.nnact = ctx->opts.nn_weight_dtype == SEA_BF16 ? take(nn_infer_layout(kNnMfmaBatch).total_bytes)
                                                         : take(nn_act_layout(kNnInferBatch, kNnGrid).total_floats * sizeof(float));
    }
    L.total = off;
    return L;
}

// Pointers into the network state: FP32 parameters, BF16 copy, Adam m, v.
struct NnState {
    float* p;
    uint16_t* p16;
    float* m;
    float* v;
};
static size_t nn_state_total(size_t P) {
    size_t off = align_up(P * sizeof(float));
    off += align_up(P * sizeof(uint16_t));
    off += 2 * align_up(P * sizeof(float));
    return off;
}
static NnState nn_state_ptrs(const void* base) {
    const size_t P = nn_param_count();
    char* b = (char*)base;
    NnState st;
    st.p = (float*)b;
    st.p16 = (uint16_t*)(b + align_up(P * sizeof(float)));
    st.m = (float*)(b + align_up(P * sizeof(float)) + align_up(P * sizeof(uint16_t)));
    st.v = (float*)((char*)st.m + align_up(P * sizeof(float)));
    return st;
}

extern "C" {

const char* sea_version(void) { return "sea-mi355x 0.1 (gfx950)"; }

void sea_opts_default(sea_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->fd_half_order = 6;
    o->lmax = 6;
    o->rel_tol = 1e-8;
    o->max_iter = 10000;
    o->stencil_dtype = SEA_F64;
    o->ace_dtype = SEA_F64;
    o->start = SEA_START_ZERO;
    o->cg_variant = -1;
    o->ace_decomp = SEA_DECOMP_CHOLESKY;
    o->cg_xc_beta_min = 0.0;
    o->profile = 0;
    o->nn_weight_dtype = SEA_BF16;
    o->hip_stream = nullptr;
}

sea_status sea_create(const sea_opts* opts, sea_ctx** out) {
    if (!out) return SEA_E_ARG;
    *out = nullptr;
    sea_ctx* ctx = new (std::nothrow) sea_ctx();
    if (!ctx) return SEA_E_NOMEM;
    sea_opts def;
    sea_opts_default(&def);
    sea_status st = check_opts(ctx, opts ? opts : &def);
    if (st != SEA_OK) {
        delete ctx;
        return st;
    }
    ctx->opts = opts ? *opts : def;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete ctx;
        return SEA_E_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete ctx;
        return SEA_E_HIP;
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
        delete ctx;
        return SEA_E_HIP;
    }
    ctx->device = dev;
    ctx->noalloc_scratch = noalloc_scratch_setup(dev);
    ctx->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    ctx->max_lds = prop.sharedMemPerBlock;
    bool ok = true;
    for (int k = 0; k < SEA_STAGE_COUNT; ++k)
        for (int e = 0; e < 2; ++e) ok = ok && hipEventCreate(&ctx->ev[k][e]) == hipSuccess;
    ctx->ev_ready = ok;
    *out = ctx;
    return SEA_OK;
}

sea_status sea_destroy(sea_ctx* ctx) {
    if (ctx && ctx->ev_ready)
        for (int k = 0; k < SEA_STAGE_COUNT; ++k)
            for (int e = 0; e < 2; ++e) (void)hipEventDestroy(ctx->ev[k][e]);

    delete ctx;
    return SEA_OK;
}

sea_status sea_stage_times(sea_ctx* ctx, float* ms_out) {
    if (!ctx || !ms_out) return SEA_E_ARG;
    for (int k = 0; k < SEA_STAGE_COUNT; ++k) {
        ms_out[k] = 0.0f;
        if (!ctx->ev_used[k]) continue;
        SEA_HIP_CHECK(ctx, hipEventSynchronize(ctx->ev[k][1]));
        float ms = 0.0f;
        SEA_HIP_CHECK(ctx, hipEventElapsedTime(&ms, ctx->ev[k][0], ctx->ev[k][1]));
        ms_out[k] = ms;
    }
    return SEA_OK;
}

const char* sea_last_error(const sea_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

sea_status sea_set_opts(sea_ctx* ctx, const sea_opts* opts) {
    if (!ctx) return SEA_E_ARG;
    sea_status st = check_opts(ctx, opts);
    if (st != SEA_OK) return st;
    ctx->opts = *opts;
    return SEA_OK;
}

sea_status sea_build_pairs(const sea_grid* grid, int n_occ, const double* c, double r_pair, double half_width,
                           sea_pair* out, int cap, int* n_out) {
    if (check_grid(nullptr, grid) != SEA_OK || n_occ < 0 || (n_occ > 0 && !c) || !n_out || cap < 0 ||
        (cap > 0 && !out) || !(r_pair >= 0.0) || !(half_width >= 0.0))
        return SEA_E_ARG;
    const int cnt = host_build_pairs(grid->n, grid->L, n_occ, c, r_pair, half_width, out, cap);
    *n_out = cnt;
    return cnt > cap ? SEA_E_NOMEM : SEA_OK;
}

static sea_cell one_cell(const sea_grid* grid, int n_occ, const void* phi, sea_dtype dt, int n_pairs,
                         const sea_pair* pairs, double* W, double* exx_dev) {
    sea_cell c{};
    if (grid) c.grid = *grid;
    c.n_occ = n_occ;
    c.phi_dtype = dt;
    c.phi_dev = phi;
    c.n_pairs = n_pairs;
    c.pairs_host = pairs;
    c.W_dev = W;
    c.exx_dev = exx_dev;
    return c;
}

sea_status sea_exx_workspace_bytes(sea_ctx* ctx, const sea_grid* grid, int n_occ, int n_pairs, const sea_pair* pairs,
                                   size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    if (!grid) return fail(ctx, SEA_E_ARG, "grid is NULL");
    sea_cell c = one_cell(grid, n_occ, (const void*)1, SEA_F64, n_pairs, pairs, (double*)1, nullptr);
    CellSet S;
    sea_status st = build_cellset(ctx, 1, &c, true, S);
    if (st != SEA_OK) return st;
    *bytes = exx_layout(ctx, S, true).total;
    return SEA_OK;
}

sea_status sea_exx_plan_workspace_bytes(sea_ctx* ctx, int n_cells, const sea_cell* cells, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    std::vector<sea_cell> cs(cells, cells + (n_cells > 0 && cells ? n_cells : 0));
    for (auto& c : cs) {
        if (!c.phi_dev) c.phi_dev = (const void*)1;  // sizing does not read buffers
        if (!c.W_dev) c.W_dev = (double*)1;
    }
    CellSet S;
    sea_status st = build_cellset(ctx, n_cells, cs.data(), true, S);
    if (st != SEA_OK) return st;
    *bytes = exx_layout(ctx, S, true, false).total;
    return SEA_OK;
}

sea_status sea_exx_batched_workspace_bytes(sea_ctx* ctx, int n_cells, const sea_cell* cells, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    std::vector<sea_cell> cs(cells, cells + (n_cells > 0 && cells ? n_cells : 0));
    for (auto& c : cs) {
        if (!c.phi_dev) c.phi_dev = (const void*)1;  // sizing does not read buffers
        if (!c.W_dev) c.W_dev = (double*)1;
    }
    CellSet S;
    sea_status st = build_cellset(ctx, n_cells, cs.data(), true, S);
    if (st != SEA_OK) return st;
    *bytes = exx_layout(ctx, S, true).total;
    return SEA_OK;
}

// Options of one enqueue of the exx kernel sequence.
struct ExxFlags {
    bool action = true;         // scatter W
    double* Q_dev = nullptr;    // orthonormal moments out
    double* e_dev = nullptr;    // per-pair energies out
    int nn_D = 0;               // training samples out
    float* nn_x = nullptr;
    float* nn_t = nullptr;
    double* nn_s = nullptr;
    bool profile = false;
};

static sea_status exx_upload(sea_ctx* ctx, const CellSet& S, const ExxLayout& Ly, char* base, hipStream_t s) {
    const size_t np = S.pairs.size();
    if (np) {
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(base + Ly.pairs, S.pairs.data(), sizeof(sea_pair) * np, hipMemcpyHostToDevice, s));
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(base + Ly.pair_cell, S.pair_cell.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(base + Ly.order, S.order.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(base + Ly.dbox, S.dbox.data(), sizeof(int) * 12 * np, hipMemcpyHostToDevice, s));
    }
    SEA_HIP_CHECK(ctx, hipMemcpyAsync(base + Ly.cells, S.dev.data(), sizeof(DevCell) * S.dev.size(), hipMemcpyHostToDevice, s));
    if (!S.csr_off.empty())
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(base + Ly.csr_off, S.csr_off.data(), sizeof(int) * S.csr_off.size(), hipMemcpyHostToDevice, s));
    if (!S.csr_ent.empty())
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(base + Ly.csr_ent, S.csr_ent.data(), sizeof(int2) * S.csr_ent.size(), hipMemcpyHostToDevice, s));
    // the host tables must outlive the copies
    SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    return SEA_OK;
}

static ExxArgs exx_args(sea_ctx* ctx, const CellSet& S, const ExxLayout& Ly, char* base, double* v_ext) {
    ExxArgs a{};
    a.pairs = (const sea_pair*)(base + Ly.pairs);
    a.n_pairs = (int)S.pairs.size();
    a.cells = (const DevCell*)(base + Ly.cells);
    a.pair_cell = (const int*)(base + Ly.pair_cell);
    a.order = S.pairs.empty() ? nullptr : (const int*)(base + Ly.order);
    a.dbox = (const int*)(base + Ly.dbox);
    a.n_cells = (int)S.cells.size();
    a.partial = (double*)(base + Ly.partial);
    a.n_chunks = Ly.n_chunks;
    a.n_zchunks = Ly.n_zchunks;
    a.racah_tab = (double*)(base + Ly.racah_tab);
    a.mpoly = (double*)(base + Ly.mpoly);
    a.mom = (double*)(base + Ly.mom);
    a.b = (double*)(base + Ly.b);
    a.v = v_ext ? v_ext : (double*)(base + Ly.v);
    a.stride = Ly.stride;
    a.pstride = Ly.pstride;
    a.slots = (double*)(base + Ly.slots);
    a.slot_stride = Ly.slot_stride;
    a.n_slots = Ly.n_slots;
    a.stats = (DevStat*)(base + Ly.stats);
    a.rel_tol = ctx->opts.rel_tol;
    a.xc_beta_min = ctx->opts.cg_xc_beta_min > 0.0 ? ctx->opts.cg_xc_beta_min : 0.25;
    a.max_iter = ctx->opts.max_iter;
    a.lmax = ctx->opts.lmax;
    a.queue_ctr = (int*)(base + Ly.counter);
    a.x_nonzero = ctx->opts.start != SEA_START_ZERO;
    a.bres = Ly.bres ? (double*)(base + Ly.bres) : nullptr;
    // spectral start: -D x0 on the face points (in the transform's scratch
    // array)
    a.fcorr = Ly.dst_tmp ? (double*)(base + Ly.dst_tmp) : nullptr;
    a.nmax = Ly.nmax;
    a.epart = nullptr;   // set by the sequences that take the energies from the scatter
    a.ep_stride = Ly.ep_stride;
    a.cg_r = Ly.cg_r ? (double*)(base + Ly.cg_r) : nullptr;
    a.cg_p = Ly.cg_p ? (double*)(base + Ly.cg_p) : nullptr;
    a.cg_part = Ly.cg_part ? (double*)(base + Ly.cg_part) : nullptr;
    a.cg_rho = Ly.cg_rho ? (double*)(base + Ly.cg_rho) : nullptr;
    a.cg_done = Ly.cg_done ? (int*)(base + Ly.cg_done) : nullptr;
    a.cg_active = Ly.cg_active ? (int*)(base + Ly.cg_active) : nullptr;
    a.cg_z = Ly.cg_z ? (double*)(base + Ly.cg_z) : nullptr;
    a.cg_pre = 0;
    a.cg_it = 0;
    a.hist = ctx->hist;
    a.hist_len = ctx->hist_len;
    return a;
}

// The FP64 row-tile CG: init, then two sweeps per iteration until every pair
// has stopped (checked from the per-iteration counters every few
// iterations, which synchronizes), then the true residual's norms into
// rel_res.  Preconditioned (`pre`, after a spectral start whose norms are in
// rnorm): the init stops the pairs whose start already meets the target,
// and z = A_odd^-1 r (three transform passes, tmp and tmp2 scratch) and
// <r, z> follow each sweep B.
struct Cg64Pre {
    double *tmp, *tmp2, *tab, *mu;
    int pv, zv;
    int shape;
};
static sea_status cg64_run(sea_ctx* ctx, const ExxArgs& a0, double* rnorm, hipStream_t s, const Cg64Pre* pre) {
    ExxArgs a = a0;
    a.cg_pre = pre ? 1 : 0;
    a.rnorm = pre ? rnorm : nullptr;   // start norms: which pairs the init stops
    SEA_HIP_CHECK(ctx, launch_fill_int(a.cg_active, (size_t)a.max_iter + 2, s));
    SEA_HIP_CHECK(ctx, launch_cg64_init(a, s));
    if (pre) {   // every start already meets the target: nothing iterates
        int active = 0;
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(&active, a.cg_active + a.max_iter + 1, sizeof(int), hipMemcpyDeviceToHost, s));
        SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
        if (active == 0) return SEA_OK;
    }
    auto precondition = [&](int k) -> sea_status {
        SEA_HIP_CHECK(ctx, launch_dst_solve(a, a.cg_r, a.cg_z, pre->tmp, pre->tmp2, pre->tab, pre->mu, pre->pv,
                                            pre->zv, pre->shape, a.cg_done, s));
        ExxArgs ad = a;
        ad.cg_it = k;
        SEA_HIP_CHECK(ctx, launch_cg64_dot(ad, s));
        return SEA_OK;
    };
    if (pre) {
        const sea_status st = precondition(-1);
        if (st != SEA_OK) return st;
    }
    const int every = pre ? 4 : 16;
    for (int k = 0;; ++k) {
        a.cg_it = k;
        SEA_HIP_CHECK(ctx, launch_cg64_sweep(a, 0, s));
        if (k >= a.max_iter) break;
        SEA_HIP_CHECK(ctx, launch_cg64_sweep(a, 1, s));
        if (pre) {
            const sea_status st = precondition(k);
            if (st != SEA_OK) return st;
        }
        if (k % every == every - 1) {
            int active = 0;
            SEA_HIP_CHECK(ctx, hipMemcpyAsync(&active, a.cg_active + k, sizeof(int), hipMemcpyDeviceToHost, s));
            SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
            if (active == 0) break;
        }
    }
    a.rnorm = rnorm;
    SEA_HIP_CHECK(ctx, launch_residual_zm(a, s, false));
    SEA_HIP_CHECK(ctx, launch_cg64_exit(a, s));
    return SEA_OK;
}

// The whole kernel sequence of one call, on stream s (capturable).
static sea_status exx_enqueue(sea_ctx* ctx, const CellSet& S, const ExxLayout& Ly, char* base, const ExxArgs& a,
                              const ExxFlags& f, hipStream_t s) {
    const int n_pairs = a.n_pairs;
    const bool prof = f.profile && ctx->opts.profile;
    auto timer_on = [&](int st) {
        if (prof && ctx->ev_ready) {
            (void)hipEventRecord(ctx->ev[st][0], s);
            ctx->ev_used[st] = true;
        }
    };
    auto timer_off = [&](int st) {
        if (prof && ctx->ev_ready) (void)hipEventRecord(ctx->ev[st][1], s);
    };
    for (int k = SEA_STAGE_GATHER; k <= SEA_STAGE_ENERGY; ++k) ctx->ev_used[k] = false;
    ctx->ev_used[SEA_STAGE_FINISH] = false;
    for (int k = SEA_STAGE_DST; k <= SEA_STAGE_FOLD; ++k) ctx->ev_used[k] = false;
    const bool zm = ctx->opts.stencil_dtype == SEA_F32 && S.cubic && cg_zm_fits(S.pairs.data(), n_pairs, nullptr) &&
                    cg_zm_lds_bytes(1) <= ctx->max_lds;
    // FP64 state: the row-tile CG, except under graph capture (its host loop
    // checks progress), where the per-pair kernel runs
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusActive;
    const bool nocap = cap == hipStreamCaptureStatusNone;
    const bool tiled64 = cg64_tiled(ctx, S) && a.cg_r && nocap;
    // the spectral start's continuation: the sine-transform-preconditioned CG
    const bool pcg = cg64_pcg(ctx, S) && a.cg_z && nocap;
    const bool finish = zm || tiled64 || pcg;   // pair energies and flags by k_cg_finish
    if (!zm && ctx->opts.stencil_dtype != SEA_F64)
        return fail(ctx, SEA_E_ARG, "SEA_F32 state needs cubic grids and pair domains with n[0], n[1] <= 64");
    int nz_max = 1;
    for (const auto& p : S.pairs) nz_max = p.n[2] > nz_max ? p.n[2] : nz_max;
    if (n_pairs > 0) {
        if (a.hist) SEA_HIP_CHECK(ctx, launch_fill_nan(a.hist, (size_t)n_pairs * (a.hist_len + 1), s));
        timer_on(SEA_STAGE_GATHER);
        SEA_HIP_CHECK(ctx, launch_gather_moments(a, s));
        SEA_HIP_CHECK(ctx, launch_moments_final(a, f.Q_dev, s));
        timer_off(SEA_STAGE_GATHER);
        const bool spectral = ctx->opts.start == SEA_START_SPECTRAL;
        timer_on(SEA_STAGE_BOUNDARY);
        // spectral start: the full multipole start for the pairs the sine
        // transform skips; the fold forms -D x0 on the others' face points
        if (spectral) {
            timer_on(SEA_STAGE_FACE);
            SEA_HIP_CHECK(ctx, launch_me_big(a, nz_max, s));
            timer_off(SEA_STAGE_FACE);
        }
        timer_on(SEA_STAGE_FOLD);
        SEA_HIP_CHECK(ctx, launch_boundary_fold(a, nz_max, s, spectral));
        timer_off(SEA_STAGE_FOLD);
        timer_off(SEA_STAGE_BOUNDARY);
        if (a.x_nonzero) {
            timer_on(SEA_STAGE_GUESS);
            if (!spectral) SEA_HIP_CHECK(ctx, launch_me_guess(a, s));
            if (ctx->opts.start == SEA_START_LEARNED) {
                float* x32 = (float*)(base + Ly.nnx);
                float* y32 = (float*)(base + Ly.nny);
                const NnState st = nn_state_ptrs(ctx->nn_state);
                const size_t d3 = (size_t)kNnGrid * kNnGrid * kNnGrid;
                SEA_HIP_CHECK(ctx, launch_nn_sample(a, kNnGrid, x32, nullptr, 0, s));
                if (ctx->opts.nn_weight_dtype == SEA_BF16) {  // matrix cores, BF16 activations
                    const NnInferLayout IL = nn_infer_layout(kNnMfmaBatch);
                    for (int p0 = 0; p0 < n_pairs; p0 += kNnMfmaBatch) {
                        const int nb = n_pairs - p0 < kNnMfmaBatch ? n_pairs - p0 : kNnMfmaBatch;
                        SEA_HIP_CHECK(ctx, nn_infer(st.p, st.p16, x32 + p0 * d3, base + Ly.nnact, IL, nb,
                                                    y32 + p0 * d3, s));
                    }
                } else {  // FP32 weights and activations (vector ALUs)
                    float* act = (float*)(base + Ly.nnact);
                    const NnActLayout AL = nn_act_layout(kNnInferBatch, kNnGrid);
                    for (int p0 = 0; p0 < n_pairs; p0 += kNnInferBatch) {
                        const int nb = n_pairs - p0 < kNnInferBatch ? n_pairs - p0 : kNnInferBatch;
                        SEA_HIP_CHECK(ctx, nn_forward(st.p, nullptr, x32 + p0 * d3, act, AL, nb, kNnGrid,
                                                      y32 + p0 * d3, s));
                    }
                }
                SEA_HIP_CHECK(ctx, launch_nn_apply(a, kNnGrid, y32, s));
            }
            if (spectral) {
                // x = A_odd^-1 (b - D x0); then, for the FP32 z-march, the true
                // residual b - A x in FP64: its norms for every pair, and bres
                // for the pairs whose start is not yet converged (the FP64
                // kernel forms its residual itself)
                int pv = 0, zv = 0;
                dst_variants(ctx, pv, zv);
                SEA_HIP_CHECK(ctx, launch_spectral_start(a, a.bres, (double*)(base + Ly.dst_tmp),
                                                         (double*)(base + Ly.dst_tab), (double*)(base + Ly.dst_mu), pv,
                                                         zv, S.dst_shape, s,
                                                         [&](int pass, bool begin) {
                                                             const int st = SEA_STAGE_DST_PLANE_FWD + pass;
                                                             if (begin) {
                                                                 if (pass == 0) timer_on(SEA_STAGE_DST);
                                                                 timer_on(st);
                                                             } else {
                                                                 timer_off(st);
                                                                 if (pass == 2) timer_off(SEA_STAGE_DST);
                                                             }
                                                         }));
                if (zm || pcg) {
                    ExxArgs ar = a;
                    ar.rnorm = (double*)(base + Ly.rnorm);
                    ar.cg_done = nullptr;   // (stale flags of an earlier call)
                    const bool rzm = residual_zm_lds_bytes() <= ctx->max_lds;
                    timer_on(SEA_STAGE_RESIDUAL);
                    // (the preconditioned continuation forms its residual itself)
                    SEA_HIP_CHECK(ctx, rzm ? launch_residual_zm(ar, s, !pcg) : launch_start_residual(ar, s));
                    timer_off(SEA_STAGE_RESIDUAL);
                }
            } else if (!zm && !tiled64 && !pcg) {
                SEA_HIP_CHECK(ctx, launch_start_residual(a, s));
            }
            timer_off(SEA_STAGE_GUESS);
        }
        timer_on(SEA_STAGE_CG);
        if (pcg) {
            int pv = 0, zv = 0;
            dst_variants(ctx, pv, zv);
            const Cg64Pre pre{(double*)(base + Ly.dst_tmp), a.bres, (double*)(base + Ly.dst_tab),
                              (double*)(base + Ly.dst_mu), pv, zv, S.dst_shape};
            sea_status st = cg64_run(ctx, a, (double*)(base + Ly.rnorm), s, &pre);
            if (st != SEA_OK) return st;
            timer_off(SEA_STAGE_CG);
            if (!f.action) {
                timer_on(SEA_STAGE_FINISH);
                SEA_HIP_CHECK(ctx, launch_cg_finish(a, s));
                timer_off(SEA_STAGE_FINISH);
            }
        } else if (zm) {
            const int var = ctx->opts.cg_variant >= 0 ? ctx->opts.cg_variant : (ctx->cg_tuned >= 0 ? ctx->cg_tuned : 0);
            ExxArgs az = a;
            // spectral start: x is the FP64 start and bres = b - A x (rnorm: its
            // norms decide first, and bres is only there for the pairs they fail)
            az.start_res = ctx->opts.start == SEA_START_SPECTRAL ? 1 : 0;
            az.rnorm = (az.start_res && residual_zm_lds_bytes() <= ctx->max_lds) ? (double*)(base + Ly.rnorm) : nullptr;
            SEA_HIP_CHECK(ctx, launch_cg_zm(az, var, s));
            timer_off(SEA_STAGE_CG);
            if (!f.action) {
                timer_on(SEA_STAGE_FINISH);
                SEA_HIP_CHECK(ctx, launch_cg_finish(a, s));
                timer_off(SEA_STAGE_FINISH);
            }
        } else if (tiled64) {
            sea_status st = cg64_run(ctx, a, (double*)(base + Ly.rnorm), s, nullptr);
            if (st != SEA_OK) return st;
            timer_off(SEA_STAGE_CG);
            if (!f.action) {
                timer_on(SEA_STAGE_FINISH);
                SEA_HIP_CHECK(ctx, launch_cg_finish(a, s));
                timer_off(SEA_STAGE_FINISH);
            }
        } else {
            SEA_HIP_CHECK(ctx, launch_cg(a, s));
            timer_off(SEA_STAGE_CG);
        }
    }
    if (f.action) {
        // z-march path: the scatter also forms the pair energies' partials,
        // which the finish pass then sums (in slot order) with the flags
        ExxArgs ae = a;
        bool lists_fit = true;   // every orbital's pair list fits the scatter's energy arrays
        for (size_t k = 0; k + 1 < S.csr_off.size(); ++k)
            lists_fit = lists_fit && S.csr_off[k + 1] - S.csr_off[k] <= SC_EP_MAXE;
        if (finish && n_pairs > 0 && lists_fit) ae.epart = (double*)(base + Ly.epart);
        timer_on(SEA_STAGE_SCATTER);
        if (ae.epart) SEA_HIP_CHECK(ctx, launch_epart_clear(ae, s));
        for (size_t c = 0; c < S.cells.size(); ++c)
            SEA_HIP_CHECK(ctx, launch_scatter(ae, S.dev[c], (const int*)(base + Ly.csr_off),
                                              (const int2*)(base + Ly.csr_ent), scatter_variant(ctx), s));
        timer_off(SEA_STAGE_SCATTER);
        if (finish && n_pairs > 0) {   // without ae.epart the finish sums rho x itself
            timer_on(SEA_STAGE_FINISH);
            SEA_HIP_CHECK(ctx, launch_cg_finish(ae, s));
            timer_off(SEA_STAGE_FINISH);
        }
    }
    timer_on(SEA_STAGE_ENERGY);
    SEA_HIP_CHECK(ctx, launch_energy_sum(a, (double*)(base + Ly.scal), f.e_dev, s));
    timer_off(SEA_STAGE_ENERGY);
    if (f.nn_x && n_pairs > 0) {
        SEA_HIP_CHECK(ctx, launch_nn_sample(a, f.nn_D, f.nn_x, f.nn_s, 0, s));
        SEA_HIP_CHECK(ctx, launch_nn_sample(a, f.nn_D, f.nn_t, nullptr, 1, s));
    }
    return SEA_OK;
}

// Read E per cell and per-pair stats after the stream has drained; sets the
// warning/error status from the per-cell counters.
static sea_status exx_results(sea_ctx* ctx, const CellSet& S, const ExxLayout& Ly, char* base, hipStream_t s,
                              double* exx_host, sea_pair_stat* stats_host) {
    const size_t nc = S.cells.size();
    std::vector<double> hs(3 * nc);
    SEA_HIP_CHECK(ctx, hipMemcpyAsync(hs.data(), base + Ly.scal, sizeof(double) * 3 * nc, hipMemcpyDeviceToHost, s));
    if (stats_host && !S.pairs.empty())
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(stats_host, base + Ly.stats, sizeof(DevStat) * S.pairs.size(),
                                          hipMemcpyDeviceToHost, s));
    SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    double nconv = 0.0, nbad = 0.0;
    for (size_t c = 0; c < nc; ++c) {
        if (exx_host) exx_host[c] = hs[3 * c];
        nconv += hs[3 * c + 1];
        nbad += hs[3 * c + 2];
        if (!std::isfinite(hs[3 * c])) nbad += 1.0;
    }
    if (nbad > 0.0) return fail(ctx, SEA_E_NONFINITE, "%d pair solves produced non-finite values", (int)nbad);
    if (nconv > 0.0) {
        fail(ctx, SEA_W_NOT_CONVERGED, "%d pairs did not reach rel_tol within max_iter", (int)nconv);
        return SEA_W_NOT_CONVERGED;
    }
    return SEA_OK;
}

static sea_status exx_run(sea_ctx* ctx, int n_cells, const sea_cell* cells, void* ws_dev, size_t ws_bytes,
                          double* v_ext, const ExxFlags& f, double* exx_host, sea_pair_stat* stats_host) {
    if (!ctx) return SEA_E_ARG;
    if (!ws_dev) return fail(ctx, SEA_E_ARG, "workspace is NULL");
    if (ctx->opts.start == SEA_START_LEARNED && !ctx->nn_state)
        return fail(ctx, SEA_E_ARG, "SEA_START_LEARNED needs a network (sea_nn_attach)");
    CellSet S;
    sea_status st = build_cellset(ctx, n_cells, cells, f.action, S);
    if (st != SEA_OK) return st;
    const ExxLayout Ly = exx_layout(ctx, S, true);
    if (ws_bytes < Ly.total) return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, Ly.total);
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    st = exx_upload(ctx, S, Ly, base, s);
    if (st != SEA_OK) return st;
    const ExxArgs a = exx_args(ctx, S, Ly, base, v_ext);
    st = exx_enqueue(ctx, S, Ly, base, a, f, s);
    if (st != SEA_OK) return st;
    if (exx_host || stats_host) return exx_results(ctx, S, Ly, base, s, exx_host, stats_host);
    return SEA_OK;
}

sea_status sea_exx_action(sea_ctx* ctx, const sea_grid* grid, int n_occ, const void* phi_dev, sea_dtype phi_dtype,
                          int n_pairs, const sea_pair* pairs_host, void* ws_dev, size_t ws_bytes, double* W_dev,
                          double* exx_dev, double* exx_host, sea_pair_stat* stats_host) {
    if (!ctx) return SEA_E_ARG;
    if (!grid) return fail(ctx, SEA_E_ARG, "grid is NULL");
    if (!W_dev) return fail(ctx, SEA_E_ARG, "W_dev is NULL");
    const sea_cell c = one_cell(grid, n_occ, phi_dev, phi_dtype, n_pairs, pairs_host, W_dev, exx_dev);
    ExxFlags f;
    f.profile = true;
    return exx_run(ctx, 1, &c, ws_dev, ws_bytes, nullptr, f, exx_host, stats_host);
}

sea_status sea_exx_action_batched(sea_ctx* ctx, int n_cells, const sea_cell* cells, void* ws_dev, size_t ws_bytes,
                                  double* exx_host, sea_pair_stat* stats_host) {
    if (!ctx) return SEA_E_ARG;
    ExxFlags f;
    f.profile = true;
    return exx_run(ctx, n_cells, cells, ws_dev, ws_bytes, nullptr, f, exx_host, stats_host);
}

sea_status sea_exx_pair_solve(sea_ctx* ctx, const sea_grid* grid, int n_occ, const void* phi_dev, sea_dtype phi_dtype,
                              int n_pairs, const sea_pair* pairs_host, void* ws_dev, size_t ws_bytes, double* v_dev,
                              double* Q_dev, double* e_dev, sea_pair_stat* stats_host) {
    if (!ctx) return SEA_E_ARG;
    if (!grid) return fail(ctx, SEA_E_ARG, "grid is NULL");
    if (!v_dev) return fail(ctx, SEA_E_ARG, "v_dev is NULL");
    const sea_cell c = one_cell(grid, n_occ, phi_dev, phi_dtype, n_pairs, pairs_host, nullptr, nullptr);
    ExxFlags f;
    f.action = false;
    f.Q_dev = Q_dev;
    f.e_dev = e_dev;
    f.profile = true;
    return exx_run(ctx, 1, &c, ws_dev, ws_bytes, v_dev, f, nullptr, stats_host);
}

sea_status sea_exx_nn_samples(sea_ctx* ctx, const sea_grid* grid, int n_occ, const void* phi_dev, sea_dtype phi_dtype,
                              int n_pairs, const sea_pair* pairs_host, void* ws_dev, size_t ws_bytes, int D,
                              float* x_dev, float* t_dev, double* s_dev, sea_pair_stat* stats_host) {
    if (!ctx) return SEA_E_ARG;
    if (!grid) return fail(ctx, SEA_E_ARG, "grid is NULL");
    if (D < 2 || !x_dev || !t_dev) return fail(ctx, SEA_E_ARG, "need D >= 2 and x_dev, t_dev");
    for (int k = 0; k < n_pairs && pairs_host; ++k)
        for (int d = 0; d < 3; ++d)
            if (pairs_host[k].n[d] < 2) return fail(ctx, SEA_E_ARG, "pair %d: domain extent < 2", k);
    const sea_cell c = one_cell(grid, n_occ, phi_dev, phi_dtype, n_pairs, pairs_host, nullptr, nullptr);
    ExxFlags f;
    f.action = false;
    f.nn_D = D;
    f.nn_x = x_dev;
    f.nn_t = t_dev;
    f.nn_s = s_dev;
    f.profile = true;
    return exx_run(ctx, 1, &c, ws_dev, ws_bytes, nullptr, f, nullptr, stats_host);
}

size_t sea_nn_param_count(void) { return nn_param_count(); }

sea_status sea_nn_state_bytes(sea_ctx* ctx, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    *bytes = nn_state_total(nn_param_count());
    return SEA_OK;
}

sea_status sea_nn_set_params(sea_ctx* ctx, void* state_dev, const float* params_host) {
    if (!ctx) return SEA_E_ARG;
    if (!state_dev || !params_host) return fail(ctx, SEA_E_ARG, "NULL argument");
    const size_t P = nn_param_count();
    for (size_t i = 0; i < P; ++i)
        if (!std::isfinite(params_host[i])) return fail(ctx, SEA_E_NONFINITE, "parameter %zu is not finite", i);
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    const NnState st = nn_state_ptrs(state_dev);
    SEA_HIP_CHECK(ctx, hipMemcpyAsync(st.p, params_host, P * sizeof(float), hipMemcpyHostToDevice, s));
    SEA_HIP_CHECK(ctx, hipMemsetAsync(st.m, 0, P * sizeof(float), s));
    SEA_HIP_CHECK(ctx, hipMemsetAsync(st.v, 0, P * sizeof(float), s));
    SEA_HIP_CHECK(ctx, nn_to_bf16(st.p, st.p16, (long)P, s));
    SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    return SEA_OK;
}

sea_status sea_nn_get_params(sea_ctx* ctx, const void* state_dev, float* params_host) {
    if (!ctx) return SEA_E_ARG;
    if (!state_dev || !params_host) return fail(ctx, SEA_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    const NnState st = nn_state_ptrs(state_dev);
    SEA_HIP_CHECK(ctx, hipMemcpyAsync(params_host, st.p, nn_param_count() * sizeof(float), hipMemcpyDeviceToHost, s));
    SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    return SEA_OK;
}

static sea_status nn_check(sea_ctx* ctx, int batch, int D) {
    if (batch < 1) return fail(ctx, SEA_E_ARG, "batch < 1");
    if (D < 8 || D > 64 || D % 8) return fail(ctx, SEA_E_ARG, "D must be a multiple of 8 in 8..64");
    return SEA_OK;
}

static size_t nn_ws_total(int batch, int D) {
    return align_up(nn_act_layout(batch, D).total_floats * sizeof(float)) + 256;
}

sea_status sea_nn_workspace_bytes(sea_ctx* ctx, int batch, int D, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    sea_status st = nn_check(ctx, batch, D);
    if (st != SEA_OK) return st;
    *bytes = nn_ws_total(batch, D);
    return SEA_OK;
}

sea_status sea_nn_forward(sea_ctx* ctx, const void* state_dev, int batch, int D, const float* x_dev, float* y_dev,
                          void* ws_dev, size_t ws_bytes) {
    if (!ctx) return SEA_E_ARG;
    sea_status st = nn_check(ctx, batch, D);
    if (st != SEA_OK) return st;
    if (!state_dev || !x_dev || !y_dev || !ws_dev) return fail(ctx, SEA_E_ARG, "NULL argument");
    if (ws_bytes < nn_ws_total(batch, D)) return fail(ctx, SEA_E_NOMEM, "workspace too small");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    const NnState ns = nn_state_ptrs(state_dev);
    const NnActLayout L = nn_act_layout(batch, D);
    SEA_HIP_CHECK(ctx, nn_forward(ns.p, ctx->opts.nn_weight_dtype == SEA_BF16 ? ns.p16 : nullptr, x_dev,
                                  (float*)ws_dev, L, batch, D, y_dev, s));
    return SEA_OK;
}

sea_status sea_nn_infer_workspace_bytes(sea_ctx* ctx, int batch, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    if (batch < 1) return fail(ctx, SEA_E_ARG, "batch must be >= 1");
    *bytes = nn_infer_layout(batch).total_bytes;
    return SEA_OK;
}

sea_status sea_nn_infer(sea_ctx* ctx, const void* state_dev, int batch, const float* x_dev, float* y_dev,
                        void* ws_dev, size_t ws_bytes) {
    if (!ctx) return SEA_E_ARG;
    if (batch < 1) return fail(ctx, SEA_E_ARG, "batch must be >= 1");
    if (!state_dev || !x_dev || !y_dev || !ws_dev) return fail(ctx, SEA_E_ARG, "NULL argument");
    if (ws_bytes < nn_infer_layout(batch).total_bytes) return fail(ctx, SEA_E_NOMEM, "workspace too small");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    const NnState ns = nn_state_ptrs(state_dev);
    SEA_HIP_CHECK(ctx, nn_infer(ns.p, ns.p16, x_dev, ws_dev, nn_infer_layout(batch), batch, y_dev, s));
    return SEA_OK;
}

sea_status sea_nn_train_step(sea_ctx* ctx, void* state_dev, int batch, int D, const float* x_dev, const float* t_dev,
                             float lr, int step, void* ws_dev, size_t ws_bytes, double* loss_host, float* grad_dev) {
    if (!ctx) return SEA_E_ARG;
    sea_status st = nn_check(ctx, batch, D);
    if (st != SEA_OK) return st;
    if (!state_dev || !x_dev || !t_dev || !ws_dev) return fail(ctx, SEA_E_ARG, "NULL argument");
    if (step < 1 || !(lr > 0.0f)) return fail(ctx, SEA_E_ARG, "need step >= 1 and lr > 0");
    if (ws_bytes < nn_ws_total(batch, D)) return fail(ctx, SEA_E_NOMEM, "workspace too small");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    const NnState ns = nn_state_ptrs(state_dev);
    const NnActLayout L = nn_act_layout(batch, D);
    float* act = (float*)ws_dev;
    double* loss_dev = (double*)((char*)ws_dev + align_up(L.total_floats * sizeof(float)));
    const uint16_t* w16 = ctx->opts.nn_weight_dtype == SEA_BF16 ? ns.p16 : nullptr;
    const long n = (long)batch * D * D * D;
    SEA_HIP_CHECK(ctx, nn_forward(ns.p, w16, x_dev, act, L, batch, D, nullptr, s));
    float* y = act + L.out[kNnNumLayers - 1];
    float* g = act + L.g2;
    SEA_HIP_CHECK(ctx, nn_mse(y, t_dev, n, g, (double*)(act + L.mse_part), loss_dev, s));
    SEA_HIP_CHECK(ctx, nn_backward(ns.p, w16, x_dev, act, L, batch, D, g, s));
    const long P = (long)nn_param_count();
    if (grad_dev)
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(grad_dev, act + L.grad, P * sizeof(float), hipMemcpyDeviceToDevice, s));
    SEA_HIP_CHECK(ctx, nn_adam(ns.p, ns.p16, ns.m, ns.v, act + L.grad, P, lr, step, s));
    if (loss_host) {
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(loss_host, loss_dev, sizeof(double), hipMemcpyDeviceToHost, s));
        SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
        if (!std::isfinite(*loss_host)) return fail(ctx, SEA_E_NONFINITE, "non-finite loss");
    }
    return SEA_OK;
}

sea_status sea_nn_attach(sea_ctx* ctx, const void* state_dev) {
    if (!ctx) return SEA_E_ARG;
    ctx->nn_state = state_dev;
    return SEA_OK;
}

sea_status sea_solid_harmonics_host(int lmax, double x, double y, double z, double* out) {
    if (lmax < 0 || lmax > SEA_LMAX || !out) return SEA_E_ARG;
    solid_harmonics_orthonormal_host(lmax, x, y, z, out);
    return SEA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// ACE entry points (k_ace.hip provides the kernels)

#include "k_ace.h"

namespace {

struct AceLayout {
    size_t part, mbar, linv, cmat, smat, lam, flag, total;
};

AceLayout ace_layout(long n_grid, int n_occ, int n_vec) {
    AceLayout L{};
    const int nv = n_vec > n_occ ? n_vec : n_occ;
    // split-K partials for every product this workspace serves:
    // (n_occ x n_occ) for M and the energy, (n_occ x n_vec) for K psi
    size_t part_elems = (size_t)ace_mfma_splits(n_grid, n_occ, n_occ) * n_occ * n_occ;
    if (n_vec > 0) {
        const size_t pv = (size_t)ace_mfma_splits(n_grid, n_occ, n_vec) * n_occ * n_vec;
        if (pv > part_elems) part_elems = pv;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    L.part = take(part_elems * sizeof(double));
    L.mbar = take((size_t)n_occ * n_occ * sizeof(double));
    L.linv = take((size_t)n_occ * n_occ * sizeof(double));
    L.cmat = take((size_t)n_occ * nv * sizeof(double));
    L.smat = take((size_t)n_occ * n_occ * sizeof(double));
    L.lam = take((size_t)n_occ * sizeof(double));
    L.flag = take(16 * sizeof(double));
    L.total = off;
    return L;
}

sea_status check_ace(sea_ctx* ctx, long n_grid, int n_occ, double dV, size_t ws_bytes, const AceLayout& Ly,
                     const void* ws) {
    if (n_grid < 1) return fail(ctx, SEA_E_ARG, "n_grid < 1");
    if (n_occ < 1 || n_occ > 4096) return fail(ctx, SEA_E_ARG, "n_occ out of range");
    if (!(dV > 0.0) || !std::isfinite(dV)) return fail(ctx, SEA_E_ARG, "dV must be positive and finite");
    if (!ws) return fail(ctx, SEA_E_ARG, "workspace is NULL");
    if (ws_bytes < Ly.total) return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, Ly.total);
    return SEA_OK;
}

}  // namespace

extern "C" {

sea_status sea_ace_workspace_bytes(sea_ctx* ctx, int64_t n_grid, int n_occ, int n_vec, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    if (n_grid < 1 || n_occ < 1 || n_vec < 0) return fail(ctx, SEA_E_ARG, "bad sizes");
    *bytes = ace_layout(n_grid, n_occ, n_vec).total;
    return SEA_OK;
}

sea_status sea_ace_build(sea_ctx* ctx, int64_t n_grid, int n_occ, double dV, const double* phi_dev,
                         const double* W_dev, void* ws_dev, size_t ws_bytes, double* M_dev, double* L_dev,
                         void* xi_dev, int* failed_pivot) {
    if (!ctx) return SEA_E_ARG;
    const AceLayout Ly = ace_layout(n_grid, n_occ, n_occ);
    sea_status st = check_ace(ctx, n_grid, n_occ, dV, ws_bytes, Ly, ws_dev);
    if (st != SEA_OK) return st;
    if (!phi_dev || !W_dev || !M_dev || !L_dev || !xi_dev) return fail(ctx, SEA_E_ARG, "NULL array argument");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    double* part = (double*)(base + Ly.part);
    double* Mb = (double*)(base + Ly.mbar);
    double* Li = (double*)(base + Ly.linv);
    int* flag = (int*)(base + Ly.flag);
    for (int k = SEA_STAGE_ACE_M; k <= SEA_STAGE_ACE_XI; ++k) ctx->ev_used[k] = false;
    {
        StageTimer t(ctx, SEA_STAGE_ACE_M, s);
        SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F64, double, double>(phi_dev, W_dev, n_occ, n_occ, n_grid, dV, part, M_dev,
                                                               s)));
        SEA_HIP_CHECK(ctx, ace_symmetrize(M_dev, n_occ, Mb, s));
    }
    int hflag = 0;
    bool eigen = ctx->opts.ace_decomp == SEA_DECOMP_EIGEN;
    if (!eigen) {
        {
            StageTimer t(ctx, SEA_STAGE_ACE_CHOL, s);
            SEA_HIP_CHECK(ctx, ace_cholesky(Mb, n_occ, L_dev, flag, s));
        }
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
        SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
        if (failed_pivot) *failed_pivot = hflag;
        if (hflag && ctx->opts.ace_decomp != SEA_DECOMP_AUTO)
            return fail(ctx, SEA_E_NOT_PD, "symmetrized M is not positive definite at pivot %d", hflag);
        eigen = hflag != 0;
    } else if (failed_pivot) {
        *failed_pivot = 0;
    }
    StageTimer t(ctx, SEA_STAGE_ACE_XI, s);
    if (eigen) {
        // App. A: Mbar = Q Lambda Q^T; the xi product takes (Q |Lambda|^{-1/2})^T
        double* lam = (double*)(base + Ly.lam);
        SEA_HIP_CHECK(ctx, ace_eig(Mb, n_occ, L_dev, lam, s));
        SEA_HIP_CHECK(ctx, ace_eig_transform(L_dev, lam, n_occ, Li, s));
        // L_dev <- Q |Lambda|^{-1/2} (transpose of Li)
        SEA_HIP_CHECK(ctx, ace_transpose(Li, n_occ, L_dev, s));
    } else {
        SEA_HIP_CHECK(ctx, ace_trtri(L_dev, n_occ, Li, s));
    }
    // xi (orbital-major) = L^{-1} W
    if (ctx->opts.ace_dtype == SEA_F64)
        SEA_HIP_CHECK(ctx, (ace_mm_nn<ACE_F64, double, double>(Li, n_occ, 1, W_dev, n_occ, n_occ, n_grid, 1.0,
                                                               (double*)xi_dev, s)));
    else if (ctx->opts.ace_dtype == SEA_F32)
        SEA_HIP_CHECK(ctx, (ace_mm_nn<ACE_F32, double, float>(Li, n_occ, 1, W_dev, n_occ, n_occ, n_grid, 1.0,
                                                              (float*)xi_dev, s)));
    else
        SEA_HIP_CHECK(ctx, (ace_mm_nn<ACE_BF16, double, uint16_t>(Li, n_occ, 1, W_dev, n_occ, n_occ, n_grid, 1.0,
                                                                  (uint16_t*)xi_dev, s)));
    if (eigen && ctx->opts.ace_decomp == SEA_DECOMP_AUTO) {
        fail(ctx, SEA_W_EIGEN_FALLBACK, "Mbar not positive definite (pivot %d): eigen decomposition used", hflag);
        return SEA_W_EIGEN_FALLBACK;
    }
    return SEA_OK;
}

sea_status sea_ace_apply(sea_ctx* ctx, int64_t n_grid, int n_occ, double dV, const void* xi_dev, int n_vec,
                         const void* psi_dev, void* ws_dev, size_t ws_bytes, void* out_dev) {
    if (!ctx) return SEA_E_ARG;
    if (n_vec < 1) return fail(ctx, SEA_E_ARG, "n_vec < 1");
    const AceLayout Ly = ace_layout(n_grid, n_occ, n_vec);
    sea_status st = check_ace(ctx, n_grid, n_occ, dV, ws_bytes, Ly, ws_dev);
    if (st != SEA_OK) return st;
    if (!xi_dev || !psi_dev || !out_dev) return fail(ctx, SEA_E_ARG, "NULL array argument");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    double* part = (double*)(base + Ly.part);
    double* Cm = (double*)(base + Ly.cmat);
    ctx->ev_used[SEA_STAGE_ACE_APPLY] = false;
    StageTimer t(ctx, SEA_STAGE_ACE_APPLY, s);
    // C (n_occ x n_vec) = dV xi psi^T ; out (n_vec x n_grid) = -C^T xi
    if (ctx->opts.ace_dtype == SEA_F64) {
        SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F64, double, double>((const double*)xi_dev, (const double*)psi_dev, n_occ,
                                                               n_vec, n_grid, dV, part, Cm, s)));
        SEA_HIP_CHECK(ctx, (ace_mm_nn<ACE_F64, double, double>(Cm, 1, n_vec, (const double*)xi_dev, n_vec, n_occ,
                                                               n_grid, -1.0, (double*)out_dev, s)));
    } else if (ctx->opts.ace_dtype == SEA_F32) {
        SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F32, float, float>((const float*)xi_dev, (const float*)psi_dev, n_occ,
                                                             n_vec, n_grid, dV, part, Cm, s)));
        SEA_HIP_CHECK(ctx, (ace_mm_nn<ACE_F32, float, float>(Cm, 1, n_vec, (const float*)xi_dev, n_vec, n_occ,
                                                             n_grid, -1.0, (float*)out_dev, s)));
    } else {
        SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_BF16, uint16_t, uint16_t>((const uint16_t*)xi_dev,
                                                                    (const uint16_t*)psi_dev, n_occ, n_vec, n_grid,
                                                                    dV, part, Cm, s)));
        SEA_HIP_CHECK(ctx, (ace_mm_nn<ACE_BF16, uint16_t, float>(Cm, 1, n_vec, (const uint16_t*)xi_dev, n_vec,
                                                                 n_occ, n_grid, -1.0, (float*)out_dev, s)));
    }
    return SEA_OK;
}

sea_status sea_ace_energy(sea_ctx* ctx, int64_t n_grid, int n_occ, double dV, const double* phi_dev,
                          const void* xi_dev, void* ws_dev, size_t ws_bytes, double* exx_host) {
    if (!ctx) return SEA_E_ARG;
    const AceLayout Ly = ace_layout(n_grid, n_occ, n_occ);
    sea_status st = check_ace(ctx, n_grid, n_occ, dV, ws_bytes, Ly, ws_dev);
    if (st != SEA_OK) return st;
    if (!phi_dev || !xi_dev || !exx_host) return fail(ctx, SEA_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    double* part = (double*)(base + Ly.part);
    double* S = (double*)(base + Ly.smat);
    double* out = (double*)(base + Ly.flag);
    // FP64 reduction whatever ace_dtype is (xi converts to FP64 exactly)
    if (ctx->opts.ace_dtype == SEA_F64)
        SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F64, double, double>(phi_dev, (const double*)xi_dev, n_occ, n_occ, n_grid,
                                                               dV, part, S, s)));
    else if (ctx->opts.ace_dtype == SEA_F32)
        SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F64, double, float>(phi_dev, (const float*)xi_dev, n_occ, n_occ, n_grid,
                                                              dV, part, S, s)));
    else
        SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F64, double, uint16_t>(phi_dev, (const uint16_t*)xi_dev, n_occ, n_occ,
                                                                 n_grid, dV, part, S, s)));
    SEA_HIP_CHECK(ctx, ace_neg_sum_squares(S, n_occ * n_occ, out, s));
    SEA_HIP_CHECK(ctx, hipMemcpyAsync(exx_host, out, sizeof(double), hipMemcpyDeviceToHost, s));
    SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    if (!std::isfinite(*exx_host)) return fail(ctx, SEA_E_NONFINITE, "non-finite ACE energy");
    return SEA_OK;
}

sea_status sea_successive_idempotency(sea_ctx* ctx, int64_t n_grid, int n_occ, double dV, const double* phi_new_dev,
                                      const double* phi_old_dev, void* ws_dev, size_t ws_bytes, double* dI_host) {
    if (!ctx) return SEA_E_ARG;
    const AceLayout Ly = ace_layout(n_grid, n_occ, n_occ);
    sea_status st = check_ace(ctx, n_grid, n_occ, dV, ws_bytes, Ly, ws_dev);
    if (st != SEA_OK) return st;
    if (!phi_new_dev || !phi_old_dev || !dI_host) return fail(ctx, SEA_E_ARG, "NULL argument");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    double* part = (double*)(base + Ly.part);
    double* S = (double*)(base + Ly.smat);
    double* out = (double*)(base + Ly.flag);
    SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F64, double, double>(phi_new_dev, phi_old_dev, n_occ, n_occ, n_grid, dV, part,
                                                           S, s)));
    SEA_HIP_CHECK(ctx, ace_neg_sum_squares(S, n_occ * n_occ, out, s));
    double neg = 0.0;
    SEA_HIP_CHECK(ctx, hipMemcpyAsync(&neg, out, sizeof(double), hipMemcpyDeviceToHost, s));
    SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    *dI_host = 1.0 + neg / n_occ;
    if (!std::isfinite(*dI_host)) return fail(ctx, SEA_E_NONFINITE, "non-finite idempotency change");
    return SEA_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// SCDM localization (Eq. 1-6) and the rotations of Eq. 6 and Eq. 15

#include "k_scdm.h"
#include <utility>

namespace {

struct ScdmFull {
    ScdmLayout piv;          // pivot search (k_scdm.hip)
    size_t G, P, Ya, Yb, err, part, total;
};

ScdmFull scdm_full_layout(long Ng, int n) {
    ScdmFull L{};
    L.piv = scdm_layout(Ng, n);
    size_t off = L.piv.total;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    const size_t nn = (size_t)n * n * sizeof(double);
    L.G = take(nn);
    L.P = take(nn);
    L.Ya = take(nn);
    L.Yb = take(nn);
    L.err = take(64);
    L.part = take((size_t)ace_mfma_splits(n, n, n) * nn);
    L.total = off;
    return L;
}

sea_status check_rot(sea_ctx* ctx, int64_t n_grid, int n_occ, sea_dtype dt) {
    if (n_occ < 1 || n_occ > SC_NMAX) return fail(ctx, SEA_E_ARG, "n_occ must be in [1, %d]", SC_NMAX);
    if (n_grid < n_occ) return fail(ctx, SEA_E_ARG, "n_grid < n_occ: Phi^T cannot have full row rank");
    if (n_grid > 0x7fffffffLL) return fail(ctx, SEA_E_ARG, "n_grid beyond 2^31 - 1");
    if (dt != SEA_F64 && dt != SEA_F32) return fail(ctx, SEA_E_ARG, "orbitals must be F64 or F32");
    return SEA_OK;
}

// Y = A X with A(r, c) = U[r*sr + c*sc] (n x n) and X, Y orbital-major.
hipError_t rotate_rows(const double* U, long sr, long sc, sea_dtype dt, int n, long Ng, const void* X, void* Y,
                       hipStream_t s) {
    if (dt == SEA_F64)
        return ace_mm_nn<ACE_F64, double, double>(U, sr, sc, (const double*)X, n, n, Ng, 1.0, (double*)Y, s);
    return ace_mm_nn<ACE_F32, float, float>(U, sr, sc, (const float*)X, n, n, Ng, 1.0, (float*)Y, s);
}

}  // namespace

extern "C" sea_status sea_scdm_workspace_bytes(sea_ctx* ctx, int64_t n_grid, int n_occ, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    sea_status st = check_rot(ctx, n_grid, n_occ, SEA_F64);
    if (st != SEA_OK) return st;
    *bytes = scdm_full_layout(n_grid, n_occ).total;
    return SEA_OK;
}

extern "C" sea_status sea_scdm(sea_ctx* ctx, int64_t n_grid, int n_occ, const void* phi_dev, sea_dtype phi_dtype,
                               void* ws_dev, size_t ws_bytes, double* U_dev, void* phi_loc_dev, int32_t* piv_host,
                               double* rdiag_host, int* rounds_host) {
    if (!ctx) return SEA_E_ARG;
    sea_status st = check_rot(ctx, n_grid, n_occ, phi_dtype);
    if (st != SEA_OK) return st;
    if (!phi_dev || !U_dev || !ws_dev) return fail(ctx, SEA_E_ARG, "NULL array argument");
    const ScdmFull L = scdm_full_layout(n_grid, n_occ);
    if (ws_bytes < L.total) return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    if (phi_loc_dev) {
        const size_t es = phi_dtype == SEA_F64 ? 8 : 4;
        const char *a = (const char*)phi_dev, *b = (const char*)phi_loc_dev;
        const size_t len = (size_t)n_grid * n_occ * es;
        if (a < b + len && b < a + len) return fail(ctx, SEA_E_ARG, "phi_loc_dev overlaps phi_dev");
    }
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* ws = (char*)ws_dev;
    const int f32 = phi_dtype == SEA_F32;
    const int n = n_occ;
    const long Ng = (long)n_grid;
    ctx->ev_used[SEA_STAGE_SCDM] = false;
    ctx->ev_used[SEA_STAGE_ROTATE] = false;
    int k = 0, fl = 0, rounds = 0;
    {
        StageTimer t(ctx, SEA_STAGE_SCDM, s);
        // Eq. 1: pivots, one pass over Phi^T per round
        SEA_HIP_CHECK(ctx, scdm_init(phi_dev, f32, Ng, n, ws, L.piv, s));
        int k0 = 0;
        for (;;) {
            SEA_HIP_CHECK(ctx, scdm_round(phi_dev, f32, Ng, n, rounds == 0, ws, L.piv, s));
            SEA_HIP_CHECK(ctx, scdm_read_state(ws, L.piv, &k, &fl, s));
            ++rounds;
            if (fl) break;
            if (k >= n) break;
            if (k <= k0 || k - k0 > SC_RB)
                return fail(ctx, SEA_E_HIP, "SCDM round made no progress (pivots %d -> %d)", k0, k);
            SEA_HIP_CHECK(ctx, scdm_update(phi_dev, f32, Ng, n, k0, k - k0, ws, L.piv, s));
            k0 = k;
        }
        if (fl)
            return fail(ctx, SEA_E_RANK, "Phi^T is rank deficient: no independent column left at pivot %d", fl);
        // Eq. 3-5: U = B P_CC^{-1/2} with P_CC = B^T B is the orthogonal polar
        // factor of B = (Phi^T)_{:,C}.  It is computed by the Newton-Schulz
        // iteration X <- X (3 I - X^T X) / 2 from X = B / |B|_F (every singular
        // value in (0, 1], each step moving it towards 1; quadratic near 1),
        // on the matrix cores, carried as Y = X^T with G = B^T (about 16 steps
        // for condition numbers near 20; 120 allow for 1e12).
        const int* piv = (const int*)(ws + L.piv.piv);
        double* G = (double*)(ws + L.G);
        double* P = (double*)(ws + L.P);
        double* part = (double*)(ws + L.part);
        SEA_HIP_CHECK(ctx, scdm_pivot_rows(phi_dev, f32, Ng, n, piv, G, s));
        double* cur = (double*)(ws + L.Ya);
        double* nxt = (double*)(ws + L.Yb);
        double* errd = (double*)(ws + L.err);
        SEA_HIP_CHECK(ctx, scdm_ns_scale(G, n, cur, s));
        bool conv = false;
        for (int it = 0; it < 120 && !conv; ++it) {
            SEA_HIP_CHECK(ctx, (ace_mm_nt<ACE_F64, double, double>(cur, cur, n, n, n, 1.0, part, P, s)));
            SEA_HIP_CHECK(ctx, scdm_ns_mid(P, n, errd, s));
            SEA_HIP_CHECK(ctx, (ace_mm_nn<ACE_F64, double, double>(P, n, 1, cur, n, n, n, 1.0, nxt, s)));
            std::swap(cur, nxt);
            if (it % 4 == 3) {
                double e = 0.0;
                SEA_HIP_CHECK(ctx, hipMemcpyAsync(&e, errd, sizeof(double), hipMemcpyDeviceToHost, s));
                SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
                conv = e <= 1e-24;   // |X^T X - I|_F <= 1e-12 before the last step
            }
        }
        if (!conv)
            return fail(ctx, SEA_E_RANK, "B = (Phi^T)_{:,C} too ill-conditioned: its polar factor did not converge");
        SEA_HIP_CHECK(ctx, ace_transpose(cur, n, U_dev, s));
    }
    if (phi_loc_dev) {
        StageTimer t(ctx, SEA_STAGE_ROTATE, s);
        // Eq. 6: phi_loc_k = sum_j phi_j U_jk
        SEA_HIP_CHECK(ctx, rotate_rows(U_dev, 1, n, phi_dtype, n, Ng, phi_dev, phi_loc_dev, s));
    }
    if (piv_host)
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(piv_host, ws + L.piv.piv, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, s));
    if (rdiag_host)
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(rdiag_host, ws + L.piv.rdiag, (size_t)n * sizeof(double),
                                          hipMemcpyDeviceToHost, s));
    if (piv_host || rdiag_host) SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    if (rounds_host) *rounds_host = rounds;
    return SEA_OK;
}

extern "C" sea_status sea_rotate(sea_ctx* ctx, int64_t n_grid, int n_occ, sea_dtype dtype, const double* U_dev,
                                 int inverse, const void* X_dev, void* Y_dev) {
    if (!ctx) return SEA_E_ARG;
    sea_status st = check_rot(ctx, n_grid, n_occ, dtype);
    if (st != SEA_OK) return st;
    if (!U_dev || !X_dev || !Y_dev) return fail(ctx, SEA_E_ARG, "NULL array argument");
    if (inverse != 0 && inverse != 1) return fail(ctx, SEA_E_ARG, "inverse must be 0 or 1");
    const size_t len = (size_t)n_grid * n_occ * (dtype == SEA_F64 ? 8 : 4);
    const char *a = (const char*)X_dev, *b = (const char*)Y_dev;
    if (a < b + len && b < a + len) return fail(ctx, SEA_E_ARG, "Y_dev overlaps X_dev");
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    ctx->ev_used[SEA_STAGE_ROTATE] = false;
    StageTimer t(ctx, SEA_STAGE_ROTATE, s);
    const int n = n_occ;
    // inverse: Y_i = sum_j U_ij X_j (U^{-1} = U^T); forward: Y_k = sum_j U_jk X_j
    SEA_HIP_CHECK(ctx, inverse ? rotate_rows(U_dev, n, 1, dtype, n, n_grid, X_dev, Y_dev, s)
                               : rotate_rows(U_dev, 1, n, dtype, n, n_grid, X_dev, Y_dev, s));
    return SEA_OK;
}

// ---------------------------------------------------------------------------
// epsilon-driven domains and pair screening (Eq. 16-17)

extern "C" sea_status sea_eps_workspace_bytes(sea_ctx* ctx, const sea_grid* grid, int n_occ, size_t* bytes) {
    if (!ctx || !bytes) return SEA_E_ARG;
    sea_status st = check_grid(ctx, grid);
    if (st != SEA_OK) return st;
    if (n_occ < 1) return fail(ctx, SEA_E_ARG, "n_occ < 1");
    const int nmax = std::max(grid->n[0], std::max(grid->n[1], grid->n[2]));
    const size_t np = (size_t)n_occ * (n_occ + 1) / 2;
    *bytes = align_up((size_t)n_occ * 3 * nmax * sizeof(double)) + align_up(np * sizeof(sea_pair)) +
             align_up(np * sizeof(double));
    return SEA_OK;
}

extern "C" sea_status sea_build_pairs_eps(sea_ctx* ctx, const sea_grid* grid, int n_occ, const void* phi_dev,
                                          sea_dtype phi_dtype, double eps, double delta, int pad, void* ws_dev,
                                          size_t ws_bytes, sea_pair* out, double* s_out, int32_t* dbox_out, int cap,
                                          int* n_out) {
    if (!ctx) return SEA_E_ARG;
    size_t need = 0;
    sea_status st = sea_eps_workspace_bytes(ctx, grid, n_occ, &need);
    if (st != SEA_OK) return st;
    if (!phi_dev || !ws_dev || !n_out || (cap > 0 && !out)) return fail(ctx, SEA_E_ARG, "NULL argument");
    if (phi_dtype != SEA_F64 && phi_dtype != SEA_F32) return fail(ctx, SEA_E_ARG, "phi_dtype must be F64 or F32");
    if (!(eps >= 0.0 && eps < 1.0)) return fail(ctx, SEA_E_ARG, "eps must be in [0, 1)");
    if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(ctx, SEA_E_ARG, "delta must be >= 0");
    if (pad < 0) return fail(ctx, SEA_E_ARG, "pad must be >= 0");
    if (ws_bytes < need) return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, need);
    const int N[3] = {grid->n[0], grid->n[1], grid->n[2]};
    double h[3];
    for (int a = 0; a < 3; ++a) h[a] = grid->L[a] / N[a];
    const double dV = h[0] * h[1] * h[2];
    const int nmax = std::max(N[0], std::max(N[1], N[2]));
    const size_t np_max = (size_t)n_occ * (n_occ + 1) / 2;
    char* base = (char*)ws_dev;
    double* m_dev = (double*)base;
    sea_pair* cand_dev = (sea_pair*)(base + align_up((size_t)n_occ * 3 * nmax * sizeof(double)));
    double* S_dev = (double*)((char*)cand_dev + align_up(np_max * sizeof(sea_pair)));
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    const int f32 = phi_dtype == SEA_F32;
    // 1. per-orbital, per-axis marginals of |phi|^2; boxes on the host
    SEA_HIP_CHECK(ctx, launch_eps_marginals(phi_dev, f32, N, n_occ, nmax, m_dev, s));
    std::vector<double> m((size_t)n_occ * 3 * nmax);
    SEA_HIP_CHECK(ctx, hipMemcpyAsync(m.data(), m_dev, m.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    std::vector<int> lo((size_t)n_occ * 3), ln((size_t)n_occ * 3);
    for (int o = 0; o < n_occ; ++o)
        for (int a = 0; a < 3; ++a)
            eps_run(&m[((size_t)o * 3 + a) * nmax], N[a], eps, &lo[3 * o + a], &ln[3 * o + a]);
    // 2. candidate pairs: non-empty box intersection on every axis
    std::vector<sea_pair> cand;
    for (int i = 0; i < n_occ; ++i)
        for (int j = i; j < n_occ; ++j) {
            sea_pair p{};
            p.i = i;
            p.j = j;
            bool empty = false;
            for (int a = 0; a < 3 && !empty; ++a) {
                int st0 = 0;
                p.n[a] = cyc_intersect(lo[3 * i + a], ln[3 * i + a], lo[3 * j + a], ln[3 * j + a], N[a], &st0);
                p.lo[a] = st0;
                p.origin[a] = (st0 + 0.5 * (p.n[a] - 1)) * h[a];
                empty = p.n[a] == 0;
            }
            if (!empty) cand.push_back(p);
        }
    // 3. absolute overlaps on the device, screening on the host
    std::vector<double> S(cand.size());
    if (!cand.empty()) {
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(cand_dev, cand.data(), cand.size() * sizeof(sea_pair),
                                          hipMemcpyHostToDevice, s));
        SEA_HIP_CHECK(ctx, launch_eps_overlap(phi_dev, f32, N, dV, cand_dev, (int)cand.size(), S_dev, s));
        SEA_HIP_CHECK(ctx, hipMemcpyAsync(S.data(), S_dev, S.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        SEA_HIP_CHECK(ctx, hipStreamSynchronize(s));
    }
    int cnt = 0;
    for (size_t k = 0; k < cand.size(); ++k) {
        if (!(S[k] >= delta)) continue;
        if (cnt < cap) {
            sea_pair p = cand[k];
            for (int a = 0; a < 3; ++a) {  // solve box: Omega_ij grown by pad points a side, at most the cell
                const int np = std::min(p.n[a] + 2 * pad, N[a]);
                p.lo[a] -= (np - p.n[a]) / 2;
                p.n[a] = np;
                p.origin[a] = (p.lo[a] + 0.5 * (p.n[a] - 1)) * h[a];
            }
            out[cnt] = p;
            if (s_out) s_out[cnt] = S[k];
            if (dbox_out) {
                // W_i: box of phi_j, or Omega_ii doubled about its centre for a self
                // pair; W_j: box of phi_i; both in the frame of the pair's domain and
                // grown to cover it
                const int i = p.i, j = p.j;
                int32_t* d = dbox_out + 12 * (size_t)cnt;
                for (int a = 0; a < 3; ++a) {
                    int l0, n0;
                    if (i == j) {
                        n0 = std::min(2 * ln[3 * i + a], N[a]);
                        l0 = lo[3 * i + a] - (n0 - ln[3 * i + a]) / 2;
                    } else {
                        n0 = ln[3 * j + a];
                        l0 = lo[3 * j + a];
                    }
                    d[a] = near_start(l0, n0, p.lo[a], p.n[a], N[a]);
                    d[3 + a] = n0;
                    d[6 + a] = near_start(lo[3 * i + a], ln[3 * i + a], p.lo[a], p.n[a], N[a]);
                    d[9 + a] = ln[3 * i + a];
                    for (int sd = 0; sd < 2; ++sd) {  // cover the pair's domain too (at most the cell)
                        const int l1 = std::min(d[6 * sd + a], p.lo[a]);
                        const int e1 = std::max(d[6 * sd + a] + d[6 * sd + 3 + a], p.lo[a] + p.n[a]);
                        d[6 * sd + a] = l1;
                        d[6 * sd + 3 + a] = std::min(e1 - l1, N[a]);
                    }
                }
            }
        }
        ++cnt;
    }
    *n_out = cnt;
    if (cnt > cap) return fail(ctx, SEA_E_NOMEM, "pair capacity %d < %d pairs", cap, cnt);
    return SEA_OK;
}

// ---------------------------------------------------------------------------
// autotuner of the FP32-state CG kernel

extern "C" int sea_cg_variant_count(void) { return cg_variant_count(); }
extern "C" const char* sea_cg_variant_name(int v) { return cg_variant_name(v); }

extern "C" int sea_spectral_variant_count(void) { return dst_variant_count(); }

extern "C" const char* sea_spectral_variant_name(int v) { return dst_variant_name(v); }

extern "C" sea_status sea_set_residual_history(sea_ctx* ctx, double* hist_dev, int len) {
    if (!ctx) return SEA_E_ARG;
    if (hist_dev && len < 0) return fail(ctx, SEA_E_ARG, "residual history length %d < 0", len);
    ctx->hist = len >= 0 ? hist_dev : nullptr;
    ctx->hist_len = ctx->hist ? len : 0;
    return SEA_OK;
}

extern "C" int sea_scatter_variant_count(void) { return scatter_variant_count(); }

extern "C" const char* sea_scatter_variant_name(int v) { return scatter_variant_name(v); }

extern "C" sea_status sea_set_scatter_variant(sea_ctx* ctx, int variant) {
    if (!ctx) return SEA_E_ARG;
    if (variant < -1 || variant >= scatter_variant_count())
        return fail(ctx, SEA_E_ARG, "scatter variant %d out of range (%d variants)", variant, scatter_variant_count());
    ctx->scatter_fixed = variant;
    return SEA_OK;
}

extern "C" sea_status sea_set_spectral_variants(sea_ctx* ctx, int plane, int zline) {
    if (!ctx) return SEA_E_ARG;
    const int np = dst_plane_variant_count(), nzv = dst_variant_count() - np;
    if (plane < -1 || plane >= np || zline < -1 || zline >= nzv)
        return fail(ctx, SEA_E_ARG, "spectral variants out of range (plane %d of %d, z line %d of %d)", plane, np,
                    zline, nzv);
    ctx->dst_plane_fixed = plane;
    ctx->dst_zline_fixed = zline;
    return SEA_OK;
}

// Strided sample of `sample_pairs` pairs of the cells, kept per cell (the
// autotuners time their kernels on it).
static void sample_cells(int n_cells, const sea_cell* cells, int sample_pairs, std::vector<std::vector<sea_pair>>& keep,
                         std::vector<sea_cell>& sc) {
    long total = 0;
    for (int c = 0; c < n_cells; ++c) total += cells[c].n_pairs > 0 ? cells[c].n_pairs : 0;
    const long step = total > sample_pairs ? (total + sample_pairs - 1) / sample_pairs : 1;
    keep.assign(n_cells, {});
    sc.assign(cells, cells + n_cells);
    long g = 0;
    for (int c = 0; c < n_cells; ++c) {
        for (int k = 0; k < cells[c].n_pairs; ++k, ++g)
            if (g % step == 0 && cells[c].pairs_host) keep[c].push_back(cells[c].pairs_host[k]);
        sc[c].n_pairs = (int)keep[c].size();
        sc[c].pairs_host = keep[c].data();
    }
}

extern "C" sea_status sea_spectral_autotune(sea_ctx* ctx, int n_cells, const sea_cell* cells, void* ws_dev,
                                            size_t ws_bytes, int sample_pairs, float* ms_host, int* best_plane,
                                            int* best_zline) {
    if (!ctx) return SEA_E_ARG;
    if (!ws_dev) return fail(ctx, SEA_E_ARG, "workspace is NULL");
    if (sample_pairs < 1) return fail(ctx, SEA_E_ARG, "need sample_pairs >= 1");
    if (n_cells < 1 || !cells) return fail(ctx, SEA_E_ARG, "need n_cells >= 1 and a cell array");
    std::vector<std::vector<sea_pair>> keep;
    std::vector<sea_cell> sc;
    sample_cells(n_cells, cells, sample_pairs, keep, sc);
    CellSet S;
    sea_status st = build_cellset(ctx, n_cells, sc.data(), false, S);
    if (st != SEA_OK) return st;
    if (S.pairs.empty()) return fail(ctx, SEA_E_ARG, "no pairs to tune on");
    const sea_opts saved = ctx->opts;
    ctx->opts.start = SEA_START_SPECTRAL;   // the layout with the transform's arrays
    const ExxLayout Ly = exx_layout(ctx, S, true);
    ctx->opts = saved;
    if (ws_bytes < Ly.total) return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, Ly.total);
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    st = exx_upload(ctx, S, Ly, base, s);
    if (st != SEA_OK) return st;
    const ExxArgs a = exx_args(ctx, S, Ly, base, nullptr);
    double* tab = (double*)(base + Ly.dst_tab);
    double* mu = (double*)(base + Ly.dst_mu);
    double* tmp = (double*)(base + Ly.dst_tmp);
    SEA_HIP_CHECK(ctx, launch_gather_moments(a, s));   // b of the sampled pairs: the passes' input
    SEA_HIP_CHECK(ctx, launch_dst_tables(tab, mu, s));
    hipEvent_t e0, e1;
    SEA_HIP_CHECK(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, SEA_E_HIP, "event creation failed");
    }
    const int np = dst_plane_variant_count(), nv = dst_variant_count();
    int bp = 0, bz = 0;
    float tp = 0.0f, tz = 0.0f;
    hipError_t err = hipSuccess;
    for (int v = 0; v < nv && err == hipSuccess; ++v) {
        const bool plane = v < np;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {   // rep 0 warms the code object
            err = hipEventRecord(e0, s);
            if (err == hipSuccess)
                err = plane ? launch_dst_pass(a, 0, v, S.dst_shape, a.b, tmp, tab, mu, s)
                            : launch_dst_pass(a, 1, v - np, S.dst_shape, tmp, a.bres, tab, mu, s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        }
        if (ms_host) ms_host[v] = ms;
        if (plane && (v == 0 || ms < tp)) {
            tp = ms;
            bp = v;
        }
        if (!plane && (v == np || ms < tz)) {
            tz = ms;
            bz = v - np;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(ctx, SEA_E_HIP, "spectral autotune: %s", hipGetErrorString(err));
    ctx->dst_plane_tuned = bp;
    ctx->dst_zline_tuned = bz;
    if (best_plane) *best_plane = bp;
    if (best_zline) *best_zline = bz;
    return SEA_OK;
}

extern "C" sea_status sea_scatter_autotune(sea_ctx* ctx, int n_cells, const sea_cell* cells, void* ws_dev,
                                           size_t ws_bytes, float* ms_host, int* best) {
    if (!ctx) return SEA_E_ARG;
    if (!ws_dev) return fail(ctx, SEA_E_ARG, "workspace is NULL");
    if (n_cells < 1 || !cells) return fail(ctx, SEA_E_ARG, "need n_cells >= 1 and a cell array");
    CellSet S;
    sea_status st = build_cellset(ctx, n_cells, cells, true, S);   // (the scatter writes W)
    if (st != SEA_OK) return st;
    if (S.pairs.empty()) return fail(ctx, SEA_E_ARG, "no pairs to tune on");
    const ExxLayout Ly = exx_layout(ctx, S, true);
    if (ws_bytes < Ly.total) return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, Ly.total);
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    st = exx_upload(ctx, S, Ly, base, s);
    if (st != SEA_OK) return st;
    ExxArgs a = exx_args(ctx, S, Ly, base, nullptr);
    // pair potentials of zero (the scatter's time does not depend on them),
    // and the pair energies' partials when the action takes them there
    SEA_HIP_CHECK(ctx, hipMemsetAsync(a.v, 0, sizeof(double) * a.stride * S.pairs.size(), s));
    bool lists_fit = true;
    for (size_t k = 0; k + 1 < S.csr_off.size(); ++k) lists_fit = lists_fit && S.csr_off[k + 1] - S.csr_off[k] <= SC_EP_MAXE;
    if (lists_fit) a.epart = (double*)(base + Ly.epart);
    hipEvent_t e0, e1;
    SEA_HIP_CHECK(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, SEA_E_HIP, "event creation failed");
    }
    const int nv = scatter_variant_count();
    int arg = 0;
    float tbest = 0.0f;
    hipError_t err = hipSuccess;
    for (int v = 0; v < nv && err == hipSuccess; ++v) {
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {   // rep 0 warms the code object
            err = hipEventRecord(e0, s);
            if (err == hipSuccess && a.epart) err = launch_epart_clear(a, s);
            for (size_t c = 0; c < S.cells.size() && err == hipSuccess; ++c)
                err = launch_scatter(a, S.dev[c], (const int*)(base + Ly.csr_off), (const int2*)(base + Ly.csr_ent), v,
                                     s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        }
        if (ms_host) ms_host[v] = ms;
        if (v == 0 || ms < tbest) {
            tbest = ms;
            arg = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(ctx, SEA_E_HIP, "scatter autotune: %s", hipGetErrorString(err));
    ctx->scatter_tuned = arg;
    if (best) *best = arg;
    return SEA_OK;
}

extern "C" sea_status sea_exx_autotune(sea_ctx* ctx, int n_cells, const sea_cell* cells, void* ws_dev,
                                       size_t ws_bytes, int sample_pairs, int iters, float* ms_host, int* best) {
    if (!ctx) return SEA_E_ARG;
    if (!ws_dev) return fail(ctx, SEA_E_ARG, "workspace is NULL");
    if (sample_pairs < 1 || iters < 1) return fail(ctx, SEA_E_ARG, "need sample_pairs >= 1 and iters >= 1");
    if (n_cells < 1 || !cells) return fail(ctx, SEA_E_ARG, "need n_cells >= 1 and a cell array");
    // strided sample of all pairs, kept per cell
    long total = 0;
    for (int c = 0; c < n_cells; ++c) total += cells[c].n_pairs > 0 ? cells[c].n_pairs : 0;
    if (total < 1) return fail(ctx, SEA_E_ARG, "no pairs to tune on");
    const long step = total > sample_pairs ? (total + sample_pairs - 1) / sample_pairs : 1;
    std::vector<std::vector<sea_pair>> keep(n_cells);
    std::vector<sea_cell> sc(cells, cells + n_cells);
    long g = 0;
    for (int c = 0; c < n_cells; ++c) {
        for (int k = 0; k < cells[c].n_pairs; ++k, ++g)
            if (g % step == 0 && cells[c].pairs_host) keep[c].push_back(cells[c].pairs_host[k]);
        sc[c].n_pairs = (int)keep[c].size();
        sc[c].pairs_host = keep[c].data();
    }
    CellSet S;
    sea_status st = build_cellset(ctx, n_cells, sc.data(), false, S);
    if (st != SEA_OK) return st;
    if (!S.cubic || !cg_zm_fits(S.pairs.data(), (int)S.pairs.size(), nullptr) || cg_zm_lds_bytes(1) > ctx->max_lds)
        return fail(ctx, SEA_E_ARG, "the FP32 state needs cubic grids and pair domains with n[0], n[1] <= 64");
    sea_opts saved = ctx->opts;
    ctx->opts.start = SEA_START_ZERO;
    const ExxLayout Ly = exx_layout(ctx, S, true);
    if (ws_bytes < Ly.total) {
        ctx->opts = saved;
        return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, Ly.total);
    }
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    char* base = (char*)ws_dev;
    st = exx_upload(ctx, S, Ly, base, s);
    ExxArgs a = exx_args(ctx, S, Ly, base, nullptr);
    ctx->opts = saved;
    if (st != SEA_OK) return st;
    a.max_iter = iters;
    a.rel_tol = 1e-300;  // never met: every pair runs exactly `iters` iterations
    int nz_max = 1;
    for (const auto& p : S.pairs) nz_max = p.n[2] > nz_max ? p.n[2] : nz_max;
    SEA_HIP_CHECK(ctx, launch_gather_moments(a, s));
    SEA_HIP_CHECK(ctx, launch_moments_final(a, nullptr, s));
    SEA_HIP_CHECK(ctx, launch_boundary_fold(a, nz_max, s));
    hipEvent_t e0, e1;
    SEA_HIP_CHECK(ctx, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, SEA_E_HIP, "event creation failed");
    }
    const int nv = cg_variant_count();
    int arg = 0;
    float tbest = 0.0f;
    hipError_t err = hipSuccess;
    for (int v = 0; v < nv && err == hipSuccess; ++v) {
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {  // rep 0 warms the code object
            err = launch_moments_final(a, nullptr, s);            // resets the pair queue
            if (err == hipSuccess) err = hipEventRecord(e0, s);
            if (err == hipSuccess) err = launch_cg_zm(a, v, s);
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        }
        if (ms_host) ms_host[v] = ms;
        if (v == 0 || ms < tbest) {
            tbest = ms;
            arg = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(ctx, SEA_E_HIP, "autotune: %s", hipGetErrorString(err));
    ctx->cg_tuned = arg;
    if (best) *best = arg;
    return SEA_OK;
}

// ---------------------------------------------------------------------------
// plans: tables uploaded once, kernel sequence captured into a HIP graph

struct sea_plan {
    sea_ctx* ctx = nullptr;
    CellSet S;
    ExxLayout Ly{};
    char* base = nullptr;
    ExxArgs a{};
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipStream_t last = nullptr;
};

extern "C" {

sea_status sea_exx_plan_create(sea_ctx* ctx, int n_cells, const sea_cell* cells, void* ws_dev, size_t ws_bytes,
                               sea_plan** out) {
    if (!ctx || !out) return SEA_E_ARG;
    *out = nullptr;
    if (!ws_dev) return fail(ctx, SEA_E_ARG, "workspace is NULL");
    if (ctx->opts.start == SEA_START_LEARNED && !ctx->nn_state)
        return fail(ctx, SEA_E_ARG, "SEA_START_LEARNED needs a network (sea_nn_attach)");
    sea_plan* P = new (std::nothrow) sea_plan();
    if (!P) return SEA_E_NOMEM;
    P->ctx = ctx;
    sea_status st = build_cellset(ctx, n_cells, cells, true, P->S);
    if (st != SEA_OK) { delete P; return st; }
    P->Ly = exx_layout(ctx, P->S, true, false);
    if (ws_bytes < P->Ly.total) {
        delete P;
        return fail(ctx, SEA_E_NOMEM, "workspace too small: %zu < %zu bytes", ws_bytes, P->Ly.total);
    }
    P->base = (char*)ws_dev;
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    st = exx_upload(ctx, P->S, P->Ly, P->base, s);
    if (st != SEA_OK) { delete P; return st; }
    P->a = exx_args(ctx, P->S, P->Ly, P->base, nullptr);
    if (hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess) {
        delete P;
        return fail(ctx, SEA_E_HIP, "stream creation failed");
    }
    ExxFlags f;  // action, no profiling inside a graph
    if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipStreamDestroy(P->cap);
        delete P;
        return fail(ctx, SEA_E_HIP, "graph capture could not start");
    }
    st = exx_enqueue(ctx, P->S, P->Ly, P->base, P->a, f, P->cap);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(P->cap, &g);
    if (st != SEA_OK || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(P->cap);
        delete P;
        return st != SEA_OK ? st : fail(ctx, SEA_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    }
    P->graph = g;
    e = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(P->cap);
        delete P;
        return fail(ctx, SEA_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    *out = P;
    return SEA_OK;
}

sea_status sea_exx_plan_launch(sea_plan* P, void* hip_stream) {
    if (!P) return SEA_E_ARG;
    hipStream_t s = (hipStream_t)hip_stream;
    SEA_HIP_CHECK(P->ctx, hipGraphLaunch(P->exec, s));
    P->last = s;
    return SEA_OK;
}

sea_status sea_exx_plan_results(sea_plan* P, double* exx_host, sea_pair_stat* stats_host) {
    if (!P) return SEA_E_ARG;
    return exx_results(P->ctx, P->S, P->Ly, P->base, P->last, exx_host, stats_host);
}

sea_status sea_exx_plan_destroy(sea_plan* P) {
    if (!P) return SEA_OK;
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->cap) (void)hipStreamDestroy(P->cap);
    delete P;
    return SEA_OK;
}

}  // extern "C"
