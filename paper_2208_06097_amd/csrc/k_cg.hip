// CG Poisson solves (Eq. 9) on the pair domains, one workgroup per pair,
// persistent over a pair queue.
//
// Each workgroup owns a whole pair: the domain (nx, ny <= 64) is marched
// plane by plane in z.  A wavefront covers one x-row of 64 points; every
// thread owns COLS (x, y) columns and keeps the 13 values p(z-6..z+6) of
// each column in registers.  x neighbours come from wavefront DPP shifts
// (zero fill at the wave edge is the zero boundary), y neighbours from the
// current plane in LDS (rows of 64 with 6 zero halo rows each side).  One
// LDS barrier per plane (double-buffered plane); no halo re-reads from HBM.
//
// One CG iteration is two sweeps (8 words of state traffic per point):
//   A: p = r + beta p (in place), d = <p, A p>           reads r, p; writes p
//   B: c += alpha p, r -= alpha A p, rr = <r, r>          reads p, c, r; writes c, r
// where A p is recomputed in B instead of being stored.  A start guess
// enters as the first FP64 residual update, so no separate start-residual
// pass is needed.
//
// Paired iterate updates (XC variants, 7 words per iteration on average):
// c is read and written only every second sweep B.  Iteration k-1 leaves
// its step alpha_{k-1} p_{k-1} pending; sweep B of iteration k adds both
// steps at once, recovering p_{k-1} = (p_k - r_k) / beta_{k-1} from the p_k
// and r_k it reads anyway:
//   c += (alpha_{k-1} / beta_{k-1} + alpha_k) p_k - (alpha_{k-1} / beta_{k-1}) r_k.
// When beta_{k-1} is small (the recovery would amplify rounding) the
// pending step is added to c before sweep A of iteration k, while p still
// holds p_{k-1}, and before a residual refresh likewise.  Any
// rounding in c is caught by the FP64 refresh, which recomputes the
// residual from x.
//
// Precision: the CG state (c, r, p) is T (double or float), with reliable
// updates (residual replacement, as in mixed-precision CG of Sleijpen and
// van der Vorst): the FP64 residual r64 starts at b; whenever the recursive
// residual has dropped by another decade (FP32 state) or has met the target,
// one more sweep applies r64 -= A c with FP64 arithmetic and x += c in FP64,
// and the recursive residual is replaced by (T) r64 while the search
// direction p is kept, so the Krylov process is never restarted.  Residual
// norms and dot products accumulate in FP64.  A separate kernel recomputes
// the true residual b - A x in FP64 at exit and the pair energy.
#include <type_traits>

#include "sea_internal.h"

namespace {

__constant__ double kCw[7] = {-5369.0 / 1800.0, 12.0 / 7.0,      -15.0 / 56.0,     10.0 / 189.0,
                              -1.0 / 112.0,     2.0 / 1925.0,    -1.0 / 16632.0};

constexpr int LW = 64;                 // LDS row length (x)
constexpr int LH = 64 + 2 * SEA_HALO;  // LDS rows per plane (y with halo)
constexpr int PL = 64 * 64;            // slot-array plane pitch (elements)

// Cubic grid: -Lap_h f = w0 f + sum_k wk (six neighbours at distance k).
template <typename T>
struct SW {
    T w[7];
};

template <typename T>
__device__ __forceinline__ SW<T> make_sw(double ih2) {
    SW<T> w;
#pragma unroll
    for (int k = 0; k < 7; ++k) w.w[k] = (T)(-kCw[k] * ih2 * (k == 0 ? 3.0 : 1.0));
    return w;
}


// Wavefront shifts by one lane with zero fill at the edge (DPP wave_shl:1 /
// wave_shr:1).  The stencil only uses sums f(x+k) + f(x-k), so it does not
// depend on which of the two is the left shift.
__device__ __forceinline__ float wshl1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float wshr1(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ double wshl1(double v) {
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __builtin_amdgcn_update_dpp(0, t.x, 0x130, 0xF, 0xF, true);
    t.y = __builtin_amdgcn_update_dpp(0, t.y, 0x130, 0xF, 0xF, true);
    return *reinterpret_cast<double*>(&t);
}
__device__ __forceinline__ double wshr1(double v) {
    int2 t = *reinterpret_cast<int2*>(&v);
    t.x = __builtin_amdgcn_update_dpp(0, t.x, 0x138, 0xF, 0xF, true);
    t.y = __builtin_amdgcn_update_dpp(0, t.y, 0x138, 0xF, 0xF, true);
    return *reinterpret_cast<double*>(&t);
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    if (wid == 0) {
        double t = (lane < NT / 64) ? lds[lane] : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) lds[NT / 64] = t;
    }
    __syncthreads();
    const double r = lds[NT / 64];
    __syncthreads();
    return r;
}

// residual history entry t of pair pid (a.hist set, t <= a.hist_len)
__device__ __forceinline__ void hist_put(const ExxArgs& a, int pid, int t, double r2, double b2) {
    if (a.hist && t <= a.hist_len) a.hist[(size_t)pid * (a.hist_len + 1) + t] = b2 > 0.0 ? sqrt(r2 / b2) : 0.0;
}

__device__ __forceinline__ int wrap_idx(int k, int N) {
    int m = k % N;
    return m < 0 ? m + N : m;
}

__device__ __forceinline__ double load_phi(const void* phi, int f32, size_t off) {
    typedef __attribute__((address_space(1))) const float gfloat;
    typedef __attribute__((address_space(1))) const double gdouble;
    return f32 ? (double)((gfloat*)phi)[off] : ((gdouble*)phi)[off];
}

struct Empty {};

// z-march of A applied to a field f.  The input of plane z is produced in
// two steps so its global loads overlap plane work: fetch(c, z) issues the
// loads DEPTH steps before plane z enters the register queue, make(c, z, F)
// turns them into f when it does (DEPTH = 1: loads issued at the start of
// the step that consumes them; DEPTH = 2: one step earlier, twice the bytes
// in flight for more registers).  pre(c, z) prefetches per-column data for
// the output plane z before the barrier; out(c, z, A f, f, PV) consumes it.
// Column c of this thread is (x, y) = (tx, ty + TY c).  Plane nz of every
// slot array is zero and every fetch beyond the domain reads it (it stays in
// cache), so the march never moves padding through HBM.
template <typename T, typename TC, int NT, int COLS, int DEPTH, typename F, typename PV, typename FetchF,
          typename MakeF, typename PreF, typename OutF>
__device__ __forceinline__ void zmarch(int nz, T* lds, const SW<TC>& w, FetchF&& fetch, MakeF&& make, PreF&& pre,
                                       OutF&& out) {
    static_assert(DEPTH == 1 || DEPTH == 2, "prefetch depth");
    constexpr int TY = NT / 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    T q[COLS][13];
#pragma unroll
    for (int c = 0; c < COLS; ++c) {
#pragma unroll
        for (int k = 0; k < 6; ++k) q[c][k] = T(0);
#pragma unroll
        for (int s = 0; s < 7; ++s) q[c][6 + s] = make(c, s, fetch(c, min(s, nz)));
    }
    F nb[COLS];
    if constexpr (DEPTH == 2) {
#pragma unroll
        for (int c = 0; c < COLS; ++c) nb[c] = fetch(c, min(7, nz));
    }
    for (int z = 0; z < nz; ++z) {
        F nxt[COLS];
        if constexpr (DEPTH == 1) {
#pragma unroll
            for (int c = 0; c < COLS; ++c) nxt[c] = fetch(c, min(z + 7, nz));
        } else {
#pragma unroll
            for (int c = 0; c < COLS; ++c) {
                nxt[c] = nb[c];
                nb[c] = fetch(c, min(z + 8, nz));
            }
        }
        PV pv[COLS];
#pragma unroll
        for (int c = 0; c < COLS; ++c) pv[c] = pre(c, z);
        T* pl = lds + (z & 1) * (LW * LH) + (ty + SEA_HALO) * LW + tx;
#pragma unroll
        for (int c = 0; c < COLS; ++c) pl[TY * c * LW] = q[c][6];
        lds_sync();
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
            __builtin_amdgcn_sched_barrier(0);
            const T* row = pl + TY * c * LW;
            TC s = w.w[0] * (TC)q[c][6];
            T u = q[c][6], d = q[c][6];
#pragma unroll
            for (int k = 1; k <= SEA_HALO; ++k) {
                u = wshl1(u);
                d = wshr1(d);
                s += w.w[k] * (((TC)u + (TC)d) + ((TC)row[k * LW] + (TC)row[-k * LW]) +
                               ((TC)q[c][6 + k] + (TC)q[c][6 - k]));
            }
            out(c, z, s, q[c][6], pv[c]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int c = 0; c < COLS; ++c) {
#pragma unroll
            for (int k = 0; k < 12; ++k) q[c][k] = q[c][k + 1];
            q[c][12] = make(c, z + 7, nxt[c]);
        }
    }
}

// -Lap_h x at interior point (x,y,z) read straight from global memory (zero
// outside the interior); used for the FP64 outer residual only.
__device__ __forceinline__ double apply_A_global(const double* __restrict__ p, int id, int x, int y, int z, int nx,
                                                 int ny, int nz, double ih2) {
    const int sy = nx, sz = nx * ny;
    double s = -3.0 * kCw[0] * ih2 * p[id];
#pragma unroll
    for (int k = 1; k <= SEA_HALO; ++k) {
        const double ax = (x - k >= 0 ? p[id - k] : 0.0) + (x + k < nx ? p[id + k] : 0.0);
        const double ay = (y - k >= 0 ? p[id - k * sy] : 0.0) + (y + k < ny ? p[id + k * sy] : 0.0);
        const double az = (z - k >= 0 ? p[id - k * sz] : 0.0) + (z + k < nz ? p[id + k * sz] : 0.0);
        s += -kCw[k] * ih2 * (ax + ay + az);
    }
    return s;
}

// FP32 z-march: the reliable-update trigger replaces the recursive residual
// by the FP64 one whenever it has dropped by another factor Delta (squared
// here).
//
// Exit target: the FP64 residual must reach `target` x rel_tol.  FP32 state
// loses the Galerkin orthogonality of CG, which makes the pair energies'
// error first order in the residual with a larger constant; at 0.3 x rel_tol
// the FP32 form's E_xx error matches the FP64 form's at rel_tol (64-molecule
// cell: |dE| 1.6e-7 Ha vs 6e-8 Ha; 1.1e-6 Ha at 1.0 x rel_tol) for about 4%
// more iterations.
template <typename T>
struct Delta;
template <>
struct Delta<float> {
    static constexpr double v2 = 1e-2;
    static constexpr double target = 0.3;
};

template <typename T>
struct F2 {
    T a, b;
};
template <typename T>
struct PVsel {
    using type = F2<T>;
};

// Whether a pair's start meets the exit test |b - A x|^2 <= tol2 |b|^2,
// from the residual sweep's norms per row tile, summed in a fixed order (the
// residual kernel's second launch and the CG take the same decision).
__device__ __forceinline__ bool start_meets_target(const ExxArgs& a, int pid, double tol2, double& b2, double& q2) {
    b2 = 0.0;
    q2 = 0.0;
    for (int t = 0; t < RZ_TILES; ++t) {
        b2 += a.rnorm[((size_t)pid * RZ_TILES + t) * 2];
        q2 += a.rnorm[((size_t)pid * RZ_TILES + t) * 2 + 1];
    }
    return q2 == q2 && b2 == b2 && q2 <= tol2 * b2;
}

// Access to one slot array at element col0 + off, off uniform across the
// workgroup (plane and column offsets).  BUF: raw buffer instructions with
// the array in a buffer resource (scalar registers), the lane's column in
// one 32-bit VGPR and the uniform offset in a scalar register, so the state
// arrays cost no 64-bit address registers; otherwise plain global pointers.
template <typename T, bool BUF>
struct SlotIO;
template <typename T>
struct SlotIO<T, false> {
    T* p;
    __device__ SlotIO(T* base, int, int col0) : p(base + col0) {}
    __device__ __forceinline__ T ld(int off) const { return p[off]; }
    __device__ __forceinline__ void st(int off, T v) const { p[off] = v; }
};
template <>
struct SlotIO<float, true> {
    __amdgpu_buffer_rsrc_t rs;
    int voff;
    __device__ SlotIO(float* base, int n_elems, int col0)
        : rs(__builtin_amdgcn_make_buffer_rsrc(base, 0, n_elems * (int)sizeof(float), 0x00020000)),
          voff(col0 * (int)sizeof(float)) {}
    __device__ __forceinline__ float ld(int off) const {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, voff, off * (int)sizeof(float), 0));
    }
    __device__ __forceinline__ void st(int off, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, voff, off * (int)sizeof(float), 0);
    }
};

template <typename T, int NT, int COLS, bool PREFETCH, int DEPTH, bool BUF, bool XC>
__device__ void solve_pair(const ExxArgs& a, int pid, T* lds, double* red, T* __restrict__ cc, T* __restrict__ rr,
                           T* __restrict__ pp, double* __restrict__ r64) {
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const double ih2 = 1.0 / (C.h[0] * C.h[0]);
    const SW<T> w = make_sw<T>(ih2);
    const SW<double> wd = make_sw<double>(ih2);
    // Slot arrays (cc, rr, pp, r64) use a padded 64 x 64 plane: element
    // (x,y,z) at (z*64 + y)*64 + x, planes 0..nz; cells outside the domain
    // (including all of plane nz) stay zero in cc, rr, pp and r64.
    constexpr int TY = NT / 64;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int npad = PL * (nz + 1);
    const double* __restrict__ b = a.b + (size_t)pid * a.stride;
    double* __restrict__ x = a.v + (size_t)pid * a.stride;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const double tol2 = Delta<T>::target * Delta<T>::target * a.rel_tol * a.rel_tol;
    T msk[COLS];
#pragma unroll
    for (int c = 0; c < COLS; ++c) msk[c] = (tx < nx && ty + TY * c < ny) ? T(1) : T(0);
    const int col0 = ty * 64 + tx;  // column c at col0 + c*TY*64 within a plane
    const SlotIO<T, BUF> io_c(cc, npad, col0), io_r(rr, npad, col0), io_p(pp, npad, col0);

    // step alpha p of the previous iteration not yet added to c (XC)
    T pend = T(0);
    // c += pend p over the padded grid (the p array holds the pending step's
    // direction when this runs)
    auto flush = [&]() {
        for (int q = threadIdx.x; q < npad; q += NT) cc[q] += pend * pp[q];
        pend = T(0);
        __syncthreads();
    };

    // FP64 residual update: r64 -= A c and x += c, one z-march; returns |r64|^2
    auto refresh = [&]() -> double {
        double uacc = 0.0;
        if (XC && pend != T(0)) flush();
        zmarch<T, double, NT, COLS, 1, T, double>(
            nz, lds, wd, [&](int c, int z) -> T { return io_c.ld(z * PL + c * TY * 64); },
            [&](int, int, T v) -> T { return v; },
            [&](int c, int z) -> double { return r64[z * PL + col0 + c * TY * 64]; },
            [&](int c, int z, double s, T ctr, double rv) {
                const int id = z * PL + col0 + c * TY * 64;
                const double rn = (double)msk[c] * (rv - s);
                r64[id] = rn;
                uacc += rn * rn;
                if (msk[c] != T(0)) x[(z * ny + ty + TY * c) * nx + tx] += (double)ctr;
            });
        return block_sum<NT>(uacc, red);
    };

    // r64 = b on the padded grid, x = 0.  A start guess x0 (in x on entry)
    // enters as the first increment c = (T) x0, so that x and r64 = b - A x
    // stay consistent in FP64 from the start.  With start_res the start is
    // kept in FP64 in x and r64 = b - A x comes precomputed in bres; with
    // rnorm too, the norms of the residual sweep decide first whether the
    // start already meets the target (bres is then not written).
    const bool sres = a.x_nonzero && a.start_res;
    const bool fold = a.x_nonzero && !a.start_res;
    if (sres && a.rnorm) {
        double b2, q2;
        if (start_meets_target(a, pid, tol2, b2, q2)) {
            if (threadIdx.x == 0) {
                a.stats[pid].iters = 0;
                a.stats[pid].converged = 1;
                a.stats[pid].rel_res = b2 > 0.0 ? sqrt(q2 / b2) : 0.0;
                hist_put(a, pid, 0, q2, b2);
            }
            return;
        }
    }
    const double* __restrict__ br = sres ? a.bres + (size_t)pid * a.stride : nullptr;
    double bb = 0.0, r2 = 0.0;
    for (int q = threadIdx.x; q < npad; q += NT) {
        const int xx = q & 63, yy = (q >> 6) & 63, zz = q >> 12;
        double rv = 0.0;
        T c0 = T(0);
        if (xx < nx && yy < ny && zz < nz) {
            const int id = (zz * ny + yy) * nx + xx;
            const double bv = b[id];
            bb += bv * bv;
            rv = sres ? br[id] : bv;
            if (fold) c0 = (T)x[id];
            if (!sres) x[id] = 0.0;
        }
        r64[q] = rv;
        if (fold) cc[q] = c0;
        r2 += rv * rv;
    }
    bb = block_sum<NT>(bb, red);
    r2 = block_sum<NT>(r2, red);
    if (fold) r2 = refresh();

    int it = 0, conv = 0;
    // inner state from r64: r = (T) r64, c = 0 (p is kept across replacements)
    auto reset = [&](bool zero_p) -> double {
        double r2t = 0.0;
        for (int q = threadIdx.x; q < npad; q += NT) {
            const T rt = (T)r64[q];
            rr[q] = rt;
            cc[q] = T(0);
            if (zero_p) pp[q] = T(0);
            r2t += (double)rt * (double)rt;
        }
        return block_sum<NT>(r2t, red);
    };
    double rho = 0.0, rupd = r2;
    T beta = T(0);
    if (threadIdx.x == 0) hist_put(a, pid, 0, r2, bb);
    if (!(r2 == r2) || !(bb == bb)) conv = -1;
    else if (r2 <= tol2 * bb) conv = 1;
    else if (a.max_iter <= 0) conv = 0;
    else rho = reset(true);
    while (conv == 0 && rho > 0.0) {
        // XC: a pending step whose recovery would need a small beta is
        // written now, while p still holds its direction
        if (XC && pend != T(0) && !((double)beta >= a.xc_beta_min)) flush();
        // sweep A: p = r + beta p, <p, A p>
        double dacc = 0.0;
        zmarch<T, T, NT, COLS, DEPTH, F2<T>, Empty>(
            nz, lds, w,
            [&](int c, int z) -> F2<T> {
                const int o = z * PL + c * TY * 64;
                return F2<T>{io_r.ld(o), io_p.ld(o)};
            },
            [&](int c, int z, F2<T> f) -> T {
                const T pn = f.a + beta * f.b;
                // beyond the domain pn = 0 (r and p read the zero plane):
                // the store lands on plane nz, which stays zero
                io_p.st(min(z, nz) * PL + c * TY * 64, pn);
                return pn;
            },
            [&](int, int) { return Empty{}; },
            [&](int, int, T s, T ctr, Empty) { dacc += (double)ctr * (double)s; });
        const double pAp = block_sum<NT>(dacc, red);
        const T al = (T)(rho / pAp);
        // coefficients of this sweep's update c += cp p + cr r (XC: none when
        // this step is left pending)
        const bool with_c = !XC || pend != T(0);
        const T cp = XC ? (pend != T(0) ? pend / beta + al : T(0)) : al;
        const T cr = XC && pend != T(0) ? -(pend / beta) : T(0);
        // sweep B: c += alpha p, r -= alpha A p, <r, r>
        using PV = typename PVsel<T>::type;
        double racc = 0.0;
        auto fetch_p = [&](int c, int z) -> T { return io_p.ld(z * PL + c * TY * 64); };
        auto make_p = [&](int, int, T v) -> T { return v; };
        if constexpr (PREFETCH) {
            zmarch<T, T, NT, COLS, DEPTH, T, PV>(
                nz, lds, w, fetch_p, make_p,
                [&](int c, int z) -> PV {
                    const int o = z * PL + c * TY * 64;
                    return PV{with_c ? io_c.ld(o) : T(0), io_r.ld(o)};
                },
                [&](int c, int z, T s, T ctr, PV v) {
                    const int o = z * PL + c * TY * 64;
                    const T rn = msk[c] * (v.b - al * s);
                    if (with_c) {
                        if constexpr (XC) io_c.st(o, v.a + cp * ctr + cr * v.b);
                        else io_c.st(o, v.a + al * ctr);
                    }
                    io_r.st(o, rn);
                    racc += (double)rn * (double)rn;
                });
        } else {
            zmarch<T, T, NT, COLS, DEPTH, T, Empty>(
                nz, lds, w, fetch_p, make_p, [&](int, int) { return Empty{}; },
                [&](int c, int z, T s, T ctr, Empty) {
                    const int o = z * PL + c * TY * 64;
                    const T rv = io_r.ld(o);
                    const T rn = msk[c] * (rv - al * s);
                    if (with_c) {
                        if constexpr (XC) io_c.st(o, io_c.ld(o) + cp * ctr + cr * rv);
                        else io_c.st(o, io_c.ld(o) + al * ctr);
                    }
                    io_r.st(o, rn);
                    racc += (double)rn * (double)rn;
                });
        }
        const double rn2 = block_sum<NT>(racc, red);
        if constexpr (XC) pend = with_c ? T(0) : al;
        ++it;
        if (threadIdx.x == 0) hist_put(a, pid, it, rn2, bb);
        const bool nan = !(rn2 == rn2);
        if (!nan && rn2 > tol2 * bb && rn2 > Delta<T>::v2 * rupd && it < a.max_iter) {
            beta = (T)(rn2 / rho);
            rho = rn2;
            continue;
        }
        // reliable update in FP64: r64 -= A c, x += c
        r2 = refresh();
        if (!(r2 == r2)) { conv = -1; break; }
        if (r2 <= tol2 * bb) { conv = 1; break; }
        if (it >= a.max_iter) break;
        // continue the same Krylov process from the replaced residual
        const double r2t = reset(false);
        beta = (T)(r2t / rho);
        rho = r2t;
        rupd = r2;
    }
    // r64 = b - A x up to the FP64 rounding of the increments: it is the
    // residual reported for this pair
    if (threadIdx.x == 0) {
        a.stats[pid].iters = it;
        a.stats[pid].converged = conv;
        a.stats[pid].rel_res = bb > 0.0 ? sqrt(r2 / bb) : 0.0;
    }
}

template <typename T, int NT, int COLS, bool PREFETCH, int DEPTH, bool BUF, bool XC>
__global__ __launch_bounds__(NT) void k_cg_zm(ExxArgs a) {
    extern __shared__ unsigned char smem[];
    T* lds = reinterpret_cast<T*>(smem);
    __shared__ double red[NT / 64 + 1];
    __shared__ int pid_sh;
    for (int i = threadIdx.x; i < 2 * LW * LH; i += NT) lds[i] = T(0);
    char* slot = reinterpret_cast<char*>(a.slots) + (size_t)blockIdx.x * 4 * a.slot_stride * sizeof(double);
    T* cc = reinterpret_cast<T*>(slot);
    T* rr = cc + a.slot_stride;
    T* pp = rr + a.slot_stride;
    double* r64 = reinterpret_cast<double*>(slot + 3 * a.slot_stride * sizeof(double));
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) pid_sh = atomicAdd(a.queue_ctr, 1);
        __syncthreads();
        const int qi = pid_sh;
        if (qi >= a.n_pairs) break;
        const int pid = a.order ? a.order[qi] : qi;  // largest domains first
        solve_pair<T, NT, COLS, PREFETCH, DEPTH, BUF, XC>(a, pid, lds, red, cc, rr, pp, r64);
    }
}

// Pair energy e_ij = dV sum rho x and the final flags, one workgroup per pair.
// With a.epart (after the scatter) a pair whose W box of orbital i holds its
// domain once has its energy from the scatter's partials, summed here in
// slot order; the others (and every pair without a.epart) sum rho x over
// the domain here.
constexpr int FIN_BS = 512;

__global__ __launch_bounds__(FIN_BS) void k_cg_finish(ExxArgs a) {
    __shared__ double red[FIN_BS / 64 + 1];
    const int pid = blockIdx.x;
    const DevCell C = a.cells[a.pair_cell[pid]];   // copied: fields stay in registers
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int n = nx * ny * nz;
    const double* x = a.v + (size_t)pid * a.stride;
    const size_t oi = (size_t)P.i * C.Ng, oj = (size_t)P.j * C.Ng;
    double e = 0.0;
    if (a.epart && ep_takes(P, a.dbox + 12 * (size_t)pid, C.N)) {
        const int ns = ep_slots(P, C.N);
        const double* ep = a.epart + (size_t)pid * a.ep_stride;
        for (int k = threadIdx.x; k < ns; k += FIN_BS) e += ep[k];
    } else {
        BoxWalk wk((int)threadIdx.x, FIN_BS, nx, ny);
        // FIN_U points per thread at a time, their loads issued together; one
        // copy per orbital precision, widened at the product.  The sum runs in
        // the same order as one point at a time.
        constexpr int FIN_U = 4;
        auto run = [&](auto f32) {
            using PT = typename std::conditional<decltype(f32)::value, float, double>::type;
            typedef __attribute__((address_space(1))) const PT gPT;
            const gPT* ph = (const gPT*)C.phi;
            for (int id0 = threadIdx.x; id0 < n; id0 += FIN_U * FIN_BS) {
                PT fi[FIN_U], fj[FIN_U];
                double xv[FIN_U];
#pragma unroll
                for (int k = 0; k < FIN_U; ++k) {
                    // past n the walk leaves the box along z, still a grid point
                    // after wrapping; x is then read at the box's last point
                    const size_t g = ((size_t)wrap_near(P.lo[2] + wk.z, C.N[2]) * C.N[1] + wrap_near(P.lo[1] + wk.y, C.N[1])) *
                                         C.N[0] +
                                     wrap_near(P.lo[0] + wk.x, C.N[0]);
                    fi[k] = ph[oi + g];
                    fj[k] = ph[oj + g];
                    xv[k] = x[min(id0 + k * FIN_BS, n - 1)];
                    wk.next();
                }
#pragma unroll
                for (int k = 0; k < FIN_U; ++k)
                    if (id0 + k * FIN_BS < n) e += (double)fi[k] * (double)fj[k] * xv[k];
            }
        };
        if (C.phi_f32) run(std::true_type());
        else run(std::false_type());
    }
    e = block_sum<FIN_BS>(e, red);
    if (threadIdx.x == 0) {
        DevStat st = a.stats[pid];
        if (st.converged >= 0) st.converged = (st.rel_res <= a.rel_tol) ? 1 : 0;
        if (!(st.rel_res == st.rel_res) || !(e == e)) st.converged = -1;
        st.e_ij = C.dV * e;
        st.s_abs = a.mom[(size_t)pid * SEA_NACC + SEA_NMOM];
        st.q = a.mom[(size_t)pid * SEA_NACC + SEA_NMOM + 1];
        a.stats[pid] = st;
    }
}

}  // namespace

bool cg_zm_fits(const sea_pair* pairs, int n_pairs, const double* h) {
    if (h && (h[0] != h[1] || h[0] != h[2])) return false;
    for (int k = 0; k < n_pairs; ++k)
        if (pairs[k].n[0] > 64 || pairs[k].n[1] > 64) return false;
    return true;
}

size_t cg_zm_lds_bytes(int state_f32) { return (size_t)2 * LW * LH * (state_f32 ? sizeof(float) : sizeof(double)); }

// b - A x0 for a start guess x0 (FP64), one workgroup per pair.
__global__ __launch_bounds__(FIN_BS) void k_start_residual(ExxArgs a) {
    const int pid = blockIdx.x;
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int n = nx * ny * nz, nxy = nx * ny;
    const double ih2 = 1.0 / (C.h[0] * C.h[0]);
    const double* b = a.b + (size_t)pid * a.stride;
    const double* x = a.v + (size_t)pid * a.stride;
    double* br = a.bres + (size_t)pid * a.stride;
    for (int id = threadIdx.x; id < n; id += FIN_BS) {
        const int xx = id % nx, yy = (id / nx) % ny, zz = id / nxy;
        br[id] = b[id] - apply_A_global(x, id, xx, yy, zz, nx, ny, nz, ih2);
    }
}

// b - A x in FP64 for every pair of a cubic grid with nx, ny <= 64, by the
// row-tile march below.  Two launches: NORMS writes |b|^2 and |b - A x|^2 of the owned rows into
// a.rnorm[pair][tile][2] and nothing else; WRITE stores b - A x into bres
// for the pairs whose start does not meet the CG's exit test (from those
// norms; the others return at once), so a start that is already converged
// costs one read of x and b.
// Workgroups are numbered so that the row tiles of one pair run together
// on one XCD (workgroup k goes to XCD k mod 8): the rows a tile fetches
// again for its neighbours' window are then served by the same L2.
constexpr int RZ_NT = 1024;
constexpr int RZ_ROWS = 16;   // rows owned per workgroup: one per wavefront
constexpr int RZ_WR = RZ_ROWS + 2 * SEA_HALO;   // rows of the window
constexpr int RZ_XCD = 8;
#ifndef SEA_RZ_PRE
#define SEA_RZ_PRE 2
#endif
#ifndef SEA_RZ_DEPTH
#define SEA_RZ_DEPTH 2
#endif
#ifndef SEA_CG64_DEPTH
#define SEA_CG64_DEPTH 1
#endif
constexpr int RZ_PRE = SEA_RZ_PRE;           // steps ahead that the owned point's data is loaded
constexpr int RZ_DEPTH = SEA_RZ_DEPTH;       // steps ahead that the residual sweep fetches x
constexpr int CG64_DEPTH = SEA_CG64_DEPTH;   // the same for the CG sweeps
static_assert(RZ_TILES * RZ_ROWS >= 64, "row tiles cover 64 rows");
static_assert(RZ_NT / 64 == RZ_ROWS, "a wavefront per owned row");

__device__ __forceinline__ void rz_block(int& pid, int& tile) {
    const int k = blockIdx.x, m = k / RZ_XCD;
    pid = (m / RZ_TILES) * RZ_XCD + k % RZ_XCD;
    tile = m % RZ_TILES;
}

// Row-tile z-march of A applied to a field f (FP64).  A workgroup owns
// RZ_ROWS rows (y) of one pair, a wavefront per row and a lane per x, and
// marches z over a window of RZ_WR rows (SEA_HALO more on each side, which
// the neighbouring workgroups own).  Only the owned rows keep the 13-plane
// register queue and form the stencil; wavefronts ty < 2 SEA_HALO also load
// one halo row's current plane into LDS for the y taps (window row ty below
// the tile, ty + RZ_ROWS above it; with fewer owned rows than halo rows a
// wavefront takes two).  fetch(yw, z) issues the loads of window
// row yw at plane z, DEPTH steps before they are used (measured: the
// residual sweep, with one plane of output loads, runs faster at DEPTH 2;
// the CG sweeps, with two, at DEPTH 1), make(yw, z, F) turns them into f,
// pre(z) loads the owned point's data of output plane z (z < nz), PRE steps
// before out(z, A f, f, PV) consumes it (issued with the step's other loads,
// so that its latency is not paid at the step's end).  Two LDS planes of
// RZ_WR x 64 doubles.
template <int DEPTH, int PRE, typename F, typename PV, typename FetchF, typename MakeF, typename PreF, typename OutF>
__device__ __forceinline__ void rtmarch(int nz, double* lds, const SW<double>& w, FetchF&& fetch, MakeF&& make,
                                        PreF&& pre, OutF&& out) {
    static_assert(DEPTH >= 1 && DEPTH <= 4, "prefetch depth");
    static_assert(PRE >= 0 && PRE <= 4, "output data prefetch depth");
    constexpr int HR = 2 * SEA_HALO;                           // halo rows of the window
    constexpr int HPW = (HR + RZ_ROWS - 1) / RZ_ROWS;           // halo rows per wavefront (at most)
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int yo = ty + SEA_HALO;                               // owned row in the window
    // halo row h = ty + RZ_ROWS e (h < HR) sits at window row h below the
    // tile and h + RZ_ROWS above it
    auto hrow = [&](int e) { const int h = ty + RZ_ROWS * e; return h < SEA_HALO ? h : h + RZ_ROWS; };
    auto has_h = [&](int e) { return ty + RZ_ROWS * e < HR; };
    double q[13];
#pragma unroll
    for (int k = 0; k < 6; ++k) q[k] = 0.0;
#pragma unroll
    for (int s = 0; s < 7; ++s) q[6 + s] = make(yo, s, fetch(yo, min(s, nz)));
    // the owned row's plane z + 7 is fetched at step z + 1 - DEPTH (DEPTH 1:
    // in the step that uses it, at its end) and the halo rows' plane z at
    // step z - DEPTH
    F oq[DEPTH > 1 ? DEPTH - 1 : 1];
#pragma unroll
    for (int i = 0; i + 1 < DEPTH; ++i) oq[i] = fetch(yo, min(7 + i, nz));
    F hq[HPW][DEPTH];
#pragma unroll
    for (int e = 0; e < HPW; ++e)
#pragma unroll
        for (int i = 0; i < DEPTH; ++i) hq[e][i] = has_h(e) ? fetch(hrow(e), min(i, nz)) : F{};
    PV pq[PRE > 0 ? PRE : 1];
#pragma unroll
    for (int i = 0; i < PRE; ++i) pq[i] = pre(min(i, nz - 1));
    for (int z = 0; z < nz; ++z) {
        F nxt;
        if constexpr (DEPTH == 1) {
            nxt = fetch(yo, min(z + 7, nz));
        } else {
            nxt = oq[0];
#pragma unroll
            for (int i = 0; i + 2 < DEPTH; ++i) oq[i] = oq[i + 1];
            oq[DEPTH - 2] = fetch(yo, min(z + 6 + DEPTH, nz));
        }
        F hc[HPW];
#pragma unroll
        for (int e = 0; e < HPW; ++e) {
            hc[e] = hq[e][0];
            if (has_h(e)) {
#pragma unroll
                for (int i = 0; i + 1 < DEPTH; ++i) hq[e][i] = hq[e][i + 1];
                hq[e][DEPTH - 1] = fetch(hrow(e), min(z + DEPTH, nz));
            }
        }
        PV pv;
        if constexpr (PRE == 0) {
            pv = pre(z);
        } else {
            pv = pq[0];
#pragma unroll
            for (int i = 0; i + 1 < PRE; ++i) pq[i] = pq[i + 1];
            pq[PRE - 1] = pre(min(z + PRE, nz - 1));   // (past the last plane: the last again, unused)
        }
        double* pl = lds + (z & 1) * (LW * RZ_WR);
        pl[yo * LW + tx] = q[6];
#pragma unroll
        for (int e = 0; e < HPW; ++e)
            if (has_h(e)) pl[hrow(e) * LW + tx] = make(hrow(e), z, hc[e]);
        lds_sync();
        __builtin_amdgcn_sched_barrier(0);
        const double* row = pl + yo * LW + tx;
        double sacc = w.w[0] * q[6];
        double u = q[6], d = q[6];
#pragma unroll
        for (int k = 1; k <= SEA_HALO; ++k) {
            u = wshl1(u);
            d = wshr1(d);
            sacc += w.w[k] * ((u + d) + (row[k * LW] + row[-k * LW]) + (q[6 + k] + q[6 - k]));
        }
        out(z, sacc, q[6], pv);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < 12; ++k) q[k] = q[k + 1];
        q[12] = make(yo, z + 7, nxt);
    }
}

template <bool WRITE>
__global__ __launch_bounds__(RZ_NT) void k_residual_zm(ExxArgs a) {
    extern __shared__ unsigned char smem[];
    double* lds = reinterpret_cast<double*>(smem);
    __shared__ double red[RZ_NT / 64 + 1];
    int pid, tile;
    rz_block(pid, tile);
    if (pid >= a.n_pairs) return;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int y0 = tile * RZ_ROWS;
    // after the row-tile CG: a pair its start stopped keeps the start's norms
    if (!WRITE && a.cg_done && a.cg_done[pid] == 2) return;
    if (WRITE) {
        double b2, q2;
        if (y0 >= ny || start_meets_target(a, pid, Delta<float>::target * Delta<float>::target * a.rel_tol * a.rel_tol,
                                           b2, q2))
            return;
    } else if (y0 >= ny) {
        if (threadIdx.x == 0) {
            a.rnorm[((size_t)pid * RZ_TILES + tile) * 2] = 0.0;
            a.rnorm[((size_t)pid * RZ_TILES + tile) * 2 + 1] = 0.0;
        }
        return;
    }
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const SW<double> w = make_sw<double>(1.0 / (C.h[0] * C.h[0]));
    const double* __restrict__ x = a.v + (size_t)pid * a.stride;
    const double* __restrict__ b = a.b + (size_t)pid * a.stride;
    double* __restrict__ r = a.bres + (size_t)pid * a.stride;
    const int tx = threadIdx.x & 63, yown = y0 + (threadIdx.x >> 6);
    const bool own = yown < ny && tx < nx;
    double bb = 0.0, rr = 0.0;
    rtmarch<RZ_DEPTH, RZ_PRE, double, double>(
        nz, lds, w,
        [&](int yw, int z) -> double {   // window row yw is grid row y0 - SEA_HALO + yw
            const int y = y0 - SEA_HALO + yw;
            return (tx < nx && y >= 0 && y < ny && z < nz) ? x[(z * ny + y) * nx + tx] : 0.0;
        },
        [&](int, int, double v) -> double { return v; },
        [&](int z) -> double { return own ? b[(z * ny + yown) * nx + tx] : 0.0; },
        [&](int z, double s, double, double bv) {
            if (own) {
                const double rv = bv - s;
                if (WRITE) r[(z * ny + yown) * nx + tx] = rv;
                bb += bv * bv;
                rr += rv * rv;
            }
        });
    if (WRITE) return;
    bb = block_sum<RZ_NT>(bb, red);
    rr = block_sum<RZ_NT>(rr, red);
    if (threadIdx.x == 0) {
        a.rnorm[((size_t)pid * RZ_TILES + tile) * 2] = bb;
        a.rnorm[((size_t)pid * RZ_TILES + tile) * 2 + 1] = rr;
    }
}

// ---------------------------------------------------------------------------
// FP64-state CG by row tiles (the plain FP64 form of Eq. 9).  Its 13-plane
// FP64 register queue does not fit a whole pair in one workgroup, so the
// state of every pair (x in v, r and p in their own arrays) stays in HBM
// and every CG sweep is one launch over all pairs and their row tiles (the
// residual sweep's 16 owned rows, 28-row window and XCD mapping).  The
// scalars of a pair come from per-tile partial sums, summed by every tile in
// the same fixed order, so all tiles of a pair take the same decisions:
//   sweep A (iteration k): rho_k = |r|^2; stop if rho_k <= tol^2 |b|^2, at
//     max_iter or on a non-finite value; else beta = rho_k / rho_{k-1}
//     (0 at k = 0), p = r + beta p on the window (the halo rows recomputed,
//     the owned rows written to the other of two p arrays), <p, A p>;
//   sweep B: alpha = rho_k / <p, A p>, x += alpha p, r -= alpha A p, |r|^2.
// The |r|^2 partials alternate between two slots by iteration parity, so a
// sweep never overwrites a partial another tile of its pair still reads.
// The stop test runs on the recursive residual at 0.9 x rel_tol; the true
// FP64 residual b - A x is formed afterwards for the reported rel_res.
// Preconditioned (a.cg_pre, the spectral form's continuation): z = M^-1 r
// with M = A_odd, the stencil with odd continuation past the faces, applied
// exactly by the sine-transform passes between the sweeps; rho = <r, z>
// takes the place of |r|^2 in alpha and beta, p = z + beta p.  M differs
// from A only next to the faces, so few iterations remain.
constexpr double CG64_TARGET = 0.9;
// partial slots per row tile: |r|^2 by parity (0, 1), <p, A p> (2), |b|^2
// (3), <r, z> by parity (4, 5; the preconditioned form's rho)
constexpr int CG64_SLOTS = 8;
__device__ __forceinline__ int cg64_rho_slot(const ExxArgs& a, int k) { return (a.cg_pre ? 4 : 0) + (k & 1); }

__device__ __forceinline__ double cg64_sum(const ExxArgs& a, int pid, int slot) {
    double s = 0.0;
    for (int t = 0; t < RZ_TILES; ++t) s += a.cg_part[((size_t)pid * RZ_TILES + t) * CG64_SLOTS + slot];
    return s;
}

__global__ __launch_bounds__(RZ_NT) void k_cg64_init(ExxArgs a) {
    extern __shared__ unsigned char smem[];
    double* lds = reinterpret_cast<double*>(smem);
    __shared__ double red[RZ_NT / 64 + 1];
    int pid, tile;
    rz_block(pid, tile);
    if (pid >= a.n_pairs) return;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int y0 = tile * RZ_ROWS;
    double* part = a.cg_part + ((size_t)pid * RZ_TILES + tile) * CG64_SLOTS;
    if (a.rnorm) {   // a start whose true residual (its norms) already meets the target stops here
        double b2, q2;
        if (start_meets_target(a, pid, CG64_TARGET * CG64_TARGET * a.rel_tol * a.rel_tol, b2, q2)) {
            if (tile == 0 && threadIdx.x == 0) {
                a.cg_done[pid] = 2;   // stopped by its start: the final norms pass skips it
                a.stats[pid].iters = 0;
                a.stats[pid].converged = 1;
                a.stats[pid].rel_res = b2 > 0.0 ? sqrt(q2 / b2) : 0.0;
                hist_put(a, pid, 0, q2, b2);
            }
            return;
        }
    }
    if (tile == 0 && threadIdx.x == 0) {
        a.cg_done[pid] = 0;
        atomicAdd(a.cg_active + a.max_iter + 1, 1);   // pairs that iterate
    }
    if (y0 >= ny) {
        if (threadIdx.x == 0)
            for (int q = 0; q < CG64_SLOTS; ++q) part[q] = 0.0;
        return;
    }
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const SW<double> w = make_sw<double>(1.0 / (C.h[0] * C.h[0]));
    double* __restrict__ x = a.v + (size_t)pid * a.stride;
    const double* __restrict__ b = a.b + (size_t)pid * a.stride;
    double* __restrict__ r = a.cg_r + (size_t)pid * a.stride;
    double* __restrict__ p = a.cg_p + (size_t)pid * a.stride;   // parity 0: read by sweep A of iteration 0
    const int tx = threadIdx.x & 63, yown = y0 + (threadIdx.x >> 6);
    const bool own = yown < ny && tx < nx;
    const bool x0 = a.x_nonzero;
    double bb = 0.0, rr = 0.0;
    rtmarch<CG64_DEPTH, RZ_PRE, double, double>(
        nz, lds, w,
        [&](int yw, int z) -> double {
            const int y = y0 - SEA_HALO + yw;
            return (x0 && tx < nx && y >= 0 && y < ny && z < nz) ? x[(z * ny + y) * nx + tx] : 0.0;
        },
        [&](int, int, double v) -> double { return v; },
        [&](int z) -> double { return own ? b[(z * ny + yown) * nx + tx] : 0.0; },
        [&](int z, double s, double, double bv) {
            if (own) {
                const int id = (z * ny + yown) * nx + tx;
                const double rv = bv - s;
                r[id] = rv;
                p[id] = rv;
                if (!x0) x[id] = 0.0;
                bb += bv * bv;
                rr += rv * rv;
            }
        });
    bb = block_sum<RZ_NT>(bb, red);
    rr = block_sum<RZ_NT>(rr, red);
    if (threadIdx.x == 0) {
        for (int q = 0; q < CG64_SLOTS; ++q) part[q] = 0.0;
        part[0] = rr;
        part[3] = bb;
    }
}

template <int SWEEP>
__global__ __launch_bounds__(RZ_NT) void k_cg64_sweep(ExxArgs a) {
    extern __shared__ unsigned char smem[];
    double* lds = reinterpret_cast<double*>(smem);
    __shared__ double red[RZ_NT / 64 + 1];
    int pid, tile;
    rz_block(pid, tile);
    if (pid >= a.n_pairs || a.cg_done[pid]) return;
    const int k = a.cg_it;
    const double rho = cg64_sum(a, pid, cg64_rho_slot(a, k));
    if (SWEEP == 0) {
        const double rr = a.cg_pre ? cg64_sum(a, pid, k & 1) : rho;
        const double bb = cg64_sum(a, pid, 3);
        const double tol2 = CG64_TARGET * CG64_TARGET * a.rel_tol * a.rel_tol;
        const bool nan = !(rr == rr) || !(bb == bb) || !(rho == rho);
        if (tile == 0 && threadIdx.x == 0) hist_put(a, pid, k, rr, bb);
        if (nan || rr <= tol2 * bb || k >= a.max_iter) {
            if (tile == 0 && threadIdx.x == 0) {
                a.stats[pid].iters = k;
                a.stats[pid].converged = nan ? -1 : (rr <= tol2 * bb ? 1 : 0);
                a.stats[pid].rel_res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
                a.cg_done[pid] = 1;
            }
            return;
        }
        if (tile == 0 && threadIdx.x == 0) {
            atomicAdd(a.cg_active + k, 1);
            a.cg_rho[(size_t)pid * 2 + (k & 1)] = rho;
        }
    }
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int y0 = tile * RZ_ROWS;
    double* part = a.cg_part + ((size_t)pid * RZ_TILES + tile) * CG64_SLOTS;
    if (y0 >= ny) {
        if (threadIdx.x == 0) part[SWEEP == 0 ? 2 : ((k + 1) & 1)] = 0.0;
        return;
    }
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const SW<double> w = make_sw<double>(1.0 / (C.h[0] * C.h[0]));
    double* __restrict__ x = a.v + (size_t)pid * a.stride;
    double* __restrict__ r = a.cg_r + (size_t)pid * a.stride;
    // p by iteration parity: sweep A of iteration k reads p_k from array
    // k & 1 (every tile reads its window's halo rows there, owned by other
    // tiles) and writes p_{k+1} = r + beta p_k into the other array, which
    // sweep B then reads
    const double* __restrict__ p_in = a.cg_p + ((size_t)(k & 1) * a.n_pairs + pid) * a.stride;
    double* __restrict__ p = a.cg_p + ((size_t)((k + 1) & 1) * a.n_pairs + pid) * a.stride;
    const int tx = threadIdx.x & 63, yown = y0 + (threadIdx.x >> 6);
    const bool own = yown < ny && tx < nx;
    auto inwin = [&](int yw, int z) {   // window row yw is grid row y0 - SEA_HALO + yw
        const int y = y0 - SEA_HALO + yw;
        return tx < nx && y >= 0 && y < ny && z < nz;
    };
    auto widx = [&](int yw, int z) { return (z * ny + y0 - SEA_HALO + yw) * nx + tx; };   // < 64^3: 32-bit
    auto oidx = [&](int z) { return (z * ny + yown) * nx + tx; };
    double acc = 0.0;
    if constexpr (SWEEP == 0) {
        // p = r + beta p (z + beta p when preconditioned) over the window (the
        // halo rows recomputed here, the owned rows written), <p, A p> over
        // the owned rows
        const double beta = k > 0 ? rho / a.cg_rho[(size_t)pid * 2 + ((k - 1) & 1)] : 0.0;
        const double* __restrict__ src = (a.cg_pre ? a.cg_z : a.cg_r) + (size_t)pid * a.stride;
        rtmarch<CG64_DEPTH, 0, F2<double>, Empty>(
            nz, lds, w,
            [&](int yw, int z) -> F2<double> {
                if (!inwin(yw, z)) return F2<double>{0.0, 0.0};
                const int id = widx(yw, z);
                return F2<double>{src[id], p_in[id]};
            },
            [&](int, int, F2<double> f) -> double { return f.a + beta * f.b; },
            [&](int) { return Empty{}; },
            [&](int z, double s, double ctr, Empty) {
                if (own) {
                    p[oidx(z)] = ctr;
                    acc += ctr * s;
                }
            });
        acc = block_sum<RZ_NT>(acc, red);
        if (threadIdx.x == 0) part[2] = acc;
    } else {
        // x += alpha p, r -= alpha A p, |r|^2 over the owned rows
        const double alpha = rho / cg64_sum(a, pid, 2);
        rtmarch<CG64_DEPTH, RZ_PRE, double, F2<double>>(
            nz, lds, w,
            [&](int yw, int z) -> double { return inwin(yw, z) ? p[widx(yw, z)] : 0.0; },
            [&](int, int, double v) -> double { return v; },
            [&](int z) -> F2<double> {
                if (!own) return F2<double>{0.0, 0.0};
                const int id = oidx(z);
                return F2<double>{x[id], r[id]};
            },
            [&](int z, double s, double ctr, F2<double> xr) {
                if (own) {
                    const int id = oidx(z);
                    x[id] = xr.a + alpha * ctr;
                    const double rn = xr.b - alpha * s;
                    r[id] = rn;
                    acc += rn * rn;
                }
            });
        acc = block_sum<RZ_NT>(acc, red);
        if (threadIdx.x == 0) part[(k + 1) & 1] = acc;
    }
}

// The reported residual: the true FP64 one from the residual sweep's norms.
__global__ __launch_bounds__(64) void k_cg64_exit(ExxArgs a) {
    const int pid = blockIdx.x * 64 + threadIdx.x;
    if (pid >= a.n_pairs) return;
    double b2 = 0.0, q2 = 0.0;
    for (int t = 0; t < RZ_TILES; ++t) {
        b2 += a.rnorm[((size_t)pid * RZ_TILES + t) * 2];
        q2 += a.rnorm[((size_t)pid * RZ_TILES + t) * 2 + 1];
    }
    DevStat st = a.stats[pid];
    st.rel_res = b2 > 0.0 ? sqrt(q2 / b2) : 0.0;
    if (!(q2 == q2)) st.converged = -1;
    a.stats[pid] = st;
}

// <r, z> per row tile of the pairs still iterating, into the rho slot of
// iteration a.cg_it + 1 (the preconditioned form; a.cg_it = -1 after the init).
__global__ __launch_bounds__(RZ_NT) void k_cg64_dot(ExxArgs a) {
    __shared__ double red[RZ_NT / 64 + 1];
    int pid, tile;
    rz_block(pid, tile);
    if (pid >= a.n_pairs || a.cg_done[pid]) return;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int y0 = tile * RZ_ROWS, y1 = min(ny, y0 + RZ_ROWS);
    const double* __restrict__ r = a.cg_r + (size_t)pid * a.stride;
    const double* __restrict__ z = a.cg_z + (size_t)pid * a.stride;
    double acc = 0.0;
    const int row = nx, rows = y1 > y0 ? y1 - y0 : 0;
    for (int zz = 0; zz < nz; ++zz)
        for (int q = threadIdx.x; q < rows * row; q += RZ_NT) {
            const int id = (zz * ny + y0) * nx + q;
            acc += r[id] * z[id];
        }
    acc = block_sum<RZ_NT>(acc, red);
    if (threadIdx.x == 0)
        a.cg_part[((size_t)pid * RZ_TILES + tile) * CG64_SLOTS + cg64_rho_slot(a, a.cg_it + 1)] = acc;
}

__global__ __launch_bounds__(256) void k_fill_int(int* p, size_t n) {
    for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) p[k] = 0;
}

size_t residual_zm_lds_bytes() { return (size_t)2 * LW * RZ_WR * sizeof(double); }

hipError_t launch_residual_zm(const ExxArgs& a, hipStream_t s, bool write) {
    if (a.n_pairs <= 0) return hipSuccess;
    const int lds = (int)residual_zm_lds_bytes();
    const unsigned nb = (unsigned)((a.n_pairs + RZ_XCD - 1) / RZ_XCD) * RZ_XCD * RZ_TILES;
    hipError_t e = hipFuncSetAttribute((const void*)k_residual_zm<false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)k_residual_zm<true>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_residual_zm<false>, dim3(nb), dim3(RZ_NT), lds, s, a);
    if (write) hipLaunchKernelGGL(k_residual_zm<true>, dim3(nb), dim3(RZ_NT), lds, s, a);
    return hipGetLastError();
}

static unsigned rz_blocks(int n_pairs) { return (unsigned)((n_pairs + RZ_XCD - 1) / RZ_XCD) * RZ_XCD * RZ_TILES; }

hipError_t launch_cg64_init(const ExxArgs& a, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    const int lds = (int)residual_zm_lds_bytes();
    hipError_t e = hipFuncSetAttribute((const void*)k_cg64_init, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cg64_init, dim3(rz_blocks(a.n_pairs)), dim3(RZ_NT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_cg64_sweep(const ExxArgs& a, int sweep, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    const int lds = (int)residual_zm_lds_bytes();
    const void* fn = sweep == 0 ? (const void*)k_cg64_sweep<0> : (const void*)k_cg64_sweep<1>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    if (sweep == 0) hipLaunchKernelGGL(k_cg64_sweep<0>, dim3(rz_blocks(a.n_pairs)), dim3(RZ_NT), lds, s, a);
    else hipLaunchKernelGGL(k_cg64_sweep<1>, dim3(rz_blocks(a.n_pairs)), dim3(RZ_NT), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_cg64_dot(const ExxArgs& a, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg64_dot, dim3(rz_blocks(a.n_pairs)), dim3(RZ_NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cg64_exit(const ExxArgs& a, hipStream_t s) {
    if (a.n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cg64_exit, dim3((a.n_pairs + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

__global__ void k_fill_nan(double* __restrict__ p, size_t n) {
    const double q = __builtin_nan("");
    for (size_t k = blockIdx.x * (size_t)256 + threadIdx.x; k < n; k += (size_t)gridDim.x * 256) p[k] = q;
}

hipError_t launch_fill_nan(double* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_nan, dim3(nb), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_fill_int(int* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned nb = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_int, dim3(nb), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_start_residual(const ExxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_start_residual, dim3(a.n_pairs), dim3(FIN_BS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cg_finish(const ExxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_finish, dim3(a.n_pairs), dim3(FIN_BS), 0, s, a);
    return hipGetLastError();
}

// Compiled z-march variants (FP32 state); the autotuner picks one per
// workload.  nt: workgroup size (rows of the 64 x 64 plane per thread =
// 4096 / nt; smaller workgroups need more queue registers than the 128 a
// lane may hold at this size and spill in the plane loop); pf: prefetch c
// and r of the output plane before the barrier; d: planes of p in flight
// ahead of the register queue; buf: state arrays through buffer
// instructions (32-bit offsets) instead of 64-bit global addresses; xc:
// paired iterate updates (c read and written every second iteration).
namespace {
using CgKernel = void (*)(ExxArgs);
struct CgVariant {
    const char* name;
    CgKernel fn;
    int nt;
};
const CgVariant kCgVariants[] = {
    {"nt1024-pf-d1", k_cg_zm<float, 1024, 4, true, 1, false, false>, 1024},
    {"nt1024-pf-d2", k_cg_zm<float, 1024, 4, true, 2, false, false>, 1024},
    {"nt1024-d1", k_cg_zm<float, 1024, 4, false, 1, false, false>, 1024},
    {"nt1024-d2", k_cg_zm<float, 1024, 4, false, 2, false, false>, 1024},
    {"buf-pf-d1", k_cg_zm<float, 1024, 4, true, 1, true, false>, 1024},
    {"buf-pf-d2", k_cg_zm<float, 1024, 4, true, 2, true, false>, 1024},
    {"buf-d2", k_cg_zm<float, 1024, 4, false, 2, true, false>, 1024},
    {"buf-pf-d1-xc", k_cg_zm<float, 1024, 4, true, 1, true, true>, 1024},
    {"buf-pf-d2-xc", k_cg_zm<float, 1024, 4, true, 2, true, true>, 1024},
    {"nt1024-pf-d1-xc", k_cg_zm<float, 1024, 4, true, 1, false, true>, 1024},
};
constexpr int kNumCgVariants = sizeof(kCgVariants) / sizeof(kCgVariants[0]);
}  // namespace

int cg_variant_count() { return kNumCgVariants; }

const char* cg_variant_name(int v) { return (v >= 0 && v < kNumCgVariants) ? kCgVariants[v].name : nullptr; }

hipError_t launch_cg_zm(const ExxArgs& a, int variant, hipStream_t s) {
    if (variant < 0 || variant >= kNumCgVariants) return hipErrorInvalidValue;
    const CgVariant& v = kCgVariants[variant];
    const int lds = (int)cg_zm_lds_bytes(1);
    hipError_t e = hipFuncSetAttribute((const void*)v.fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(v.fn, dim3(a.n_slots), dim3(v.nt), lds, s, a);
    return hipGetLastError();
}
