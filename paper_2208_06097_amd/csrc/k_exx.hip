// exx kernels for gfx950: pair-density gather with multipole moments,
// ghost-layer boundary values, the start guesses, CG Poisson solve per pair
// and the energy sum (the owner-computes scatter is in k_scatter.hip).
//
// Pair-domain arrays (b, v and the CG state) are stored compactly as
// [z][y][x] over the interior (n0*n1*n2 points), one array of `stride`
// doubles per pair (b, v) or per CG slot (r, p, q).
#include <type_traits>

#include "exx_device.h"
#include "harmonics.h"
#include "sea_internal.h"

namespace {

// O(h^12) central second-difference weights (half order 6):
// f'' ~ h^-2 (c0 f0 + sum_k ck (f_k + f_-k)).
__constant__ double kC[7] = {-5369.0 / 1800.0, 12.0 / 7.0,      -15.0 / 56.0,     10.0 / 189.0,
                             -1.0 / 112.0,     2.0 / 1925.0,    -1.0 / 16632.0};


// Deterministic block sum of one double (fixed shuffle tree, then LDS).
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) lds[wid] = v;
    __syncthreads();
    if (wid == 0) {
        double t = (lane < BS / 64) ? lds[lane] : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) lds[BS / 64] = t;
    }
    __syncthreads();
    const double r = lds[BS / 64];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// 1. gather rho_ij, write b = 4 pi rho, and the multipole moments (Eq. 11).
//
// The Racah solid harmonics are homogeneous polynomials of degree l in the
// displacement (dx, dy, dz) from the pair origin, so the moments Q_lm =
// dV sum rho R_lm are fixed linear combinations of the 84 Cartesian moments
// M_abc = sum rho dx^a dy^b dz^c (a + b + c <= 6).  Those separate: a
// workgroup takes 16 planes of a pair, a thread one x column position; per
// (y, column) it sums rho dz^c over the planes (7 products), folds them
// into sum rho dy^b dz^c (28 values) per row, and at the end the x powers
// make M_abc, summed over the lanes.  The polynomial coefficients of R_lm
// come from the same recurrence the kernels evaluate (k_racah_poly).

constexpr int GM_BS = 256;
constexpr int GM_CHUNK = 4096;
constexpr int GC_NM = 84;   // monomials of degree <= 6
constexpr int GC_ZB = 8;    // planes whose orbital loads the gather issues together
static_assert(GC_NM + 2 <= GC_N, "chunk record too short");

// position of x^a y^b z^c (a + b + c <= 6) in the order a, then b, then c
__host__ __device__ constexpr int mono_idx(int a, int b, int c) {
    int off = 0;
    for (int a2 = 0; a2 < a; ++a2) off += (7 - a2) * (8 - a2) / 2;
    for (int b2 = 0; b2 < b; ++b2) off += 7 - a - b2;
    return off + c;
}
// degree of the monomial at position t
__host__ __device__ inline int mono_deg(int t) {
    for (int a = 0; a <= 6; ++a)
        for (int b = 0; b <= 6 - a; ++b) {
            const int c = t - mono_idx(a, b, 0);
            if (c >= 0 && c <= 6 - a - b) return a + b + c;
        }
    return -1;
}

// position of y^b z^c (b + c <= 6)
__host__ __device__ constexpr int bc_idx(int b, int c) { return mono_idx(0, b, c); }

// tab[k * 84 + t]: coefficient of monomial t in the Racah harmonic k (one
// workgroup; thread t owns monomial t through the recurrence of
// racah_solid, with products by x, y, z and r^2 read as index shifts)
__global__ __launch_bounds__(128) void k_racah_poly(double* __restrict__ tab) {
    __shared__ double P[SEA_NMOM][GC_NM];
    const int t = threadIdx.x;
    int ta = 0, tb = 0, tc = 0;
    for (int a = 0; a <= 6; ++a)
        for (int b = 0; b <= 6 - a; ++b)
            for (int c = 0; c <= 6 - a - b; ++c)
                if (mono_idx(a, b, c) == t) {
                    ta = a;
                    tb = b;
                    tc = c;
                }
    const bool live = t < GC_NM;
    auto shx = [&](int k) { return (live && ta >= 1) ? P[k][mono_idx(ta - 1, tb, tc)] : 0.0; };
    auto shy = [&](int k) { return (live && tb >= 1) ? P[k][mono_idx(ta, tb - 1, tc)] : 0.0; };
    auto shz = [&](int k) { return (live && tc >= 1) ? P[k][mono_idx(ta, tb, tc - 1)] : 0.0; };
    auto shr2 = [&](int k) {
        double v = 0.0;
        if (live && ta >= 2) v += P[k][mono_idx(ta - 2, tb, tc)];
        if (live && tb >= 2) v += P[k][mono_idx(ta, tb - 2, tc)];
        if (live && tc >= 2) v += P[k][mono_idx(ta, tb, tc - 2)];
        return v;
    };
    if (live)
        for (int k = 0; k < SEA_NMOM; ++k) P[k][t] = (k == 0 && t == 0) ? 1.0 : 0.0;
    __syncthreads();
    for (int l = 0; l < 6; ++l) {
        double nv[2 * 7 + 1];
        const int cll = l * l + 2 * l, sll = l * l;
        const double f = -sqrt((2.0 * l + 1.0) / (2.0 * l + 2.0));
        nv[l + 1] = f * (shx(cll) - (l == 0 ? 0.0 : shy(sll)));          // C_{l+1,l+1}
        nv[7 + l + 1] = f * (shy(cll) + (l == 0 ? 0.0 : shx(sll)));      // S_{l+1,l+1}
        for (int m = 0; m <= l; ++m) {
            const double den = 1.0 / sqrt((double)((l + m + 1) * (l - m + 1)));
            const double aa = (2.0 * l + 1.0) * den;
            const double bb = sqrt((double)((l + m) * (l - m))) * den;
            const int base = l * l + l, basem = (l - 1) * (l - 1) + (l - 1);
            double c = aa * shz(base + m), sv = (m > 0) ? aa * shz(base - m) : 0.0;
            if (m <= l - 1) {
                c -= bb * shr2(basem + m);
                if (m > 0) sv -= bb * shr2(basem - m);
            }
            nv[m] = c;
            nv[7 + m] = sv;
        }
        __syncthreads();
        const int base1 = (l + 1) * (l + 1) + (l + 1);
        if (live) {
            for (int m = 0; m <= l + 1; ++m) {
                P[base1 + m][t] = nv[m];
                if (m > 0) P[base1 - m][t] = nv[7 + m];
            }
        }
        __syncthreads();
    }
    if (live)
        for (int k = 0; k < SEA_NMOM; ++k) tab[k * GC_NM + t] = P[k][t];
}

// One workgroup per (pair, plane chunk of GC_ZC), in a one-dimensional
// grid numbered so that each XCD (workgroup k runs on XCD k mod 8) takes a
// contiguous eighth of the pair list, every chunk of a pair in turn: the
// pairs of one orbital, which are neighbours in the list, then read its
// values through the same L2.
constexpr int GC_XCD = 8;
__device__ __forceinline__ void gc_block(int n_pairs, int n_zchunks, int& pid, int& zc) {
    const int k = blockIdx.x, x = k % GC_XCD, m = k / GC_XCD;
    const int per = (n_pairs + GC_XCD - 1) / GC_XCD;
    pid = x * per + m / n_zchunks;
    zc = m % n_zchunks;
}

// per chunk record of GC_N doubles: M_abc (84), sum |rho|, sum |rho| r^2
__global__ __launch_bounds__(GM_BS) void k_gather_cart(ExxArgs a) {
    __shared__ double red[GM_BS / 64][4][64];
    __shared__ double red2[GM_BS / 64][2][64];
    __shared__ double tot[GC_N];
    int pid, zc;
    gc_block(a.n_pairs, a.n_zchunks, pid, zc);
    if (pid >= a.n_pairs) return;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int z0 = zc * GC_ZC;
    if (z0 >= nz) return;
    const int z1 = min(z0 + GC_ZC, nz);
    // the cell record copied: its fields stay in registers across the stores to b
    const DevCell C = a.cells[a.pair_cell[pid]];
    const size_t oi = (size_t)P.i * C.Ng, oj = (size_t)P.j * C.Ng;
    double* __restrict__ b = a.b + (size_t)pid * a.stride;
    const int lane = threadIdx.x & 63, yg = threadIdx.x >> 6;
    constexpr int NG = GM_BS / 64;
    for (int t = threadIdx.x; t < GC_N; t += GM_BS) tot[t] = 0.0;
    __syncthreads();
    for (int xb = 0; xb < nx; xb += 64) {
        const int x = xb + lane;
        const bool live = x < nx;
        const size_t gx = (size_t)wrap_near(P.lo[0] + (live ? x : 0), C.N[0]);
        const double dx = (P.lo[0] + x) * C.h[0] - P.origin[0];
        double w[28];
#pragma unroll
        for (int q = 0; q < 28; ++q) w[q] = 0.0;
        double s0 = 0.0, s2 = 0.0;
        for (int y = yg; y < ny; y += NG) {
            const size_t gy = (size_t)wrap_near(P.lo[1] + y, C.N[1]);
            const double dy = (P.lo[1] + y) * C.h[1] - P.origin[1];
            double v[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            double t0 = 0.0, t2 = 0.0;
            // planes in batches: the batch's loads first (in flight together),
            // one copy per orbital precision, widened only at the product
            auto zbatch = [&](auto f32, int zb) {
                using PT = typename std::conditional<decltype(f32)::value, float, double>::type;
                const global_ptr<PT> ph = as_global((const PT*)C.phi);
                PT fi[GC_ZB], fj[GC_ZB];
#pragma unroll
                for (int k = 0; k < GC_ZB; ++k) {
                    const int z = min(zb + k, z1 - 1);   // past z1: a repeated plane, not used
                    const size_t g = ((size_t)wrap_near(P.lo[2] + z, C.N[2]) * C.N[1] + gy) * C.N[0] + gx;
                    fi[k] = ph[oi + g];
                    fj[k] = ph[oj + g];
                }
#pragma unroll
                for (int k = 0; k < GC_ZB; ++k) {
                    const int z = zb + k;
                    if (z >= z1) break;
                    const double dz = (P.lo[2] + z) * C.h[2] - P.origin[2];
                    const double rho = live ? (double)fi[k] * (double)fj[k] : 0.0;
                    if (live) b[((size_t)z * ny + y) * nx + x] = 4.0 * kPi * rho;
                    double p = rho;
                    v[0] += p;
#pragma unroll
                    for (int c = 1; c < 7; ++c) {
                        p *= dz;
                        v[c] += p;
                    }
                    t0 += fabs(rho);
                    t2 += fabs(rho) * dz * dz;
                }
            };
            for (int zb = z0; zb < z1; zb += GC_ZB) {
                if (C.phi_f32) zbatch(std::true_type(), zb);
                else zbatch(std::false_type(), zb);
            }
            double yp = 1.0;
#pragma unroll
            for (int bb = 0; bb < 7; ++bb) {
#pragma unroll
                for (int c = 0; c < 7 - bb; ++c) w[bc_idx(bb, c)] += yp * v[c];
                yp *= dy;
            }
            s0 += t0;
            s2 += t2 + dy * dy * t0;
        }
        // rows of one x summed over the row groups, then x powers over the
        // lanes: four (b, c) entries per phase, wave g taking entry 4 ph + g
#pragma unroll
        for (int ph = 0; ph < 7; ++ph) {
#pragma unroll
            for (int i = 0; i < 4; ++i) red[yg][i][lane] = w[4 * ph + i];
            if (ph == 0) {
                red2[yg][0][lane] = s0;
                red2[yg][1][lane] = s2;
            }
            lds_sync();   // (not a fence: the stores of b need not complete here)
            const int q = 4 * ph + yg;
            int bb = 0, c = q;
            while (c > 6 - bb) {
                c -= 7 - bb;
                ++bb;
            }
            double ws = 0.0;
            for (int g = 0; g < NG; ++g) ws += red[g][yg][lane];
            double xp = 1.0;
            for (int aa = 0; aa <= 6 - bb - c; ++aa) {
                double val = xp * ws;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) val += __shfl_down(val, off, 64);
                if (lane == 0) tot[mono_idx(aa, bb, c)] += val;
                xp *= dx;
            }
            if (ph == 0 && yg == 0) {
                double S0 = 0.0, S2 = 0.0;
                for (int g = 0; g < NG; ++g) {
                    S0 += red2[g][0][lane];
                    S2 += red2[g][1][lane];
                }
                S2 += dx * dx * S0;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
                    S0 += __shfl_down(S0, off, 64);
                    S2 += __shfl_down(S2, off, 64);
                }
                if (lane == 0) {
                    tot[GC_NM] += S0;
                    tot[GC_NM + 1] += S2;
                }
            }
            lds_sync();
        }
    }
    double* out = a.partial + ((size_t)pid * a.n_zchunks + zc) * GC_N;
    for (int t = threadIdx.x; t < GC_NM + 2; t += GM_BS) out[t] = tot[t];
}

// 2. sum the chunk partials in chunk order, convert to Racah moments with
//    the polynomial table; optional orthonormal copy
__global__ void k_moments_final(ExxArgs a, double* Q_orth) {
    __shared__ double M[GC_NM + 2];
    const int pid = blockIdx.x;
    const int k = threadIdx.x;
    if (pid == 0 && k == 0 && a.queue_ctr) *a.queue_ctr = 0;
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const sea_pair P = a.pairs[pid];
    const int used = (P.n[2] + GC_ZC - 1) / GC_ZC;
    for (int t = k; t < GC_NM + 2; t += blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < used; ++c) s += a.partial[((size_t)pid * a.n_zchunks + c) * GC_N + t];
        M[t] = s;
    }
    __syncthreads();
    __shared__ double Qs[SEA_NMOM];
    if (k < SEA_NACC) {
        double s;
        if (k < SEA_NMOM) {
            s = 0.0;
            for (int t = 0; t < GC_NM; ++t) s += a.racah_tab[k * GC_NM + t] * M[t];
        } else if (k == SEA_NMOM) {
            s = M[GC_NM];                        // sum |rho|
        } else if (k == SEA_NMOM + 1) {
            s = M[0];                            // sum rho
        } else {
            s = M[GC_NM + 1];                    // sum |rho| r^2
        }
        s *= C.dV;
        if (k < SEA_NMOM) {
            int l = 0;
            while ((l + 1) * (l + 1) <= k) ++l;
            if (l > a.lmax) s = 0.0;
            Qs[k] = s;
        }
        a.mom[(size_t)pid * SEA_NACC + k] = s;
        if (Q_orth && k < SEA_NMOM) {
            int l = 0;
            while ((l + 1) * (l + 1) <= k) ++l;
            const int m = k - l * l - l;
            Q_orth[(size_t)pid * SEA_NMOM + k] = s * racah_to_orthonormal(l, m);
        }
    }
    __syncthreads();
    // the degree-l part of the multipole sum as a homogeneous polynomial:
    // coefficient of monomial t (degree l) = sum over the harmonics of degree
    // l of eps_m Q_lm times the harmonic's coefficient of t (eps_0 = 1, else 2)
    for (int t = k; t < GC_NM; t += blockDim.x) {
        const int l = mono_deg(t);
        double c = 0.0;
        for (int q = l * l; q < (l + 1) * (l + 1); ++q) c += (q == l * l + l ? 1.0 : 2.0) * Qs[q] * a.racah_tab[q * GC_NM + t];
        a.mpoly[(size_t)pid * GC_NM + t] = c;
    }
}

// The multipole sum's homogeneous parts P_l(dx, dy, dz), l = 0..6, from the
// pair's monomial coefficients cf (the same order as mono_idx).
__device__ __forceinline__ void me_parts(const double* cf, double dx, double dy, double dz, double P[SEA_LMAX + 1]) {
#pragma unroll
    for (int l = 0; l <= SEA_LMAX; ++l) P[l] = 0.0;
    double xa = 1.0;
    int t = 0;
#pragma unroll
    for (int ea = 0; ea <= 6; ++ea) {
        double yb = xa;
#pragma unroll
        for (int eb = 0; eb <= 6 - ea; ++eb) {
            double mz = yb;
#pragma unroll
            for (int ec = 0; ec <= 6 - ea - eb; ++ec) {
                P[ea + eb + ec] += cf[t++] * mz;
                mz *= dz;
            }
            yb *= dy;
        }
        xa *= dx;
    }
}

// The multipole sum's parts along a line parallel to axis AX: with the
// other two displacement components fixed (d[AX] is ignored), P_l(s) =
// sum_{e <= l} q[l][e] s^e for the displacement s along AX.
template <int AX>
__device__ __forceinline__ void me_line_coeffs(const double* cf, const double d[3], double q[SEA_LMAX + 1][SEA_LMAX + 1]) {
#pragma unroll
    for (int l = 0; l <= SEA_LMAX; ++l)
#pragma unroll
        for (int e = 0; e <= SEA_LMAX; ++e) q[l][e] = 0.0;
    double pw[3][7];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pw[k][0] = 1.0;
#pragma unroll
        for (int e = 1; e <= 6; ++e) pw[k][e] = (k == AX) ? 1.0 : pw[k][e - 1] * d[k];
    }
    int t = 0;
#pragma unroll
    for (int ea = 0; ea <= 6; ++ea)
#pragma unroll
        for (int eb = 0; eb <= 6 - ea; ++eb)
#pragma unroll
            for (int ec = 0; ec <= 6 - ea - eb; ++ec) {
                const int e = AX == 0 ? ea : (AX == 1 ? eb : ec);
                q[ea + eb + ec][e] += cf[t++] * pw[0][ea] * pw[1][eb] * pw[2][ec];
            }
}

// 1/sqrt(x) for x > 0: the hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2 (each roughly doubles the correct bits, from about
// 23 to full double precision), a handful of FMAs instead of a correctly
// rounded square root and division.
__device__ __forceinline__ double rsqrt_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    y = y * fma(-0.5 * x * y, y, 1.5);
    y = y * fma(-0.5 * x * y, y, 1.5);
    return y;
}

// Multipole potential (Eq. 10) on the line: sum_l P_l(s) r^-(2l+1), r^2 = s^2 + rt2
__device__ __forceinline__ double me_line_potential(const double q[SEA_LMAX + 1][SEA_LMAX + 1], double s, double rt2) {
    const double rinv = rsqrt_nr(s * s + rt2), rinv2 = rinv * rinv;
    double v = 0.0, pw = rinv;
#pragma unroll
    for (int l = 0; l <= SEA_LMAX; ++l) {
        double p = q[l][l];
#pragma unroll
        for (int e = l - 1; e >= 0; --e) p = p * s + q[l][e];
        v += p * pw;
        pw *= rinv2;
    }
    return v;
}

// Multipole potential (Eq. 10) from the monomial coefficients: sum_l P_l r^-(2l+1)
__device__ __forceinline__ double me_poly_potential(const double* cf, double dx, double dy, double dz) {
    double P[SEA_LMAX + 1];
    me_parts(cf, dx, dy, dz, P);
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double rinv = 1.0 / sqrt(r2), rinv2 = rinv * rinv;
    double v = 0.0, pw = rinv;
#pragma unroll
    for (int l = 0; l <= SEA_LMAX; ++l) {
        v += P[l] * pw;
        pw *= rinv2;
    }
    return v;
}

// ---------------------------------------------------------------------------
// 3. boundary values (Eq. 10) on the ghost layers, folded into b:
//    b += sum over ghost taps (c_k / h_a^2) v_ME(ghost)
//
// One axis per launch and one face column per thread: the
// thread evaluates the 6 ghost values beyond each of the two faces of its
// (u, v) column and adds their taps to the 6 nearest interior points.  Axes
// run in separate launches (x, then y, then z), so every b point is updated
// by one thread at a time, in a fixed order; no ghost buffer is kept.
// Neighbouring lanes take neighbouring x for the y and z faces, so those
// updates are coalesced; the x faces' targets are 6 contiguous points of a
// row, so their updates go through LDS and out with a lane per target point.
constexpr int GA_BS = 256;
constexpr int GA_COLS = GA_BS / 2;   // lines per workgroup (two threads each)

// sum over the stencil taps of a column point i that fall past a face, of
// c_k times the odd continuation (period 2 (n + 1), zeros at -1 and n) of
// the column values val(index)
// Index of a face point of a line of n points within that line's frame (its
// first and last FF_W points; the whole line when n <= 2 FF_W).
__device__ __forceinline__ int frame_k(int i, int n) { return (n <= 2 * FF_W || i < FF_W) ? i : i - (n - 2 * FF_W); }

template <typename F>
__device__ __forceinline__ double face_taps(int i, int n, F&& val) {
    if (n >= 2 * FF_W) {
        // the faces apart: a tap past a face mirrors onto the same face, index
        // d from the face taking -c_k val(k - d - 2) (d + 1 past the face is a
        // zero of the continuation)
        const bool low = i < FF_W;
        const int d = low ? i : n - 1 - i;
        double c = 0.0;
        // every tap reads (a tap that does not reach reads the face point
        // with weight 0, which leaves c unchanged), so that the reads of a
        // line are issued together rather than one branch at a time
#pragma unroll
        for (int k = 2; k <= SEA_HALO; ++k) {
            const int q = max(k - d - 2, 0);
            c -= (k >= d + 2 ? kC[k] : 0.0) * val(low ? q : n - 1 - q);
        }
        return c;
    }
    auto ext = [&](int q) {
        const int per = 2 * (n + 1);
        while (q < -1) q += per;
        while (q > 2 * n) q -= per;
        if (q == -1 || q == n) return 0.0;
        return q > n ? -val(2 * n - q) : val(q);
    };
    double c = 0.0;
#pragma unroll
    for (int k = 1; k <= SEA_HALO; ++k) {
        if (i - k < 0) c += kC[k] * ext(i - k);
        if (i + k >= n) c += kC[k] * ext(i + k);
    }
    return c;
}

// Two threads per line, one per face (side 0: the low face, 1: the high
// face; the first and second half of the workgroup take the same GA_COLS
// lines), each forming its face's line coefficients; a line shorter than
// 2 SEA_HALO points, whose faces' taps overlap, is done by side 0 alone.
// FACE (spectral start, pairs the sine transform takes): the line also
// evaluates the multipole potential x0 (Eq. 10, the ghost values' own
// expansion) at its face points, the first and last FF_W points of the line
// (all of it when n <= 2 FF_W), and adds the taps of -D x0 along this axis
// there into a.fcorr.  The x launch writes every point within FF_W of an x
// face; the y launch adds at the points within FF_W of an x face and writes
// the rest of its points, the z launch likewise after x and y, so every face
// point of the pair is set once and then summed in x, y, z order.
template <int AX, bool FACE>
__global__ __launch_bounds__(GA_BS) void k_ghost_axis(ExxArgs a) {
    constexpr int ax = AX;
    constexpr int FS = 2 * FF_W;   // frame of a line
    __shared__ double cf[GC_NM];
    __shared__ double tap[GA_COLS][2 * SEA_HALO];
    __shared__ double xs[FACE ? GA_COLS : 1][2 * FS];   // x launch: a line's -D x0; thin lines: its x0 after it
    const int pid = blockIdx.x;
    if (threadIdx.x < GC_NM) cf[threadIdx.x] = a.mpoly[(size_t)pid * GC_NM + threadIdx.x];
    __syncthreads();
    const DevCell C = a.cells[a.pair_cell[pid]];   // copied: fields stay in registers across stores
    const sea_pair P = a.pairs[pid];
    const int u = ax == 0 ? 1 : 0, v = ax == 2 ? 1 : 2;   // line coordinates, x first where it is one
    const int n = P.n[ax];
    const double ih2 = 1.0 / (C.h[ax] * C.h[ax]);
    const size_t st[3] = {1, (size_t)P.n[0], (size_t)P.n[0] * P.n[1]};
    const int c0 = blockIdx.y * GA_COLS;
    const int lc = threadIdx.x % GA_COLS, side = threadIdx.x / GA_COLS;
    auto column = [&](int c, int& au, int& av) {
        au = c % a.nmax;
        av = c / a.nmax;
        return av < a.nmax && au < P.n[u] && av < P.n[v];
    };
    int au, av;
    const bool live = column(c0 + lc, au, av);
    const bool staged = ax == 0 && n >= 2 * SEA_HALO;   // x faces, the two faces' targets disjoint
    const bool face = FACE && spectral_pair(P);          // uniform
    const bool split = n >= 2 * SEA_HALO;                // the faces' ghost taps apart
    const int nf = n < FS ? n : FS;                      // frame points of the line
    auto frame_pt = [&](int j) { return (n <= FS || j < FF_W) ? j : n - FS + j; };
    double* b = a.b + (size_t)pid * a.stride;
    if (live && (split || side == 0)) {
        int pos[3];
        pos[u] = au;
        pos[v] = av;
        const size_t base = pos[u] * st[u] + pos[v] * st[v];
        // set by an earlier launch: the line lies within FF_W of an x face
        // (or, for z, of a y face)
        const bool set_before = near_face(pos[0], P.n[0]) || (ax == 2 && near_face(pos[1], P.n[1]));
        double* fc = FACE ? a.fcorr + (size_t)pid * a.stride + base : nullptr;
        // y and z faces of a long line: the b values this face's taps update
        // (and the -D x0 values an earlier launch set there), loaded before
        // the multipole work so that their latency overlaps it; the points
        // are distinct, so the updates need not wait for one another
        const bool pre = split && !staged;
        double bpre[SEA_HALO], fpre[FF_W];
        if (pre) {
#pragma unroll
            for (int d = 0; d < SEA_HALO; ++d) bpre[d] = b[base + (size_t)(side ? n - 1 - d : d) * st[ax]];
            if (FACE && face && set_before) {
#pragma unroll
                for (int d = 0; d < FF_W; ++d) fpre[d] = fc[(size_t)(side ? n - 1 - d : d) * st[ax]];
            }
        }
        // the line's fixed displacements folded into line coefficients once
        double dv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) dv[k] = k == ax ? 0.0 : (P.lo[k] + pos[k]) * C.h[k] - P.origin[k];
        double q[SEA_LMAX + 1][SEA_LMAX + 1];
        me_line_coeffs<AX>(cf, dv, q);
        const double rt2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
        // the ghost values beyond one face folded into b
        auto fold = [&](int plus) {
            double g[SEA_HALO + 1];
#pragma unroll
            for (int L = 1; L <= SEA_HALO; ++L) {
                const int pa = plus ? n - 1 + L : -L;
                g[L] = me_line_potential(q, (P.lo[ax] + pa) * C.h[ax] - P.origin[ax], rt2);
            }
#pragma unroll
            for (int d = 0; d < SEA_HALO; ++d) {
                if (d >= n) break;
                double acc = 0.0;
#pragma unroll
                for (int k = d + 1; k <= SEA_HALO; ++k) acc += kC[k] * ih2 * g[k - d];
                const int p = plus ? n - 1 - d : d;
                if (staged) tap[lc][plus ? 2 * SEA_HALO - 1 - d : d] = acc;   // slot j: point j or n - 12 + j
                else if (pre) b[base + (size_t)p * st[ax]] = bpre[d] + acc;
                else b[base + (size_t)p * st[ax]] += acc;
            }
        };
        if (split) {
            fold(side);
            if (FACE && face) {
                // -D x0 at this face's 5 frame points: x0 there in registers,
                // every index known at compile time; point d from the face
                // takes sum_{k >= d + 2} c_k x0(k - d - 2) of the same face
                double xf[FF_W];
#pragma unroll
                for (int j = 0; j < FF_W; ++j)
                    xf[j] = me_line_potential(q, (P.lo[ax] + (side ? n - 1 - j : j)) * C.h[ax] - P.origin[ax], rt2);
#pragma unroll
                for (int d = 0; d < FF_W; ++d) {
                    double acc = 0.0;
#pragma unroll
                    for (int k = d + 2; k <= SEA_HALO; ++k) acc -= kC[k] * xf[k - d - 2];
                    const double t = acc * ih2;
                    if (ax == 0) {   // out through LDS below, a lane per point
                        xs[lc][side ? FS - 1 - d : d] = -t;
                    } else {         // neighbouring lanes take neighbouring x: straight out
                        fc[(size_t)(side ? n - 1 - d : d) * st[ax]] = set_before ? fpre[d] - t : -t;
                    }
                }
            }
        } else {   // a line shorter than 2 SEA_HALO: both faces here
            fold(0);
            fold(1);
            if (FACE && face) {
                // x0 on the frame (LDS), then the taps of the odd
                // continuation over the whole line
                for (int j = 0; j < nf; ++j)
                    xs[lc][FS + j] = me_line_potential(q, (P.lo[ax] + frame_pt(j)) * C.h[ax] - P.origin[ax], rt2);
                for (int j = 0; j < nf; ++j) {
                    const int p = frame_pt(j);
                    const double t = face_taps(p, n, [&](int i) { return xs[lc][FS + frame_k(i, n)]; }) * ih2;
                    if (ax == 0) {
                        xs[lc][j] = -t;
                    } else {
                        double* f = fc + (size_t)p * st[ax];
                        *f = set_before ? *f - t : -t;
                    }
                }
            }
        }
    }
    if (FACE && face && ax == 0) {   // the x face points out through LDS, a lane per point
        __syncthreads();
        double* fc = a.fcorr + (size_t)pid * a.stride;
        for (int t = threadIdx.x; t < GA_COLS * FS; t += GA_BS) {
            const int c = t / FS, j = t % FS;
            int cu, cv;
            if (j >= nf || !column(c0 + c, cu, cv)) continue;
            fc[(size_t)cu * st[1] + (size_t)cv * st[2] + frame_pt(j)] = xs[c][j];
        }
    }
    if (!staged) return;
    __syncthreads();
    // every b value first (distinct points: the loads need not wait for the
    // stores), then the sums
    constexpr int NU = GA_COLS * 2 * SEA_HALO / GA_BS;
    static_assert(NU * GA_BS == GA_COLS * 2 * SEA_HALO, "whole rounds of updates");
    double bv[NU];
    size_t off[NU];
    bool ok[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const int t = threadIdx.x + i * GA_BS;
        const int c = t / (2 * SEA_HALO), j = t % (2 * SEA_HALO);
        int cu, cv;
        ok[i] = column(c0 + c, cu, cv);
        const int p = j < SEA_HALO ? j : n - 2 * SEA_HALO + j;
        off[i] = (size_t)cu * st[1] + (size_t)cv * st[2] + p;
        bv[i] = ok[i] ? b[off[i]] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NU; ++i) {
        const int t = threadIdx.x + i * GA_BS;
        if (ok[i]) b[off[i]] = bv[i] + tap[t / (2 * SEA_HALO)][t % (2 * SEA_HALO)];
    }
}

// ---------------------------------------------------------------------------
// 3b. multipole start: x0 = regularized multipole potential on the interior.
//     l = 0: q erf(r/r_s)/r; l >= 1: the l-th term times (1 - exp(-r^2/r_s^2))^{l+1};
//     r_s = sqrt(2 <r^2>/3) from the |rho|-weighted second moment (the
//     exact width for a spherical Gaussian density).

// Regularized multipole potential at displacement (dx,dy,dz); Q = the 52
// accumulators of a pair (Racah moments, |rho| sum, q, |rho| r^2 sum).
template <int LM>
__device__ __forceinline__ double me_start_value(const double* Q, int lmax, double dx, double dy, double dz) {
    const double r2m = Q[SEA_NMOM] > 0.0 ? Q[SEA_NMOM + 2] / Q[SEA_NMOM] : 1.0;
    const double rs = sqrt(fmax(2.0 * r2m / 3.0, 1e-6));
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double r = sqrt(r2);
    if (r < 1e-12) return Q[0] * 2.0 / (rs * sqrt(kPi));
    double R[(LM + 1) * (LM + 1)];
    racah_solid<LM>(dx, dy, dz, R);
    const double rinv = 1.0 / r, rinv2 = rinv * rinv;
    const double damp = 1.0 - exp(-r2 / (rs * rs));
    double val = Q[0] * erf(r / rs) * rinv;
    double pw = rinv * rinv2, dl = damp;
#pragma unroll
    for (int l = 1; l <= LM; ++l) {
        dl *= damp;
        if (l <= lmax) {
            const int base = l * l + l;
            double acc = Q[base] * R[base];
#pragma unroll
            for (int m = 1; m <= l; ++m) acc += 2.0 * (Q[base + m] * R[base + m] + Q[base - m] * R[base - m]);
            val += acc * pw * dl;
        }
        pw *= rinv2;
    }
    return val;
}

// The same start value from the degree-l parts P_l of the multipole sum
// (which replace the per-degree harmonic sums) at squared distance r2.
__device__ __forceinline__ double me_start_from_parts(const double* Q, const double P[SEA_LMAX + 1], double r2) {
    const double r2m = Q[SEA_NMOM] > 0.0 ? Q[SEA_NMOM + 2] / Q[SEA_NMOM] : 1.0;
    const double rs = sqrt(fmax(2.0 * r2m / 3.0, 1e-6));
    const double r = sqrt(r2);
    if (r < 1e-12) return Q[0] * 2.0 / (rs * sqrt(kPi));
    const double rinv = 1.0 / r, rinv2 = rinv * rinv;
    const double damp = 1.0 - exp(-r2 / (rs * rs));
    double val = Q[0] * erf(r / rs) * rinv;
    double pw = rinv * rinv2, dl = damp;
#pragma unroll
    for (int l = 1; l <= SEA_LMAX; ++l) {
        dl *= damp;
        val += P[l] * pw * dl;
        pw *= rinv2;
    }
    return val;
}

// ... from the pair's monomial coefficients cf
__device__ __forceinline__ double me_start_poly(const double* cf, const double* Q, double dx, double dy, double dz) {
    double P[SEA_LMAX + 1];
    me_parts(cf, dx, dy, dz, P);
    return me_start_from_parts(Q, P, dx * dx + dy * dy + dz * dz);
}

template <int LM>
__global__ __launch_bounds__(GM_BS) void k_me_guess(ExxArgs a) {
    __shared__ double Q[SEA_NACC];
    const int pid = blockIdx.x;
    if (threadIdx.x < SEA_NACC) Q[threadIdx.x] = a.mom[(size_t)pid * SEA_NACC + threadIdx.x];
    __syncthreads();
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const long n_int = (long)nx * ny * nz;
    const long beg = (long)blockIdx.y * GM_CHUNK;
    if (beg >= n_int) return;
    const long end = min(beg + GM_CHUNK, n_int);
    double* x = a.v + (size_t)pid * a.stride;
    BoxWalk wk((int)(beg + threadIdx.x), GM_BS, nx, ny);
    for (long id = beg + threadIdx.x; id < end; id += GM_BS, wk.next()) {
        const int xx = wk.x, yy = wk.y, zz = wk.z;
        x[id] = me_start_value<LM>(Q, a.lmax, (P.lo[0] + xx) * C.h[0] - P.origin[0],
                                   (P.lo[1] + yy) * C.h[1] - P.origin[1], (P.lo[2] + zz) * C.h[2] - P.origin[2]);
    }
}

// The whole multipole start on the planes of the pairs the sine transform
// skips (an axis beyond 64 points).
__global__ __launch_bounds__(GM_BS) void k_me_big(ExxArgs a) {
    __shared__ double Q[SEA_NACC];
    __shared__ double cf[GC_NM];
    const int pid = blockIdx.x, z = blockIdx.y;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    if (z >= nz || spectral_pair(P)) return;
    if (threadIdx.x < SEA_NACC) Q[threadIdx.x] = a.mom[(size_t)pid * SEA_NACC + threadIdx.x];
    if (threadIdx.x < GC_NM) cf[threadIdx.x] = a.mpoly[(size_t)pid * GC_NM + threadIdx.x];
    __syncthreads();
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const double dz = (P.lo[2] + z) * C.h[2] - P.origin[2];
    double* x = a.v + (size_t)pid * a.stride + (size_t)z * nx * ny;
    for (int t = threadIdx.x; t < nx * ny; t += GM_BS)
        x[t] = me_start_poly(cf, Q, (P.lo[0] + t % nx) * C.h[0] - P.origin[0], (P.lo[1] + t / nx) * C.h[1] - P.origin[1],
                             dz);
}

// ---------------------------------------------------------------------------
// 3c. learned start: corner-aligned trilinear maps between a pair domain
//     (n per axis) and the network grid (D per axis).  Sample k of D sits at
//     fine coordinate k (n-1)/(D-1); fine point i sits at coarse i (D-1)/(n-1).

struct Lerp {
    int i0;
    double t;
};

__device__ __forceinline__ Lerp lerp_at(int k, int from, int to) {
    // position of sample k of a `to`-grid on a `from`-grid
    if (from < 2) return Lerp{0, 0.0};
    const double u = (double)k * (double)(from - 1) / (double)(to - 1);
    int i0 = (int)floor(u);
    if (i0 > from - 2) i0 = from - 2;
    return Lerp{i0, u - i0};
}

constexpr int NNS_BS = 256;

// mode 0: x32 = resample(rho / s); mode 1: t32 = resample((v - v_ME) / s)
template <int LM>
__global__ __launch_bounds__(NNS_BS) void k_nn_sample(ExxArgs a, int D, float* __restrict__ out, double* s_out,
                                                      int mode) {
    __shared__ double Q[SEA_NACC];
    const int pid = blockIdx.x;
    if (threadIdx.x < SEA_NACC) Q[threadIdx.x] = a.mom[(size_t)pid * SEA_NACC + threadIdx.x];
    __syncthreads();
    const DevCell& C = a.cells[a.pair_cell[pid]];
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int D3 = D * D * D;
    const int k = blockIdx.y * NNS_BS + threadIdx.x;
    const double s = Q[SEA_NMOM];
    if (k == 0 && s_out) s_out[pid] = s;
    if (k >= D3) return;
    const Lerp lx = lerp_at(k % D, nx, D), ly = lerp_at((k / D) % D, ny, D), lz = lerp_at(k / (D * D), nz, D);
    const size_t oi = (size_t)P.i * C.Ng, oj = (size_t)P.j * C.Ng;
    const double* v = a.v + (size_t)pid * a.stride;
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
        const int cx = lx.i0 + (c & 1), cy = ly.i0 + ((c >> 1) & 1), cz = lz.i0 + (c >> 2);
        const double wgt = ((c & 1) ? lx.t : 1.0 - lx.t) * (((c >> 1) & 1) ? ly.t : 1.0 - ly.t) *
                           ((c >> 2) ? lz.t : 1.0 - lz.t);
        if (wgt == 0.0 || cx >= nx || cy >= ny || cz >= nz) continue;
        double f;
        if (mode == 0) {
            const size_t g = ((size_t)wrap_idx(P.lo[2] + cz, C.N[2]) * C.N[1] + wrap_idx(P.lo[1] + cy, C.N[1])) *
                                 C.N[0] +
                             wrap_idx(P.lo[0] + cx, C.N[0]);
            f = load_phi(C.phi, C.phi_f32, oi + g) * load_phi(C.phi, C.phi_f32, oj + g);
        } else {
            f = v[((size_t)cz * ny + cy) * nx + cx] -
                me_start_value<LM>(Q, a.lmax, (P.lo[0] + cx) * C.h[0] - P.origin[0],
                                   (P.lo[1] + cy) * C.h[1] - P.origin[1], (P.lo[2] + cz) * C.h[2] - P.origin[2]);
        }
        acc += wgt * f;
    }
    out[(size_t)pid * D3 + k] = s > 0.0 ? (float)(acc / s) : 0.0f;
}

// Cubic interpolation weights along one axis: fine point k of a `to`-grid
// sits at coarse coordinate u = k (from - 1) / (to - 1) (corners aligned);
// the 4-point Lagrange cubic through nodes i0 - 1 .. i0 + 2 (i0 = floor(u)),
// with the nodes past either end continued oddly (y_{-1} = 2 y_0 - y_1,
// y_from = 2 y_{from-1} - y_{from-2}), folded into 4 weights w[q] of nodes
// base + q.  At a node (u integer) it is that node's value.
struct Cub {
    int base;
    double w[4];
};

__device__ __forceinline__ Cub cubic_at(int k, int from, int to) {
    Cub c{0, {0.0, 0.0, 0.0, 0.0}};   // needs from >= 4 (checked at launch)
    const double u = to > 1 ? (double)k * (double)(from - 1) / (double)(to - 1) : 0.0;
    int i0 = (int)floor(u);
    if (i0 > from - 2) i0 = from - 2;
    const double f = u - i0;
    const double wq[4] = {-f * (f - 1.0) * (f - 2.0) / 6.0, (f + 1.0) * (f - 1.0) * (f - 2.0) / 2.0,
                          -(f + 1.0) * f * (f - 2.0) / 2.0, (f + 1.0) * f * (f - 1.0) / 6.0};
    c.base = min(max(i0 - 1, 0), from - 4);
    // node q of the stencil lands on point i0 - 1 + q; one beyond an end is
    // the linear extrapolation 2 f(end) - f(end -+ 1).  Summed per output
    // slot in node order, with compile-time slots (no indexed registers).
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int idx = c.base + m;
        double w = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = i0 - 1 + q;
            if (j < 0) w += idx == 0 ? 2.0 * wq[q] : (idx == 1 ? -wq[q] : 0.0);
            else if (j >= from) w += idx == from - 1 ? 2.0 * wq[q] : (idx == from - 2 ? -wq[q] : 0.0);
            else w += j == idx ? wq[q] : 0.0;
        }
        c.w[m] = w;
    }
    return c;
}

// x += s * upsample(y32) on the pair domain: tricubic interpolation of the
// network grid (a fine point on a coarse node takes that node's value; with
// 63 points per axis and a 32-point network grid every other point is one).
// A trilinear map would leave the interpolant's second differences wrong by
// a factor of 2 at every point, a high-frequency residual the CG then has
// to remove.
__global__ __launch_bounds__(GM_BS) void k_nn_apply(ExxArgs a, int D, const float* __restrict__ y32) {
    const int pid = blockIdx.x;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const long n_int = (long)nx * ny * nz;
    const long beg = (long)blockIdx.y * GM_CHUNK;
    if (beg >= n_int) return;
    const long end = min(beg + GM_CHUNK, n_int);
    if (nx <= 64 && ny <= 64 && nz <= 64) return;   // k_nn_apply_ring takes those
    const double s = a.mom[(size_t)pid * SEA_NACC + SEA_NMOM];
    if (!(s > 0.0)) return;
    const float* y = y32 + (size_t)pid * D * D * D;
    double* x = a.v + (size_t)pid * a.stride;
    for (long id = beg + threadIdx.x; id < end; id += GM_BS) {
        const int ix = (int)(id % nx), iy = (int)((id / nx) % ny), iz = (int)(id / ((long)nx * ny));
        const Cub cx = cubic_at(ix, D, nx), cy = cubic_at(iy, D, ny), cz = cubic_at(iz, D, nz);
        double acc = 0.0;
        for (int c = 0; c < 4; ++c) {
            if (cz.w[c] == 0.0) continue;
            double accy = 0.0;
            for (int b = 0; b < 4; ++b) {
                if (cy.w[b] == 0.0) continue;
                const float* row = y + ((size_t)(cz.base + c) * D + cy.base + b) * D + cx.base;
                double accx = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) accx += cx.w[q] * (double)row[q];
                accy += cy.w[b] * accx;
            }
            acc += cz.w[c] * accy;
        }
        x[id] += s * acc;
    }
}

// The same map, separably, for pairs with every axis <= 64: a workgroup
// takes NA_ZC output planes of one pair; each network plane it needs is
// interpolated in x and y once into a ring of four LDS planes (FP32, the
// network's precision), and an output plane is the cubic combination of the
// four ring planes its z weights name.  The per-axis weights come from
// cubic_at once per grid index, not per point.
constexpr int NA_BS = 256;
constexpr int NA_ZC = 16;   // output planes per workgroup

__global__ __launch_bounds__(NA_BS) void k_nn_apply_ring(ExxArgs a, int D, const float* __restrict__ y32) {
    __shared__ float U[4][64 * 64];   // network planes interpolated in x and y (ring by plane index mod 4)
    __shared__ double wt[3][64][4];
    __shared__ int bs[3][64];
    const int pid = blockIdx.x;
    const sea_pair P = a.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    if (nx > 64 || ny > 64 || nz > 64) return;   // k_nn_apply takes those
    const int z0 = blockIdx.y * NA_ZC;
    if (z0 >= nz) return;
    const int z1 = min(nz, z0 + NA_ZC);
    const double s = a.mom[(size_t)pid * SEA_NACC + SEA_NMOM];
    if (!(s > 0.0)) return;
    for (int t = threadIdx.x; t < 3 * 64; t += NA_BS) {
        const int ax = t / 64, k = t % 64;
        const int n = ax == 0 ? nx : (ax == 1 ? ny : nz);
        if (k < n) {
            const Cub c = cubic_at(k, D, n);
            bs[ax][k] = c.base;
#pragma unroll
            for (int q = 0; q < 4; ++q) wt[ax][k][q] = c.w[q];
        }
    }
    __syncthreads();
    const float* y = y32 + (size_t)pid * D * D * D;
    double* x = a.v + (size_t)pid * a.stride;
    const int npl = nx * ny;
    int hi = -1;   // the ring holds network planes hi - 3 .. hi
    for (int z = z0; z < z1; ++z) {
        const int cb = bs[2][z];
        if (cb + 3 > hi) {
            for (int k = max(cb, hi + 1); k <= cb + 3; ++k) {   // planes the ring lacks
                const float* yk = y + (size_t)k * D * D;
                float* Uk = U[k & 3];
                for (int t = threadIdx.x; t < npl; t += NA_BS) {
                    const int ix = t % nx, iy = t / nx;
                    const float* r0 = yk + bs[1][iy] * D + bs[0][ix];
                    double acc = 0.0;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const float* row = r0 + b * D;
                        double ax = 0.0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) ax += wt[0][ix][q] * (double)row[q];
                        acc += wt[1][iy][b] * ax;
                    }
                    Uk[t] = (float)acc;
                }
            }
            hi = cb + 3;
            __syncthreads();
        }
        double* xz = x + (size_t)z * npl;
        const double w0 = wt[2][z][0], w1 = wt[2][z][1], w2 = wt[2][z][2], w3 = wt[2][z][3];
        const float* u0 = U[cb & 3];
        const float* u1 = U[(cb + 1) & 3];
        const float* u2 = U[(cb + 2) & 3];
        const float* u3 = U[(cb + 3) & 3];
        for (int t = threadIdx.x; t < npl; t += NA_BS)
            xz[t] += s * (((w0 * (double)u0[t] + w1 * (double)u1[t]) + w2 * (double)u2[t]) + w3 * (double)u3[t]);
        __syncthreads();   // before the ring's next planes overwrite these
    }
}

// ---------------------------------------------------------------------------
// 4. CG on A v = b, A = -Lap_h on the interior (zero outside), one workgroup
//    per pair, persistent over the pair list.

constexpr int CG_BS = 256;

struct StencilW {
    double diag;
    double wx[7], wy[7], wz[7];
};

__device__ __forceinline__ StencilW make_weights(const double* h) {
    StencilW w;
    const double ix = 1.0 / (h[0] * h[0]), iy = 1.0 / (h[1] * h[1]), iz = 1.0 / (h[2] * h[2]);
    w.diag = -kC[0] * (ix + iy + iz);
#pragma unroll
    for (int k = 0; k < 7; ++k) {
        w.wx[k] = -kC[k] * ix;
        w.wy[k] = -kC[k] * iy;
        w.wz[k] = -kC[k] * iz;
    }
    return w;
}

__device__ __forceinline__ double apply_A_pt(const double* __restrict__ p, long id, int x, int y, int z,
                                             int nx, int ny, int nz, const StencilW& w) {
    const long sy = nx, sz = (long)nx * ny;
    double s = w.diag * p[id];
#pragma unroll
    for (int k = 1; k <= SEA_HALO; ++k) {
        const double ax = (x - k >= 0 ? p[id - k] : 0.0) + (x + k < nx ? p[id + k] : 0.0);
        const double ay = (y - k >= 0 ? p[id - k * sy] : 0.0) + (y + k < ny ? p[id + k * sy] : 0.0);
        const double az = (z - k >= 0 ? p[id - k * sz] : 0.0) + (z + k < nz ? p[id + k * sz] : 0.0);
        s += w.wx[k] * ax + w.wy[k] * ay + w.wz[k] * az;
    }
    return s;
}

__global__ __launch_bounds__(CG_BS) void k_cg_f64(ExxArgs a) {
    __shared__ double red[CG_BS / 64 + 1];
    double* r = a.slots + (size_t)blockIdx.x * 3 * a.slot_stride;
    double* p = r + a.stride;
    double* q = p + a.stride;
    const double tol2 = a.rel_tol * a.rel_tol;
    for (int qi = blockIdx.x; qi < a.n_pairs; qi += gridDim.x) {
        const int pid = a.order ? a.order[qi] : qi;  // largest domains first
        const DevCell& C = a.cells[a.pair_cell[pid]];
        const StencilW w = make_weights(C.h);
        const sea_pair P = a.pairs[pid];
        const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
        const long n = (long)nx * ny * nz;
        const long nxy = (long)nx * ny;
        const double* b = a.b + (size_t)pid * a.stride;
        double* x = a.v + (size_t)pid * a.stride;

        // bnorm^2, and x0 = 0
        double bb = 0.0;
        for (long id = threadIdx.x; id < n; id += CG_BS) {
            const double t = b[id];
            bb += t * t;
            if (!a.x_nonzero) x[id] = 0.0;
        }
        bb = block_sum<CG_BS>(bb, red);
        int it = 0;
        double rel = 0.0;
        int conv = 0;
        if (!(bb > 0.0)) {
            conv = (bb == 0.0) ? 1 : -1;
        } else {
            bool restart = true;
            double rr = 0.0;
            for (;;) {
                if (restart) {
                    // r = b - A x, p = r
                    double t2 = 0.0;
                    for (long id = threadIdx.x; id < n; id += CG_BS) {
                        const int xx = (int)(id % nx), yy = (int)((id / nx) % ny), zz = (int)(id / nxy);
                        const double ri = b[id] - apply_A_pt(x, id, xx, yy, zz, nx, ny, nz, w);
                        r[id] = ri;
                        p[id] = ri;
                        t2 += ri * ri;
                    }
                    rr = block_sum<CG_BS>(t2, red);
                    rel = sqrt(rr / bb);
                    if (!(rr == rr)) { conv = -1; break; }
                    if (rr <= tol2 * bb) { conv = 1; break; }
                    if (it >= a.max_iter) { conv = 0; break; }
                    restart = false;
                }
                // q = A p, pq
                double pq = 0.0;
                for (long id = threadIdx.x; id < n; id += CG_BS) {
                    const int xx = (int)(id % nx), yy = (int)((id / nx) % ny), zz = (int)(id / nxy);
                    const double qi = apply_A_pt(p, id, xx, yy, zz, nx, ny, nz, w);
                    q[id] = qi;
                    pq += p[id] * qi;
                }
                pq = block_sum<CG_BS>(pq, red);
                const double alpha = rr / pq;
                double rn = 0.0;
                for (long id = threadIdx.x; id < n; id += CG_BS) {
                    x[id] += alpha * p[id];
                    const double ri = r[id] - alpha * q[id];
                    r[id] = ri;
                    rn += ri * ri;
                }
                rn = block_sum<CG_BS>(rn, red);
                ++it;
                if (rn <= tol2 * bb || it >= a.max_iter || !(rn == rn)) {
                    restart = true;   // verify with the true residual
                    continue;
                }
                const double beta = rn / rr;
                rr = rn;
                for (long id = threadIdx.x; id < n; id += CG_BS) p[id] = r[id] + beta * p[id];
                __syncthreads();
            }
        }
        // e_ij = dV sum rho v with rho gathered again
        const size_t oi = (size_t)P.i * C.Ng, oj = (size_t)P.j * C.Ng;
        double e = 0.0;
        for (long id = threadIdx.x; id < n; id += CG_BS) {
            const int xx = (int)(id % nx), yy = (int)((id / nx) % ny), zz = (int)(id / nxy);
            const size_t g = ((size_t)wrap_idx(P.lo[2] + zz, C.N[2]) * C.N[1] + wrap_idx(P.lo[1] + yy, C.N[1])) * C.N[0]
                             + wrap_idx(P.lo[0] + xx, C.N[0]);
            e += load_phi(C.phi, C.phi_f32, oi + g) * load_phi(C.phi, C.phi_f32, oj + g) * x[id];
        }
        e = block_sum<CG_BS>(e, red);
        if (threadIdx.x == 0) {
            DevStat st;
            st.iters = it;
            st.converged = conv;
            st.rel_res = rel;
            st.e_ij = C.dV * e;
            st.s_abs = a.mom[(size_t)pid * SEA_NACC + SEA_NMOM];
            st.q = a.mom[(size_t)pid * SEA_NACC + SEA_NMOM + 1];
            a.stats[pid] = st;
            if (a.hist && it <= a.hist_len) a.hist[(size_t)pid * (a.hist_len + 1) + it] = rel;   // its exit only
        }
    }
}

// ---------------------------------------------------------------------------
// 6. E = -sum_i e_ii - 2 sum_{i<j} e_ij, plus counters, in a fixed order.
//    out[0] = E, out[1] = #not converged, out[2] = #nonfinite.

constexpr int ES_BS = 256;

__global__ __launch_bounds__(ES_BS) void k_energy_sum(ExxArgs a, double* out, double* e_dev) {
    __shared__ double red[ES_BS / 64 + 1];
    const DevCell& C = a.cells[blockIdx.x];
    double e = 0.0, nc = 0.0, nf = 0.0;
    for (int k = C.pair_begin + threadIdx.x; k < C.pair_end; k += ES_BS) {
        const DevStat st = a.stats[k];
        const sea_pair P = a.pairs[k];
        e -= (P.i == P.j ? 1.0 : 2.0) * st.e_ij;
        nc += (st.converged == 0) ? 1.0 : 0.0;
        nf += (st.converged < 0 || !(st.e_ij == st.e_ij)) ? 1.0 : 0.0;
        if (e_dev) e_dev[k] = st.e_ij;
    }
    e = block_sum<ES_BS>(e, red);
    nc = block_sum<ES_BS>(nc, red);
    nf = block_sum<ES_BS>(nf, red);
    if (threadIdx.x == 0) {
        out[3 * blockIdx.x] = e;
        out[3 * blockIdx.x + 1] = nc;
        out[3 * blockIdx.x + 2] = nf;
        if (C.exx) *C.exx = e;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers

int exx_n_chunks(long n_int_max) { return (int)((n_int_max + GM_CHUNK - 1) / GM_CHUNK); }

hipError_t launch_gather_moments(const ExxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_racah_poly, dim3(1), dim3(128), 0, s, a.racah_tab);
    const long nb = (long)((a.n_pairs + GC_XCD - 1) / GC_XCD) * GC_XCD * a.n_zchunks;
    if (nb > 0x7fffffffL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather_cart, dim3((unsigned)nb), dim3(GM_BS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_moments_final(const ExxArgs& a, double* Q_orth, hipStream_t s) {
    hipLaunchKernelGGL(k_moments_final, dim3(a.n_pairs), dim3(64), 0, s, a, Q_orth);
    return hipGetLastError();
}

hipError_t launch_boundary_fold(const ExxArgs& a, int nz_max, hipStream_t s, bool face) {
    (void)nz_max;
    if (face && !a.fcorr) return hipErrorInvalidValue;
    const unsigned gy = (unsigned)(((long)a.nmax * a.nmax + GA_COLS - 1) / GA_COLS);
    const dim3 g(a.n_pairs, gy);
    if (face) {
        hipLaunchKernelGGL((k_ghost_axis<0, true>), g, dim3(GA_BS), 0, s, a);
        hipLaunchKernelGGL((k_ghost_axis<1, true>), g, dim3(GA_BS), 0, s, a);
        hipLaunchKernelGGL((k_ghost_axis<2, true>), g, dim3(GA_BS), 0, s, a);
    } else {
        hipLaunchKernelGGL((k_ghost_axis<0, false>), g, dim3(GA_BS), 0, s, a);
        hipLaunchKernelGGL((k_ghost_axis<1, false>), g, dim3(GA_BS), 0, s, a);
        hipLaunchKernelGGL((k_ghost_axis<2, false>), g, dim3(GA_BS), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_me_guess(const ExxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_me_guess<SEA_LMAX>, dim3(a.n_pairs, a.n_chunks), dim3(GM_BS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_me_big(const ExxArgs& a, int nz_max, hipStream_t s) {
    hipLaunchKernelGGL(k_me_big, dim3(a.n_pairs, nz_max), dim3(GM_BS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_nn_sample(const ExxArgs& a, int D, float* out, double* s_out, int mode, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_sample<SEA_LMAX>, dim3(a.n_pairs, (D * D * D + NNS_BS - 1) / NNS_BS), dim3(NNS_BS), 0, s,
                       a, D, out, s_out, mode);
    return hipGetLastError();
}

hipError_t launch_nn_apply(const ExxArgs& a, int D, const float* y32, hipStream_t s) {
    if (D < 4) return hipErrorInvalidValue;   // the cubic map needs 4 network points per axis
    hipLaunchKernelGGL(k_nn_apply_ring, dim3(a.n_pairs, (64 + NA_ZC - 1) / NA_ZC), dim3(NA_BS), 0, s, a, D, y32);
    hipLaunchKernelGGL(k_nn_apply, dim3(a.n_pairs, a.n_chunks), dim3(GM_BS), 0, s, a, D, y32);
    return hipGetLastError();
}

hipError_t launch_cg(const ExxArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_f64, dim3(a.n_slots), dim3(CG_BS), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_energy_sum(const ExxArgs& a, double* out_scalars, double* e_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_sum, dim3(a.n_cells), dim3(ES_BS), 0, s, a, out_scalars, e_dev);
    return hipGetLastError();
}

void solid_harmonics_orthonormal_host(int lmax, double x, double y, double z, double* out) {
    double R[SEA_NMOM];
    racah_solid<SEA_LMAX>(x, y, z, R);
    for (int l = 0; l <= lmax; ++l)
        for (int m = -l; m <= l; ++m) out[l * l + l + m] = R[l * l + l + m] * racah_to_orthonormal(l, m);
}
