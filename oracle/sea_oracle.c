/*
 * sea_oracle.c - plain FP64 CPU oracle for the exact-exchange (exx) action on
 * localized orbitals and the ACE build of Ko et al., "High-Throughput
 * Condensed-Phase Hybrid DFT for Large-Scale Finite-Gap Systems: The SeA
 * Approach" (arXiv 2208.06097).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the benchmark's CPU
 * baseline leg do.  It shares no code, header or constant table with the GPU
 * library: every formula here is written out from the paper and from the
 * textbook definitions it relies on.
 *
 * What it computes, step by step (Sec. II.B, Eq. 8-14, plus the readings
 * listed in the design notes):
 *   pairs      keep (i<=j) when the minimum-image distance of the orbital
 *              centres is below r_pair (pair selection, Sec. II.B);
 *   domain     a cube of half-width w = ceil(half_width/h) points around the
 *              grid-snapped pair midpoint (domain truncation, Sec. II.B);
 *   rho_ij     phi_i * phi_j gathered with periodic (wrapped) indices (Eq. 8);
 *   Q_lm       h^3 sum rho r^l Y_lm(r - o), real orthonormal Y_lm, l <= 6
 *              (Eq. 11), Y_lm from associated Legendre functions and the
 *              azimuthal angle;
 *   boundary   v = 4 pi sum Q_lm Y_lm / ((2l+1) r^{l+1}) on the ghost layers
 *              the stencil reaches (Eq. 10);
 *   solve      -Lap_h v = 4 pi rho on the interior (Eq. 9) with the
 *              2M-th order central-difference Laplacian (M = 6 gives O(h^12),
 *              App. C), ghost values moved to the right-hand side, plain
 *              conjugate gradients to a relative true residual;
 *   energy     e_ij = h^3 sum rho v; E = -sum_i e_ii - 2 sum_{i<j} e_ij
 *              (Eq. 8 over ordered pairs);
 *   action     W_i += v phi_j and, for i != j, W_j += v phi_i on the pair
 *              domain (Eq. 13-14);
 *   eps rule   orbital boxes at 1 - eps coverage, pair boxes as their
 *              intersection, pairs screened by the absolute overlap
 *              (Eq. 16-17; readings at orc_eps_boxes);
 *   Cholesky   unblocked lower Cholesky of the symmetrized M (Eq. 18, App. A).
 *
 * Grid: point (ix,iy,iz) at (ix*hx, iy*hy, iz*hz), x fastest.  Orbital arrays
 * are orbital-major: phi[i*Ng + (iz*Ny + iy)*Nx + ix].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846
#define ORC_LMAX_CAP 12
#define ORC_MCAP 12

/* ---------------------------------------------------------------------- */
/* central-difference weights for the second derivative                    */
/* ---------------------------------------------------------------------- */

static double orc_fact(int n) {
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= (double)k;
    return f;
}

/* c[0..M]: f''(0) ~ h^-2 (c0 f(0) + sum_k c_k (f(k) + f(-k))).
 * Closed form of the order-2M central stencil:
 *   c_k = 2 (-1)^{k+1} (M!)^2 / (k^2 (M-k)! (M+k)!),  c_0 = -2 sum_k c_k. */
int orc_fd_weights(int M, double *c) {
    if (M < 1 || M > ORC_MCAP) return -1;
    double s = 0.0, mf = orc_fact(M);
    for (int k = 1; k <= M; ++k) {
        double sign = (k % 2 == 1) ? 1.0 : -1.0;
        c[k] = 2.0 * sign * mf * mf / ((double)k * k * orc_fact(M - k) * orc_fact(M + k));
        s += c[k];
    }
    c[0] = -2.0 * s;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* pair selection and domains                                              */
/* ---------------------------------------------------------------------- */

static double orc_minimg(double d, double L) {
    /* nearbyint rounds half to even (default rounding mode) */
    return d - L * nearbyint(d / L);
}

/* pairs_out: cap x 8 int32 {i, j, lo0, lo1, lo2, n0, n1, n2}; origin_out: cap x 3.
 * Returns 0, or -1 for bad arguments, -2 when cap is too small (n_out then
 * holds the count that would have been written). */
int orc_build_pairs(const int32_t *N, const double *L, int n_occ, const double *cen,
                    double r_pair, double half_width, int cap,
                    int32_t *pairs_out, double *origin_out, int *n_out) {
    if (n_occ < 0 || r_pair < 0.0 || half_width < 0.0) return -1;
    int cnt = 0;
    for (int i = 0; i < n_occ; ++i) {
        for (int j = i; j < n_occ; ++j) {
            double d[3], d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = orc_minimg(cen[3 * j + a] - cen[3 * i + a], L[a]);
                d2 += d[a] * d[a];
            }
            if (i != j && !(sqrt(d2) < r_pair)) continue;
            if (cnt < cap) {
                int32_t *o = pairs_out + 8 * cnt;
                o[0] = i;
                o[1] = j;
                for (int a = 0; a < 3; ++a) {
                    double h = L[a] / N[a];
                    double m = cen[3 * i + a] + 0.5 * d[a];
                    int kc = (int)floor(m / h + 0.5);
                    int w = (int)ceil(half_width / h - 1e-12);
                    o[2 + a] = kc - w;
                    o[5 + a] = 2 * w + 1;
                    origin_out[3 * cnt + a] = kc * h;
                }
            }
            ++cnt;
        }
    }
    *n_out = cnt;
    return cnt > cap ? -2 : 0;
}

/* ---------------------------------------------------------------------- */
/* real orthonormal spherical harmonics from Legendre functions            */
/* ---------------------------------------------------------------------- */

/* Associated Legendre P_l^m(x), 0 <= m <= l <= lmax, without the
 * Condon-Shortley phase, by the standard upward recurrences:
 *   P_m^m = (2m-1)!! (1-x^2)^{m/2},  P_{m+1}^m = x (2m+1) P_m^m,
 *   (l-m) P_l^m = x (2l-1) P_{l-1}^m - (l+m-1) P_{l-2}^m.
 * P[l*(lmax+1)+m]. */
static void orc_legendre(int lmax, double x, double *P) {
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;
    for (int m = 0; m <= lmax; ++m) {
        if (m > 0) pmm *= (2.0 * m - 1.0) * s;
        P[m * (lmax + 1) + m] = pmm;
        if (m + 1 <= lmax) P[(m + 1) * (lmax + 1) + m] = x * (2.0 * m + 1.0) * pmm;
        for (int l = m + 2; l <= lmax; ++l)
            P[l * (lmax + 1) + m] = (x * (2.0 * l - 1.0) * P[(l - 1) * (lmax + 1) + m]
                                    - (l + m - 1.0) * P[(l - 2) * (lmax + 1) + m]) / (double)(l - m);
    }
}

/* out[l*l + l + m], m = -l..l: real orthonormal Y_lm at the direction of
 * (x, y, z) (any nonzero length); m > 0 uses cos(m phi), m < 0 uses
 * sin(|m| phi), both with sqrt(2) N_lm, N_lm^2 = (2l+1)/(4 pi) (l-m)!/(l+m)!.
 * At the origin only Y_00 is defined; higher l are set to 0. */
void orc_real_ylm(int lmax, double x, double y, double z, double *out) {
    double P[(ORC_LMAX_CAP + 1) * (ORC_LMAX_CAP + 1)];
    double r = sqrt(x * x + y * y + z * z);
    if (r == 0.0) {
        for (int k = 0; k < (lmax + 1) * (lmax + 1); ++k) out[k] = 0.0;
        out[0] = 1.0 / sqrt(4.0 * ORC_PI);
        return;
    }
    double ct = z / r, phi = atan2(y, x);
    orc_legendre(lmax, ct, P);
    for (int l = 0; l <= lmax; ++l) {
        for (int m = 0; m <= l; ++m) {
            double nlm = sqrt((2.0 * l + 1.0) / (4.0 * ORC_PI) * orc_fact(l - m) / orc_fact(l + m));
            double plm = P[l * (lmax + 1) + m];
            if (m == 0) {
                out[l * l + l] = nlm * plm;
            } else {
                out[l * l + l + m] = sqrt(2.0) * nlm * plm * cos(m * phi);
                out[l * l + l - m] = sqrt(2.0) * nlm * plm * sin(m * phi);
            }
        }
    }
}

/* Multipole moments of point charges: Q_lm = sum_k q_k r_k^l Y_lm(r_k - o). */
void orc_moments_points(int lmax, int n, const double *pos, const double *q,
                        const double *o, double *Q) {
    int nlm = (lmax + 1) * (lmax + 1);
    double Y[(ORC_LMAX_CAP + 1) * (ORC_LMAX_CAP + 1)];
    for (int k = 0; k < nlm; ++k) Q[k] = 0.0;
    for (int c = 0; c < n; ++c) {
        double dx = pos[3 * c] - o[0], dy = pos[3 * c + 1] - o[1], dz = pos[3 * c + 2] - o[2];
        double r = sqrt(dx * dx + dy * dy + dz * dz);
        orc_real_ylm(lmax, dx, dy, dz, Y);
        for (int l = 0; l <= lmax; ++l) {
            double rl = pow(r, l);
            for (int m = -l; m <= l; ++m) Q[l * l + l + m] += q[c] * rl * Y[l * l + l + m];
        }
    }
}

/* Far-field potential of the expansion (Eq. 10) at target t. */
double orc_me_eval(int lmax, const double *Q, const double *o, const double *t) {
    double Y[(ORC_LMAX_CAP + 1) * (ORC_LMAX_CAP + 1)];
    double dx = t[0] - o[0], dy = t[1] - o[1], dz = t[2] - o[2];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    orc_real_ylm(lmax, dx, dy, dz, Y);
    double v = 0.0;
    for (int l = 0; l <= lmax; ++l) {
        double acc = 0.0;
        for (int m = -l; m <= l; ++m) acc += Q[l * l + l + m] * Y[l * l + l + m];
        v += 4.0 * ORC_PI * acc / ((2.0 * l + 1.0) * pow(r, l + 1));
    }
    return v;
}

/* ---------------------------------------------------------------------- */
/* the discrete operator -Lap_h                                            */
/* ---------------------------------------------------------------------- */

/* out = -Lap_h f on an interior of n[0] x n[1] x n[2] points, with f given on
 * the padded box (n + 2M per axis, x fastest) so every stencil tap exists. */
int orc_neg_lap_padded(const int32_t *n, const double *h, int M, const double *f, double *out) {
    double c[ORC_MCAP + 1];
    if (orc_fd_weights(M, c)) return -1;
    int px = n[0] + 2 * M, py = n[1] + 2 * M;
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                size_t ctr = ((size_t)(z + M) * py + (y + M)) * px + (x + M);
                double s = 0.0;
                double hh[3] = {1.0 / (h[0] * h[0]), 1.0 / (h[1] * h[1]), 1.0 / (h[2] * h[2])};
                size_t stride[3] = {1, (size_t)px, (size_t)px * py};
                for (int a = 0; a < 3; ++a) {
                    double t = c[0] * f[ctr];
                    for (int k = 1; k <= M; ++k)
                        t += c[k] * (f[ctr + k * stride[a]] + f[ctr - k * stride[a]]);
                    s += hh[a] * t;
                }
                out[((size_t)z * n[1] + y) * n[0] + x] = -s;
            }
    return 0;
}

/* y = A x for the interior operator (zero values outside the interior). */
static void orc_apply_A(const int32_t *n, const double *h, int M, const double *c,
                        const double *x, double *pad, double *y) {
    int px = n[0] + 2 * M, py = n[1] + 2 * M, pz = n[2] + 2 * M;
    memset(pad, 0, sizeof(double) * (size_t)px * py * pz);
    for (int z = 0; z < n[2]; ++z)
        for (int yy = 0; yy < n[1]; ++yy)
            memcpy(pad + ((size_t)(z + M) * py + (yy + M)) * px + M,
                   x + ((size_t)z * n[1] + yy) * n[0], sizeof(double) * n[0]);
    double hh[3] = {1.0 / (h[0] * h[0]), 1.0 / (h[1] * h[1]), 1.0 / (h[2] * h[2])};
    size_t stride[3] = {1, (size_t)px, (size_t)px * py};
    for (int z = 0; z < n[2]; ++z)
        for (int yy = 0; yy < n[1]; ++yy)
            for (int xx = 0; xx < n[0]; ++xx) {
                size_t ctr = ((size_t)(z + M) * py + (yy + M)) * px + (xx + M);
                double s = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double t = c[0] * pad[ctr];
                    for (int k = 1; k <= M; ++k)
                        t += c[k] * (pad[ctr + k * stride[a]] + pad[ctr - k * stride[a]]);
                    s += hh[a] * t;
                }
                y[((size_t)z * n[1] + yy) * n[0] + xx] = -s;
            }
}

static double orc_dot(size_t n, const double *a, const double *b) {
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) s += a[k] * b[k];
    return s;
}

/* Plain conjugate gradients for A x = b (A = -Lap_h with zero Dirichlet
 * values outside the interior).  x holds the start on entry and the solution
 * on exit.  Stops when the recursively updated residual satisfies
 * |r| <= tol |b|; the true residual b - A x is then recomputed and, if it
 * does not meet the bar, the iteration restarts from it.
 * info[0] = iterations, info[1] = final true relative residual.
 * Returns 0 when converged, 1 when max_iter was reached, -1 on bad input. */
int orc_cg(const int32_t *n, const double *h, int M, const double *b, double *x,
           double tol, int max_iter, double *info) {
    double c[ORC_MCAP + 1];
    if (orc_fd_weights(M, c)) return -1;
    size_t nn = (size_t)n[0] * n[1] * n[2];
    size_t npad = (size_t)(n[0] + 2 * M) * (n[1] + 2 * M) * (n[2] + 2 * M);
    double *r = malloc(sizeof(double) * nn), *p = malloc(sizeof(double) * nn);
    double *q = malloc(sizeof(double) * nn), *pad = malloc(sizeof(double) * npad);
    double bnorm = sqrt(orc_dot(nn, b, b));
    int it = 0, status = 1;
    double rel = 0.0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * nn);
        status = 0;
        goto done;
    }
    for (;;) {
        /* (re)start from the true residual */
        orc_apply_A(n, h, M, c, x, pad, q);
        for (size_t k = 0; k < nn; ++k) { r[k] = b[k] - q[k]; p[k] = r[k]; }
        double rr = orc_dot(nn, r, r);
        rel = sqrt(rr) / bnorm;
        if (rel <= tol) { status = 0; break; }
        if (it >= max_iter) break;
        while (it < max_iter) {
            orc_apply_A(n, h, M, c, p, pad, q);
            double alpha = rr / orc_dot(nn, p, q);
            for (size_t k = 0; k < nn; ++k) { x[k] += alpha * p[k]; r[k] -= alpha * q[k]; }
            double rr_new = orc_dot(nn, r, r);
            ++it;
            if (sqrt(rr_new) <= tol * bnorm) break;
            double beta = rr_new / rr;
            for (size_t k = 0; k < nn; ++k) p[k] = r[k] + beta * p[k];
            rr = rr_new;
        }
    }
done:
    info[0] = it;
    info[1] = rel;
    free(r); free(p); free(q); free(pad);
    return status;
}

/* ---------------------------------------------------------------------- */
/* one pair: gather, moments, boundary, solve, energy                      */
/* ---------------------------------------------------------------------- */

static inline int orc_wrap(int k, int N) {
    int m = k % N;
    return m < 0 ? m + N : m;
}

/* ---- epsilon-driven domains and pair screening (Eq. 16-17) --------------
 *
 * Omega_ii (Eq. 16) is a box on the grid that holds at least 1 - eps of
 * |phi_i|^2.  Reading: per axis, the shortest cyclic run of grid indices
 * whose marginal mass (sum of |phi_i|^2 over the other two axes) is at least
 * (1 - eps/3) of the orbital's total; among runs of that length the one with
 * the largest mass, then the smallest start.  The mass outside the product
 * box is at most the sum of the three per-axis tails, i.e. at most eps.
 * lo_out[3i+a] in [0, N[a]), len_out[3i+a] in [1, N[a]]. */
int orc_eps_boxes(const int32_t *N, int n_occ, const double *phi, double eps, int32_t *lo_out,
                  int32_t *len_out) {
    if (n_occ < 0 || !(eps >= 0.0) || !(eps < 1.0)) return -1;
    const size_t Ng = (size_t)N[0] * N[1] * N[2];
    int nmax = N[0] > N[1] ? N[0] : N[1];
    nmax = nmax > N[2] ? nmax : N[2];
    double *m = (double *)malloc(sizeof(double) * nmax);
    if (!m) return -3;
    for (int i = 0; i < n_occ; ++i) {
        const double *f = phi + (size_t)i * Ng;
        for (int a = 0; a < 3; ++a) {
            for (int k = 0; k < N[a]; ++k) m[k] = 0.0;
            for (int iz = 0; iz < N[2]; ++iz)
                for (int iy = 0; iy < N[1]; ++iy)
                    for (int ix = 0; ix < N[0]; ++ix) {
                        const double v = f[((size_t)iz * N[1] + iy) * N[0] + ix];
                        const int k = a == 0 ? ix : (a == 1 ? iy : iz);
                        m[k] += v * v;
                    }
            double T = 0.0;
            for (int k = 0; k < N[a]; ++k) T += m[k];
            const double target = (1.0 - eps / 3.0) * T;
            int best_s = 0, best_len = N[a];
            for (int len = 1; len < N[a]; ++len) {
                int found = 0;
                double best_mass = -1.0;
                for (int s0 = 0; s0 < N[a]; ++s0) {
                    double mass = 0.0;
                    for (int t = 0; t < len; ++t) mass += m[(s0 + t) % N[a]];
                    if (mass >= target && mass > best_mass) {
                        best_mass = mass;
                        best_s = s0;
                        found = 1;
                    }
                }
                if (found) {
                    best_len = len;
                    break;
                }
            }
            if (best_len == N[a]) best_s = 0;
            lo_out[3 * i + a] = best_s;
            len_out[3 * i + a] = best_len;
        }
    }
    free(m);
    return 0;
}

/* Intersection of two cyclic index runs [a, a+la) and [b, b+lb) on Z_N.
 * A run of length N is the whole axis.  When the intersection has two
 * pieces (runs longer than half the axis), the longer piece is kept (the
 * first one on a tie).  Returns the length (0 if empty) and the start,
 * unwrapped so that it lies in [a, a + la). */
static int orc_cyc_intersect(int a, int la, int b, int lb, int N, int *start) {
    if (la >= N) {
        *start = b;
        return lb;
    }
    if (lb >= N) {
        *start = a;
        return la;
    }
    int best = 0;
    for (int k = -1; k <= 1; ++k) {
        const int s = a > b + k * N ? a : b + k * N;
        const int e = a + la < b + k * N + lb ? a + la : b + k * N + lb;
        if (e - s > best) {
            best = e - s;
            *start = s;
        }
    }
    return best;
}

/* Pair domains Omega_ij = Omega_ii intersect Omega_jj and pair screening
 * (Eq. 17): keep (i <= j) when the intersection is non-empty on every axis
 * and S_ij = h^3 sum over Omega_ij of |phi_i phi_j| >= delta (wrapped
 * indices).  The box written out (where rho_ij is taken and the Poisson
 * equation solved) is Omega_ij grown by `pad` points on each side, at most
 * the cell per axis (reading: the paper leaves the margin between the pair
 * density and the multipole boundary open).  Output as orc_build_pairs,
 * plus S per kept pair; the multipole origin is the box centre,
 * (lo + (n - 1)/2) h per axis. */
/* Box of an orbital run shifted by a multiple of N to lie nearest (by its
 * centre) to the reference start r0 with length rn. */
static int orc_near_start(int lo, int ln, int r0, int rn, int N) {
    int best = lo, bd = -1;
    for (int k = -1; k <= 1; ++k) {
        const int c2 = 2 * (lo + k * N) + ln, r2 = 2 * r0 + rn;
        const int d = c2 > r2 ? c2 - r2 : r2 - c2;
        if (bd < 0 || d < bd) {
            bd = d;
            best = lo + k * N;
        }
    }
    return best;
}

int orc_eps_pairs(const int32_t *N, const double *L, int n_occ, const double *phi, const int32_t *lo,
                  const int32_t *len, double delta, int pad, int cap, int32_t *pairs_out, double *origin_out,
                  double *s_out, int32_t *dbox_out, int *n_out) {
    if (n_occ < 0) return -1;
    const size_t Ng = (size_t)N[0] * N[1] * N[2];
    double h[3];
    for (int a = 0; a < 3; ++a) h[a] = L[a] / N[a];
    const double dV = h[0] * h[1] * h[2];
    int cnt = 0;
    for (int i = 0; i < n_occ; ++i) {
        for (int j = i; j < n_occ; ++j) {
            int st[3] = {0, 0, 0}, n[3], empty = 0;
            for (int a = 0; a < 3; ++a) {
                n[a] = orc_cyc_intersect(lo[3 * i + a], len[3 * i + a], lo[3 * j + a], len[3 * j + a], N[a], &st[a]);
                if (n[a] == 0) empty = 1;
            }
            if (empty) continue;
            double S = 0.0;
            for (int z = 0; z < n[2]; ++z)
                for (int y = 0; y < n[1]; ++y)
                    for (int x = 0; x < n[0]; ++x) {
                        const size_t g = ((size_t)orc_wrap(st[2] + z, N[2]) * N[1] + orc_wrap(st[1] + y, N[1])) * N[0] +
                                         orc_wrap(st[0] + x, N[0]);
                        S += fabs(phi[(size_t)i * Ng + g] * phi[(size_t)j * Ng + g]);
                    }
            S *= dV;
            if (!(S >= delta)) continue;
            if (cnt < cap) {
                int32_t *o = pairs_out + 8 * cnt;
                o[0] = i;
                o[1] = j;
                for (int a = 0; a < 3; ++a) {
                    /* solve box: Omega_ij grown by pad points a side, at most the cell */
                    int np = n[a] + 2 * pad;
                    if (np > N[a]) np = N[a];
                    const int sp = st[a] - (np - n[a]) / 2;
                    o[2 + a] = sp;
                    o[5 + a] = np;
                    origin_out[3 * cnt + a] = (sp + 0.5 * (np - 1)) * h[a];
                }
                s_out[cnt] = S;
                if (dbox_out) {
                    /* boxes where W takes this pair (the paper's Omega^D): for
                     * W_i the box of phi_j (i != j) or Omega_ii doubled about its
                     * centre (i == j); for W_j the box of phi_i; each placed in
                     * the frame of the pair's domain and grown to cover it */
                    int32_t *d = dbox_out + 12 * cnt;
                    for (int a = 0; a < 3; ++a) {
                        int l0, n0;
                        if (i == j) {
                            n0 = 2 * len[3 * i + a] < N[a] ? 2 * len[3 * i + a] : N[a];
                            l0 = lo[3 * i + a] - (n0 - len[3 * i + a]) / 2;
                        } else {
                            n0 = len[3 * j + a];
                            l0 = lo[3 * j + a];
                        }
                        d[a] = orc_near_start(l0, n0, o[2 + a], o[5 + a], N[a]);
                        d[3 + a] = n0;
                        d[6 + a] = orc_near_start(lo[3 * i + a], len[3 * i + a], o[2 + a], o[5 + a], N[a]);
                        d[9 + a] = len[3 * i + a];
                        /* each box also covers the pair's domain, so that W takes
                         * the pair wherever e_ij does (at most the cell) */
                        for (int sd = 0; sd < 2; ++sd) {
                            int32_t *bl = d + 6 * sd + a, *bn = d + 6 * sd + 3 + a;
                            const int l1 = *bl < o[2 + a] ? *bl : o[2 + a];
                            const int e1 = *bl + *bn > o[2 + a] + o[5 + a] ? *bl + *bn : o[2 + a] + o[5 + a];
                            *bl = l1;
                            *bn = e1 - l1 < N[a] ? e1 - l1 : N[a];
                        }
                    }
                }
            }
            ++cnt;
        }
    }
    *n_out = cnt;
    return cnt > cap ? -2 : 0;
}

/* v_out: n0*n1*n2 interior potential.  info (8 doubles): iterations,
 * true relative residual, e_ij, S_abs = h^3 sum |rho|, q = h^3 sum rho,
 * |b|_2, status.  x0 (nullable) is the CG start on the interior. */
int orc_pair_potential(const int32_t *N, const double *L, int n_occ, const double *phi,
                       const int32_t *pair, const double *origin, int M, int lmax,
                       double tol, int max_iter, const double *x0, double *v_out,
                       double *Q_out, double *info) {
    int i = pair[0], j = pair[1];
    const int32_t *lo = pair + 2, *n = pair + 5;
    if (i < 0 || j < i || j >= n_occ || n[0] < 1 || n[1] < 1 || n[2] < 1 || lmax > ORC_LMAX_CAP)
        return -1;
    double c[ORC_MCAP + 1];
    if (orc_fd_weights(M, c)) return -1;
    double h[3] = {L[0] / N[0], L[1] / N[1], L[2] / N[2]};
    double dV = h[0] * h[1] * h[2];
    size_t Ng = (size_t)N[0] * N[1] * N[2];
    size_t nn = (size_t)n[0] * n[1] * n[2];
    int nlm = (lmax + 1) * (lmax + 1);
    double *rho = malloc(sizeof(double) * nn), *b = malloc(sizeof(double) * nn);
    double Q[(ORC_LMAX_CAP + 1) * (ORC_LMAX_CAP + 1)], Y[(ORC_LMAX_CAP + 1) * (ORC_LMAX_CAP + 1)];
    const double *pi_ = phi + (size_t)i * Ng, *pj_ = phi + (size_t)j * Ng;

    /* pair density on the interior (Eq. 8), wrapped indices */
    double sabs = 0.0, qsum = 0.0;
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                size_t g = ((size_t)orc_wrap(lo[2] + z, N[2]) * N[1] + orc_wrap(lo[1] + y, N[1])) * N[0]
                           + orc_wrap(lo[0] + x, N[0]);
                double r = pi_[g] * pj_[g];
                rho[((size_t)z * n[1] + y) * n[0] + x] = r;
                sabs += fabs(r);
                qsum += r;
            }

    /* moments (Eq. 11) about the domain origin */
    for (int k = 0; k < nlm; ++k) Q[k] = 0.0;
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                double dx = (lo[0] + x) * h[0] - origin[0];
                double dy = (lo[1] + y) * h[1] - origin[1];
                double dz = (lo[2] + z) * h[2] - origin[2];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                double rv = rho[((size_t)z * n[1] + y) * n[0] + x];
                orc_real_ylm(lmax, dx, dy, dz, Y);
                for (int l = 0; l <= lmax; ++l) {
                    double rl = pow(r, l);
                    for (int m = -l; m <= l; ++m) Q[l * l + l + m] += rv * rl * Y[l * l + l + m];
                }
            }
    for (int k = 0; k < nlm; ++k) Q[k] *= dV;
    if (Q_out) memcpy(Q_out, Q, sizeof(double) * nlm);

    /* right-hand side 4 pi rho plus the known ghost values (Eq. 9-10) */
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                size_t id = ((size_t)z * n[1] + y) * n[0] + x;
                double acc = 4.0 * ORC_PI * rho[id];
                int pos[3] = {x, y, z};
                for (int a = 0; a < 3; ++a)
                    for (int k = 1; k <= M; ++k)
                        for (int s = -1; s <= 1; s += 2) {
                            int q = pos[a] + s * k;
                            if (q >= 0 && q < n[a]) continue;
                            int gp[3] = {x, y, z};
                            gp[a] = q;
                            double t[3] = {(lo[0] + gp[0]) * h[0], (lo[1] + gp[1]) * h[1],
                                           (lo[2] + gp[2]) * h[2]};
                            acc += c[k] / (h[a] * h[a]) * orc_me_eval(lmax, Q, origin, t);
                        }
                b[id] = acc;
            }

    /* CG (Eq. 9) */
    if (x0) memcpy(v_out, x0, sizeof(double) * nn);
    else memset(v_out, 0, sizeof(double) * nn);
    double cg_info[2];
    int st = orc_cg(n, h, M, b, v_out, tol, max_iter, cg_info);

    double e = 0.0;
    for (size_t k = 0; k < nn; ++k) e += rho[k] * v_out[k];
    info[0] = cg_info[0];
    info[1] = cg_info[1];
    info[2] = dV * e;
    info[3] = dV * sabs;
    info[4] = dV * qsum;
    info[5] = sqrt(orc_dot(nn, b, b));
    info[6] = st;
    info[7] = 0.0;
    free(rho); free(b);
    return st;
}

/* Regularized multipole start v_ME of pair `pair` on its interior (the
 * initial guess of the CG of Eq. 9 that the multipole and learned starts
 * use; the paper leaves the guess open, so this follows the reading in the
 * design notes).  The expansion of Eq. 10 diverges inside the charge; here
 *   v_ME(p) = q erf(r / r_s) / r
 *           + sum_{l=1..lmax} (1 - exp(-r^2 / r_s^2))^{l+1}
 *                             4 pi / (2l+1) sum_m Q_lm Y_lm(p - o) / r^{l+1},
 * r = |p - o|, q = h^3 sum rho, Q_lm of Eq. 11 about the domain origin o, and
 * r_s = sqrt(2 <r^2> / 3) with <r^2> = sum |rho| r^2 / sum |rho| (the width
 * of a spherical Gaussian charge exp(-r^2 / r_s^2), whose potential the
 * l = 0 term then is exactly).  At r = 0 the l = 0 term is its limit
 * 2 q / (r_s sqrt(pi)) and the damped terms vanish.  Returns -1 on bad input. */
int orc_pair_me_start(const int32_t *N, const double *L, int n_occ, const double *phi,
                      const int32_t *pair, const double *origin, int lmax, double *out) {
    int i = pair[0], j = pair[1];
    const int32_t *lo = pair + 2, *n = pair + 5;
    if (i < 0 || j < i || j >= n_occ || n[0] < 1 || n[1] < 1 || n[2] < 1 || lmax > ORC_LMAX_CAP) return -1;
    double h[3] = {L[0] / N[0], L[1] / N[1], L[2] / N[2]};
    double dV = h[0] * h[1] * h[2];
    size_t Ng = (size_t)N[0] * N[1] * N[2];
    size_t nn = (size_t)n[0] * n[1] * n[2];
    int nlm = (lmax + 1) * (lmax + 1);
    double *rho = malloc(sizeof(double) * nn);
    double Q[(ORC_LMAX_CAP + 1) * (ORC_LMAX_CAP + 1)], Y[(ORC_LMAX_CAP + 1) * (ORC_LMAX_CAP + 1)];
    const double *pi_ = phi + (size_t)i * Ng, *pj_ = phi + (size_t)j * Ng;
    for (int k = 0; k < nlm; ++k) Q[k] = 0.0;
    double sabs = 0.0, m2 = 0.0, qsum = 0.0;
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                size_t g = ((size_t)orc_wrap(lo[2] + z, N[2]) * N[1] + orc_wrap(lo[1] + y, N[1])) * N[0]
                           + orc_wrap(lo[0] + x, N[0]);
                double rv = pi_[g] * pj_[g];
                rho[((size_t)z * n[1] + y) * n[0] + x] = rv;
                double dx = (lo[0] + x) * h[0] - origin[0];
                double dy = (lo[1] + y) * h[1] - origin[1];
                double dz = (lo[2] + z) * h[2] - origin[2];
                double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
                sabs += fabs(rv);
                m2 += fabs(rv) * r2;
                qsum += rv;
                orc_real_ylm(lmax, dx, dy, dz, Y);
                for (int l = 0; l <= lmax; ++l) {
                    double rl = pow(r, l);
                    for (int m = -l; m <= l; ++m) Q[l * l + l + m] += rv * rl * Y[l * l + l + m];
                }
            }
    for (int k = 0; k < nlm; ++k) Q[k] *= dV;
    double q = dV * qsum;
    double rs = sqrt(sabs > 0.0 ? fmax(2.0 * (m2 / sabs) / 3.0, 1e-6) : 2.0 / 3.0);
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                double dx = (lo[0] + x) * h[0] - origin[0];
                double dy = (lo[1] + y) * h[1] - origin[1];
                double dz = (lo[2] + z) * h[2] - origin[2];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                double v;
                if (r == 0.0) {
                    v = 2.0 * q / (rs * sqrt(ORC_PI));
                } else {
                    v = q * erf(r / rs) / r;
                    double damp = 1.0 - exp(-(r * r) / (rs * rs));
                    orc_real_ylm(lmax, dx, dy, dz, Y);
                    for (int l = 1; l <= lmax; ++l) {
                        double acc = 0.0;
                        for (int m = -l; m <= l; ++m) acc += Q[l * l + l + m] * Y[l * l + l + m];
                        v += pow(damp, l + 1) * 4.0 * ORC_PI * acc / ((2.0 * l + 1.0) * pow(r, l + 1));
                    }
                }
                out[((size_t)z * n[1] + y) * n[0] + x] = v;
            }
    free(rho);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* the whole action: all pairs, then the scatter in pair order             */
/* ---------------------------------------------------------------------- */

/* W (n_occ x Ng) is overwritten.  e_pairs, iters, relres: per pair.
 * E_out: Eq. 8 energy.  Pairs are solved in parallel; the scatter runs in
 * pair order afterwards so the result does not depend on the thread count.
 * Returns the number of pairs that did not converge, or -1 on bad input. */
int orc_exx(const int32_t *N, const double *L, int n_occ, const double *phi, int n_pairs,
            const int32_t *pairs, const double *origins, const int32_t *dbox, int M, int lmax,
            double tol, int max_iter, int n_threads, double *W, double *e_pairs, int32_t *iters,
            double *relres, double *E_out) {
    size_t Ng = (size_t)N[0] * N[1] * N[2];
    for (int p = 0; p < n_pairs; ++p) {
        const int32_t *pp = pairs + 8 * p;
        if (pp[0] < 0 || pp[1] < pp[0] || pp[1] >= n_occ) return -1;
    }
    size_t *off = malloc(sizeof(size_t) * (n_pairs + 1));
    off[0] = 0;
    for (int p = 0; p < n_pairs; ++p) {
        const int32_t *n = pairs + 8 * p + 5;
        off[p + 1] = off[p] + (size_t)n[0] * n[1] * n[2];
    }
    double *v = malloc(sizeof(double) * (off[n_pairs] ? off[n_pairs] : 1));
    const int nq = (lmax + 1) * (lmax + 1);
    double *Qall = malloc(sizeof(double) * (size_t)nq * (n_pairs ? n_pairs : 1));
    int bad = 0;
#ifdef _OPENMP
    if (n_threads > 0) omp_set_num_threads(n_threads);
#endif
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int p = 0; p < n_pairs; ++p) {
        double info[8];
        int st = orc_pair_potential(N, L, n_occ, phi, pairs + 8 * p, origins + 3 * p, M, lmax,
                                    tol, max_iter, NULL, v + off[p], Qall + (size_t)nq * p, info);
        e_pairs[p] = info[2];
        iters[p] = (int32_t)info[0];
        relres[p] = info[1];
        if (st != 0) bad += 1;
    }
    memset(W, 0, sizeof(double) * Ng * n_occ);
    double E = 0.0;
    double h[3];
    for (int a = 0; a < 3; ++a) h[a] = L[a] / N[a];
    for (int p = 0; p < n_pairs; ++p) {
        const int32_t *pp = pairs + 8 * p;
        int i = pp[0], j = pp[1];
        const int32_t *lo = pp + 2, *n = pp + 5;
        const double *vp = v + off[p];
        if (!dbox) {
            /* W on the pair's own domain */
            for (int z = 0; z < n[2]; ++z)
                for (int y = 0; y < n[1]; ++y)
                    for (int x = 0; x < n[0]; ++x) {
                        size_t g = ((size_t)orc_wrap(lo[2] + z, N[2]) * N[1] + orc_wrap(lo[1] + y, N[1])) * N[0]
                                   + orc_wrap(lo[0] + x, N[0]);
                        double vv = vp[((size_t)z * n[1] + y) * n[0] + x];
                        W[(size_t)i * Ng + g] += vv * phi[(size_t)j * Ng + g];
                        if (i != j) W[(size_t)j * Ng + g] += vv * phi[(size_t)i * Ng + g];
                    }
        } else {
            /* W_i += v phi_j on box side 0 and, for i != j, W_j += v phi_i on
             * box side 1; v is the solution inside the pair's domain and the
             * multipole potential (Eq. 10) outside it */
            for (int side = 0; side < (i == j ? 1 : 2); ++side) {
                const int32_t *dl = dbox + 12 * p + 6 * side, *dn = dl + 3;
                const int o = side == 0 ? i : j, q = side == 0 ? j : i;
                for (int z = 0; z < dn[2]; ++z)
                    for (int y = 0; y < dn[1]; ++y)
                        for (int x = 0; x < dn[0]; ++x) {
                            const int P3[3] = {dl[0] + x, dl[1] + y, dl[2] + z};
                            const int s0 = P3[0] - lo[0], s1 = P3[1] - lo[1], s2 = P3[2] - lo[2];
                            double vv;
                            if (s0 >= 0 && s0 < n[0] && s1 >= 0 && s1 < n[1] && s2 >= 0 && s2 < n[2]) {
                                vv = vp[((size_t)s2 * n[1] + s1) * n[0] + s0];
                            } else {
                                const double t[3] = {P3[0] * h[0], P3[1] * h[1], P3[2] * h[2]};
                                vv = orc_me_eval(lmax, Qall + (size_t)nq * p, origins + 3 * p, t);
                            }
                            size_t g = ((size_t)orc_wrap(P3[2], N[2]) * N[1] + orc_wrap(P3[1], N[1])) * N[0] +
                                       orc_wrap(P3[0], N[0]);
                            W[(size_t)o * Ng + g] += vv * phi[(size_t)q * Ng + g];
                        }
            }
        }
        E -= (i == j ? 1.0 : 2.0) * e_pairs[p];
    }
    *E_out = E;
    free(v); free(off); free(Qall);
    return bad;
}

/* ---------------------------------------------------------------------- */
/* ACE: unblocked Cholesky of a symmetric matrix                           */
/* ---------------------------------------------------------------------- */

/* A (n x n, row-major, only the lower triangle is read) = L L^T, L lower,
 * positive diagonal; the upper triangle of L is zeroed.  Returns 0, or k+1
 * when the k-th pivot is not positive (matrix not positive definite). */
int orc_cholesky(int n, const double *A, double *Lo) {
    memset(Lo, 0, sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j) {
        double d = A[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= Lo[(size_t)j * n + k] * Lo[(size_t)j * n + k];
        if (!(d > 0.0)) return j + 1;
        double ljj = sqrt(d);
        Lo[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double s = A[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= Lo[(size_t)i * n + k] * Lo[(size_t)j * n + k];
            Lo[(size_t)i * n + j] = s / ljj;
        }
    }
    return 0;
}
