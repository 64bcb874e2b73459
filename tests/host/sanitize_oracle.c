/* The C oracle's entry points exercised under the address and
 * undefined-behaviour sanitizers on a small synthetic cell (two Gaussian
 * orbitals on a 24^3 grid): pair list, pair potentials and the multipole
 * start, the whole action with and without W boxes, epsilon boxes and
 * pairs, harmonics, moments, the stencil, CG and Cholesky.  Return codes and
 * finiteness are checked; the sanitizers check every access. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_fd_weights(int M, double *c);
int orc_build_pairs(const int32_t *N, const double *L, int n_occ, const double *cen, double r_pair,
                    double half_width, int cap, int32_t *pairs_out, double *origin_out, int *n_out);
void orc_real_ylm(int lmax, double x, double y, double z, double *out);
void orc_moments_points(int lmax, int n, const double *pos, const double *q, const double *o, double *Q);
double orc_me_eval(int lmax, const double *Q, const double *o, const double *t);
int orc_neg_lap_padded(const int32_t *n, const double *h, int M, const double *f, double *out);
int orc_cg(const int32_t *n, const double *h, int M, const double *b, double *x, double tol, int max_iter,
           double *info);
int orc_eps_boxes(const int32_t *N, int n_occ, const double *phi, double eps, int32_t *lo_out, int32_t *len_out);
int orc_eps_pairs(const int32_t *N, const double *L, int n_occ, const double *phi, const int32_t *lo,
                  const int32_t *len, double delta, int pad, int cap, int32_t *pairs_out, double *origin_out,
                  double *s_out, int32_t *dbox_out, int *n_out);
int orc_pair_potential(const int32_t *N, const double *L, int n_occ, const double *phi, const int32_t *pair,
                       const double *origin, int M, int lmax, double tol, int max_iter, const double *x0,
                       double *v_out, double *Q_out, double *info);
int orc_pair_me_start(const int32_t *N, const double *L, int n_occ, const double *phi, const int32_t *pair,
                      const double *origin, int lmax, double *out);
int orc_exx(const int32_t *N, const double *L, int n_occ, const double *phi, int n_pairs, const int32_t *pairs,
            const double *origins, const int32_t *dbox, int M, int lmax, double tol, int max_iter, int n_threads,
            double *W, double *e_pairs, int32_t *iters, double *relres, double *E_out);
int orc_cholesky(int n, const double *A, double *Lo);

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            printf("check failed at line %d: %s\n", __LINE__, #c);     \
            ++fails;                                                    \
        }                                                               \
    } while (0)

int main(void) {
    const int32_t N[3] = {24, 24, 24};
    const double L[3] = {7.2, 7.2, 7.2};
    const int n_occ = 2;
    const size_t Ng = (size_t)N[0] * N[1] * N[2];
    const double cen[6] = {3.0, 3.1, 3.2, 4.1, 3.6, 3.3};
    double *phi = malloc(sizeof(double) * n_occ * Ng);
    const double h = L[0] / N[0];
    for (int o = 0; o < n_occ; ++o) {
        double s = 0.0;
        for (int z = 0; z < N[2]; ++z)
            for (int y = 0; y < N[1]; ++y)
                for (int x = 0; x < N[0]; ++x) {
                    double d[3] = {x * h - cen[3 * o], y * h - cen[3 * o + 1], z * h - cen[3 * o + 2]};
                    double r2 = 0.0;
                    for (int a = 0; a < 3; ++a) {
                        d[a] -= L[a] * nearbyint(d[a] / L[a]);
                        r2 += d[a] * d[a];
                    }
                    const double v = (1.0 + 0.3 * d[0] - 0.2 * d[1]) * exp(-r2 / (2 * 0.64));
                    phi[o * Ng + ((size_t)z * N[1] + y) * N[0] + x] = v;
                    s += v * v;
                }
        for (size_t g = 0; g < Ng; ++g) phi[o * Ng + g] /= sqrt(s * h * h * h);
    }
    int32_t pairs[3 * 8];
    double org[3 * 3];
    int np = 0;
    CHECK(orc_build_pairs(N, L, n_occ, cen, 6.0, 2.0, 3, pairs, org, &np) == 0 && np == 3);
    CHECK(orc_build_pairs(N, L, n_occ, cen, 6.0, 2.0, 1, pairs, org, &np) == -2 && np == 3);
    CHECK(orc_build_pairs(N, L, n_occ, cen, 6.0, 2.0, 3, pairs, org, &np) == 0);
    const int32_t *pk = pairs + 8;
    const size_t nn = (size_t)pk[5] * pk[6] * pk[7];
    double *v = malloc(sizeof(double) * nn), *vme = malloc(sizeof(double) * nn), Q[49], info[8];
    CHECK(orc_pair_potential(N, L, n_occ, phi, pk, org + 3, 6, 6, 1e-10, 2000, NULL, v, Q, info) == 0);
    CHECK(isfinite(info[2]) && info[1] <= 1e-10);
    CHECK(orc_pair_me_start(N, L, n_occ, phi, pk, org + 3, 6, vme) == 0);
    CHECK(orc_pair_potential(N, L, n_occ, phi, pk, org + 3, 6, 6, 1e-10, 2000, vme, v, Q, info) == 0);
    double *W = malloc(sizeof(double) * n_occ * Ng), e[3], rr[3], E = 0.0;
    int32_t it[3];
    CHECK(orc_exx(N, L, n_occ, phi, np, pairs, org, NULL, 6, 6, 1e-8, 2000, 2, W, e, it, rr, &E) == 0);
    CHECK(isfinite(E) && E < 0.0);
    int32_t db[3 * 12];
    for (int p = 0; p < np; ++p)
        for (int s2 = 0; s2 < 2; ++s2)
            for (int a = 0; a < 3; ++a) {
                db[12 * p + 6 * s2 + a] = pairs[8 * p + 2 + a] - 2;
                db[12 * p + 6 * s2 + 3 + a] = pairs[8 * p + 5 + a] + 4;
            }
    CHECK(orc_exx(N, L, n_occ, phi, np, pairs, org, db, 6, 6, 1e-8, 2000, 2, W, e, it, rr, &E) == 0);
    int32_t lo[6], len[6];
    CHECK(orc_eps_boxes(N, n_occ, phi, 1e-3, lo, len) == 0);
    int32_t ep[8 * 3], edb[12 * 3];
    double eorg[9], es[3];
    int ne = 0;
    CHECK(orc_eps_pairs(N, L, n_occ, phi, lo, len, 1e-3, 2, 3, ep, eorg, es, edb, &ne) == 0 && ne >= 2);
    double Y[49], pos[9] = {0.1, 0.2, 0.3, -0.2, 0.1, 0.0, 0.3, -0.1, 0.2}, q[3] = {1.0, -0.5, 0.25}, o[3] = {0, 0, 0};
    orc_real_ylm(6, 0.3, -0.2, 0.1, Y);
    orc_real_ylm(6, 0.0, 0.0, 0.0, Y);
    orc_moments_points(6, 3, pos, q, o, Q);
    const double t[3] = {3.0, 1.0, -2.0};
    CHECK(isfinite(orc_me_eval(6, Q, o, t)));
    const int32_t n5[3] = {5, 6, 7};
    const double h3[3] = {0.2, 0.2, 0.2};
    double *f = calloc((5 + 12) * (6 + 12) * (7 + 12), sizeof(double)), *lap = malloc(sizeof(double) * 210);
    for (int k = 0; k < (5 + 12) * (6 + 12) * (7 + 12); ++k) f[k] = sin(0.01 * k);
    CHECK(orc_neg_lap_padded(n5, h3, 6, f, lap) == 0);
    double b[210], x[210] = {0};
    for (int k = 0; k < 210; ++k) b[k] = cos(0.1 * k);
    CHECK(orc_cg(n5, h3, 6, b, x, 1e-12, 1000, info) == 0 && info[1] <= 1e-12);
    double A[9] = {4, 1, 0.5, 1, 3, 0.2, 0.5, 0.2, 2}, Lo[9];
    CHECK(orc_cholesky(3, A, Lo) == 0);
    double Bad[4] = {1, 2, 2, 1};
    CHECK(orc_cholesky(2, Bad, Lo) != 0);
    double c[13];
    CHECK(orc_fd_weights(6, c) == 0 && orc_fd_weights(99, c) != 0);
    free(phi); free(v); free(vme); free(W); free(f); free(lap);
    printf("oracle: %d failures\n", fails);
    return fails ? 1 : 0;
}
