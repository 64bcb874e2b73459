// Host geometry of the library (pair list and cube domains, epsilon-box run
// search, cyclic intersections) exercised under the address and
// undefined-behaviour sanitizers: random cells, caps smaller and larger than
// the pair count, and marginals of every shape, checked against brute force.
#include <cstdio>
#include <random>
#include <vector>

#include "host_geometry.h"

static int fails = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("check failed at line %d: %s\n", __LINE__, #c); \
            ++fails;                                                    \
        }                                                               \
    } while (0)

int main() {
    std::mt19937 rng(12345);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (int it = 0; it < 300; ++it) {
        const int n_occ = rng() % 41;
        int32_t n[3];
        double L[3];
        for (int a = 0; a < 3; ++a) {
            n[a] = 8 + rng() % 120;
            L[a] = 5.0 + 30.0 * U(rng);
        }
        std::vector<double> c(3 * (n_occ > 0 ? n_occ : 1));
        for (int k = 0; k < 3 * n_occ; ++k) c[k] = (U(rng) * 3.0 - 1.0) * L[k % 3];
        const double rp = 8.0 * U(rng), hw = 6.0 * U(rng);
        const int total = host_build_pairs(n, L, n_occ, c.data(), rp, hw, nullptr, 0);
        std::vector<sea_pair> out(total + 1);
        const int cap = total > 0 ? (int)(rng() % (total + 1)) : 0;
        CHECK(host_build_pairs(n, L, n_occ, c.data(), rp, hw, out.data(), cap) == total);
        std::vector<sea_pair> all(total + 1);
        CHECK(host_build_pairs(n, L, n_occ, c.data(), rp, hw, all.data(), total) == total);
        int brute = 0;
        for (int i = 0; i < n_occ; ++i)
            for (int j = i; j < n_occ; ++j) {
                double d2 = 0.0;
                for (int a = 0; a < 3; ++a) {
                    double d = c[3 * j + a] - c[3 * i + a];
                    d -= L[a] * std::nearbyint(d / L[a]);
                    d2 += d * d;
                }
                if (i == j || std::sqrt(d2) < rp) ++brute;
            }
        CHECK(brute == total);
        for (int k = 0; k < total; ++k) {
            CHECK(all[k].i <= all[k].j && all[k].j < n_occ);
            for (int a = 0; a < 3; ++a) CHECK(all[k].n[a] % 2 == 1 && all[k].n[a] >= 1);
        }
    }
    for (int it = 0; it < 2000; ++it) {
        const int N = 1 + rng() % 70;
        std::vector<double> m(N);
        const int kind = rng() % 3;
        for (int k = 0; k < N; ++k) m[k] = kind == 0 ? U(rng) : (kind == 1 ? (k == (int)(rng() % N) ? 1.0 : 0.0) : 0.0);
        const double eps = kind == 2 ? 0.5 : U(rng) * 0.9;
        int lo = -1, len = -1;
        eps_run(m.data(), N, eps, &lo, &len);
        CHECK(lo >= 0 && lo < N && len >= 1 && len <= N);
        double T = 0.0, got = 0.0;
        for (int k = 0; k < N; ++k) T += m[k];
        for (int t = 0; t < len; ++t) got += m[(lo + t) % N];
        CHECK(len == N || got >= (1.0 - eps / 3.0) * T);
        for (int ln = 1; ln < len; ++ln)   // no shorter run holds the mass
            for (int s0 = 0; s0 < N; ++s0) {
                double mass = 0.0;
                for (int t = 0; t < ln; ++t) mass += m[(s0 + t) % N];
                CHECK(!(mass >= (1.0 - eps / 3.0) * T));
            }
    }
    for (int N = 1; N <= 12; ++N)
        for (int a = 0; a < N; ++a)
            for (int la = 1; la <= N; ++la)
                for (int b = 0; b < N; ++b)
                    for (int lb = 1; lb <= N; ++lb) {
                        int st = -7;
                        const int len = cyc_intersect(a, la, b, lb, N, &st);
                        CHECK(len >= 0 && len <= (la < lb ? la : lb));
                        if (len > 0) {
                            CHECK(st != -7);
                            for (int t = 0; t < len; ++t) {   // every point of the piece is in both runs
                                const int p = ((st + t) % N + N) % N;
                                const int ia = ((p - a) % N + N) % N, ib = ((p - b) % N + N) % N;
                                CHECK(la >= N || ia < la);
                                CHECK(lb >= N || ib < lb);
                            }
                        }
                        const int s2 = near_start(b, lb, a, la, N);
                        CHECK(((s2 - b) % N + N) % N == 0);
                    }
    std::printf("host geometry: %d failures\n", fails);
    return fails ? 1 : 0;
}
