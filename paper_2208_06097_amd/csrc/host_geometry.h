// Host-only geometry of the pair list and the epsilon-driven boxes: plain
// C++ (no HIP), shared by the library's C entry points and the host tests
// that build it with address and undefined-behaviour sanitizers.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "sea.h"

// minimum-image difference on a periodic axis of length L
inline double host_minimg(double d, double L) { return d - L * std::nearbyint(d / L); }

// Pair selection and cube domains (Sec. II.B): i <= j kept when the
// minimum-image distance of the centres is below r_pair (self pairs always);
// the domain is the cube of w = ceil(half_width / h) points on each side of
// the grid point nearest the canonical (i <= j) midpoint, the multipole
// origin that point.  Writes at most `cap` pairs; returns how many there are.
inline int host_build_pairs(const int32_t* n, const double* L, int n_occ, const double* c, double r_pair,
                            double half_width, sea_pair* out, int cap) {
    int cnt = 0;
    for (int i = 0; i < n_occ; ++i) {
        for (int j = i; j < n_occ; ++j) {
            double d[3], d2 = 0.0;
            for (int a = 0; a < 3; ++a) {
                d[a] = host_minimg(c[3 * j + a] - c[3 * i + a], L[a]);
                d2 += d[a] * d[a];
            }
            if (i != j && !(std::sqrt(d2) < r_pair)) continue;
            if (cnt < cap) {
                sea_pair& p = out[cnt];
                p.i = i;
                p.j = j;
                for (int a = 0; a < 3; ++a) {
                    const double h = L[a] / n[a];
                    const double m = c[3 * i + a] + 0.5 * d[a];
                    const int kc = (int)std::floor(m / h + 0.5);
                    const int w = (int)std::ceil(half_width / h - 1e-12);
                    p.lo[a] = kc - w;
                    p.n[a] = 2 * w + 1;
                    p.origin[a] = kc * h;
                }
            }
            ++cnt;
        }
    }
    return cnt;
}

// Shortest cyclic run of m[0..N) with mass >= target; among runs of that
// length the largest mass, then the smallest start.  Direct sums, in the
// order the runs are listed.
inline void eps_run(const double* m, int N, double eps, int* lo, int* len) {
    double T = 0.0;
    for (int k = 0; k < N; ++k) T += m[k];
    const double target = (1.0 - eps / 3.0) * T;
    for (int ln = 1; ln < N; ++ln) {
        double best = -1.0;
        int bs = -1;
        for (int s0 = 0; s0 < N; ++s0) {
            double mass = 0.0;
            for (int t = 0; t < ln; ++t) mass += m[(s0 + t) % N];
            if (mass >= target && mass > best) {
                best = mass;
                bs = s0;
            }
        }
        if (bs >= 0) {
            *lo = bs;
            *len = ln;
            return;
        }
    }
    *lo = 0;
    *len = N;
}

// Intersection of cyclic runs [a, a+la) and [b, b+lb) on Z_N; the longer
// piece when there are two; start unwrapped into [a, a+la).
inline int cyc_intersect(int a, int la, int b, int lb, int N, int* start) {
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
        const int s0 = std::max(a, b + k * N);
        const int e0 = std::min(a + la, b + k * N + lb);
        if (e0 - s0 > best) {
            best = e0 - s0;
            *start = s0;
        }
    }
    return best;
}

// Start of a run of length ln shifted by a multiple of N so that its centre
// is nearest the centre of the reference run [r0, r0 + rn).
inline int near_start(int lo, int ln, int r0, int rn, int N) {
    int best = lo, bd = -1;
    for (int k = -1; k <= 1; ++k) {
        const int d = std::abs(2 * (lo + k * N) + ln - (2 * r0 + rn));
        if (bd < 0 || d < bd) {
            bd = d;
            best = lo + k * N;
        }
    }
    return best;
}

