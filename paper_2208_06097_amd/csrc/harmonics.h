// Real regular solid harmonics by the Cartesian recurrence (no trigonometry).
//
// Racah-normalized real solid harmonics C_lm, S_lm (0 <= m <= l), with the
// Condon-Shortley phase, satisfy
//   C_00 = 1, S_00 = 0,
//   C_{l+1,l+1} = -sqrt((2l+1)/(2l+2)) (x C_ll - y S_ll),
//   S_{l+1,l+1} = -sqrt((2l+1)/(2l+2)) (y C_ll + x S_ll),
//   C_{l+1,m} = ((2l+1) z C_lm - sqrt((l+m)(l-m)) r^2 C_{l-1,m}) / sqrt((l+m+1)(l-m+1)),
// and the same for S.  Storage index: C_lm at l*l + l + m, S_lm at l*l + l - m.
//
// With these, the multipole expansion (Eq. 10-11) becomes
//   v(t) = sum_l r^{-(2l+1)} sum_{m>=0} eps_m (QC_lm C_lm(t) + QS_lm S_lm(t)),
//   QC_lm = dV sum rho C_lm,  QS_lm = dV sum rho S_lm,  eps_0 = 1, eps_m = 2,
// which is the addition theorem for 1/|t - s| written in the Racah form; the
// orthonormal real Y_lm follow from r^l Y_lm = sqrt((2l+1)/(4 pi)) f_m {C,S}
// with f_0 = 1 and f_m = sqrt(2) (-1)^m.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

template <int LM>
__host__ __device__ __forceinline__ void racah_solid(double x, double y, double z, double* R) {
    const double r2 = x * x + y * y + z * z;
    R[0] = 1.0;
#pragma unroll
    for (int l = 0; l < LM; ++l) {
        const double Cll = R[l * l + 2 * l];
        const double Sll = (l == 0) ? 0.0 : R[l * l];
        const double f = -sqrt((2.0 * l + 1.0) / (2.0 * l + 2.0));
        const int base1 = (l + 1) * (l + 1) + (l + 1);
        R[base1 + (l + 1)] = f * (x * Cll - y * Sll);
        R[base1 - (l + 1)] = f * (y * Cll + x * Sll);
#pragma unroll
        for (int m = 0; m <= l; ++m) {
            const double den = 1.0 / sqrt((double)((l + m + 1) * (l - m + 1)));
            const double a = (2.0 * l + 1.0) * den;
            const double bb = sqrt((double)((l + m) * (l - m))) * den;
            const int base = l * l + l;
            double c = a * z * R[base + m];
            double s = (m > 0) ? a * z * R[base - m] : 0.0;
            if (m <= l - 1) {
                const int basem = (l - 1) * (l - 1) + (l - 1);
                c -= bb * r2 * R[basem + m];
                if (m > 0) s -= bb * r2 * R[basem - m];
            }
            R[base1 + m] = c;
            if (m > 0) R[base1 - m] = s;
        }
    }
}

// Multipole potential at displacement (x,y,z) from the origin, Racah moments
// Q (dV already applied), orders 0..lmax (runtime cut <= LM).
template <int LM>
__host__ __device__ __forceinline__ double racah_me_potential(const double* Q, int lmax, double x,
                                                              double y, double z) {
    double R[(LM + 1) * (LM + 1)];
    racah_solid<LM>(x, y, z, R);
    const double r2 = x * x + y * y + z * z;
    const double rinv = 1.0 / sqrt(r2);
    const double rinv2 = rinv * rinv;
    double pw = rinv;  // r^{-(2l+1)}
    double v = 0.0;
#pragma unroll
    for (int l = 0; l <= LM; ++l) {
        if (l <= lmax) {
            const int base = l * l + l;
            double acc = Q[base] * R[base];
#pragma unroll
            for (int m = 1; m <= l; ++m)
                acc += 2.0 * (Q[base + m] * R[base + m] + Q[base - m] * R[base - m]);
            v += acc * pw;
        }
        pw *= rinv2;
    }
    return v;
}

// Factor that maps Racah C/S at index l*l+l+m to r^l Y_lm (orthonormal real).
__host__ __device__ __forceinline__ double racah_to_orthonormal(int l, int m) {
    const double s = sqrt((2.0 * l + 1.0) / (4.0 * 3.14159265358979323846));
    if (m == 0) return s;
    const int am = m < 0 ? -m : m;
    return s * sqrt(2.0) * ((am & 1) ? -1.0 : 1.0);
}
