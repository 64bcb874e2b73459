// Launchers of the SCDM pivot kernels (k_scdm.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

constexpr int SC_RB = 32;        // pivots per round at most
constexpr int SC_TMAX = 8192;    // candidates per round at most (plus the round's first pivot)
constexpr int SC_NMAX = 2048;    // orbitals at most

// Byte offsets of the pivot search's workspace.
struct ScdmLayout {
    size_t state, nrm, upv, upj, hist, cidx, cval, cvec, dv, dj, Q, piv, rdiag, total;
    long n_upd_blocks;
    int n_down_blocks;
};

ScdmLayout scdm_layout(long Ng, int n);
// Column norms |a_j|^2 and their per-block maxima.
hipError_t scdm_init(const void* phi, int f32, long Ng, int n, char* ws, const ScdmLayout& L, hipStream_t s);
// Column norms brought up to date with the b directions chosen from pivot k0 on.
hipError_t scdm_update(const void* phi, int f32, long Ng, int n, int k0, int b, char* ws, const ScdmLayout& L,
                       hipStream_t s);
// One round: candidate set, then up to SC_RB pivots (kernels turn into no-ops
// once the round has ended).  first = 1 for the first round.
hipError_t scdm_round(const void* phi, int f32, long Ng, int n, int first, char* ws, const ScdmLayout& L,
                      hipStream_t s);
// G (n x n, row a) = Phi^T(:, piv[a])
hipError_t scdm_pivot_rows(const void* phi, int f32, long Ng, int n, const int* piv, double* G, hipStream_t s);
// Synchronizing read of the pivot count and the rank flag.
hipError_t scdm_read_state(const char* ws, const ScdmLayout& L, int* k, int* fail, hipStream_t s);
// Newton-Schulz helpers (one workgroup each): Y = G / |G|_F, and
// S <- 1.5 I - 0.5 S with *err = |S - I|_F^2 of the incoming S.
hipError_t scdm_ns_scale(const double* G, int n, double* Y, hipStream_t s);
hipError_t scdm_ns_mid(double* S, int n, double* err, hipStream_t s);
