// Spectral start for the pair Poisson solves (an extension of the CG start
// guess of Eq. 9; the CG still drives every pair to the same true residual).
//
// With x0 the multipole start, the correction e = x - x0 solves A e = r0,
// r0 = b - A x0, where A is the O(h^12) Laplacian with zero values beyond
// the domain.  The same stencil with odd (instead of zero) continuation
// beyond each face is diagonalized exactly by the type-I discrete sine
// transform: for the mode sin((i+1) theta), theta = pi m / (n+1), one axis
// contributes -(c0 + 2 sum_k ck cos(k theta)) / h^2.  The two operators
// differ only where the stencil reaches past a face, i.e. within 6 points
// of the boundary, and there e is tiny because x0 already carries the
// multipole potential that sets the boundary values.  So e ~ S^-1 (r0 ./
// lambda) with S the separable sine transform, and x0 + e leaves a
// residual many decades below r0.
//
// The transform along one axis is a dense product with the symmetric,
// orthogonal matrix S_n[j][k] = sqrt(2/(n+1)) sin(pi (j+1)(k+1)/(n+1))
// (n <= 64 here, so a 64 x 64 product on the matrix cores beats an FFT of
// this length on this part).  Each pass transforms the slowest axis of a pair's array (a, b, c)
// and writes (b, c, a'): the axes rotate, so three passes transform z, y,
// x and restore the layout.  Forward passes end with the division by
// lambda, inverse passes (the same matrices: S is its own inverse) with
// the addition into x.  FP64 throughout; pairs with an axis longer than
// 64 keep the multipole start.
#include "sea_internal.h"

namespace {

constexpr int DS_BS = 256;
constexpr int DS_N = 64;        // longest axis handled
constexpr int DS_TC = 64;       // columns per workgroup tile
constexpr double kPiD = 3.14159265358979323846;
// second-derivative weights of the O(h^12) central difference (App. C)
constexpr double kW[7] = {-5369.0 / 1800.0, 12.0 / 7.0, -15.0 / 56.0, 10.0 / 189.0,
                          -1.0 / 112.0, 2.0 / 1925.0, -1.0 / 16632.0};

__host__ __device__ constexpr int tab_off(int n) { return (n - 1) * n * (2 * n - 1) / 6; }  // sum of m^2, m < n
__host__ __device__ constexpr int mu_off(int n) { return (n - 1) * n / 2; }                  // sum of m, m < n

// S_n and the one-axis eigenvalues (h = 1) for n = blockIdx.x + 1
__global__ __launch_bounds__(DS_BS) void k_dst_tables(double* __restrict__ S, double* __restrict__ mu) {
    const int n = blockIdx.x + 1;
    double* Sn = S + tab_off(n);
    const double sc = sqrt(2.0 / (n + 1));
    for (int t = threadIdx.x; t < n * n; t += DS_BS) {
        const int j = t / n, k = t % n;
        const int m = ((j + 1) * (k + 1)) % (2 * (n + 1));   // argument reduced to [0, 2 pi)
        Sn[t] = sc * sin(kPiD * (double)m / (double)(n + 1));
    }
    for (int m = threadIdx.x; m < n; m += DS_BS) {
        const double th = kPiD * (double)(m + 1) / (double)(n + 1);
        double s = kW[0];
#pragma unroll
        for (int k = 1; k <= 6; ++k) s += 2.0 * kW[k] * cos(k * th);
        mu[mu_off(n) + m] = -s;
    }
}

struct DstArgs {
    const sea_pair* pairs;
    const DevCell* cells;
    const int* pair_cell;
    size_t stride;
    const double* in;
    double* out;
    const double* S;
    const double* mu;
    int pass;   // 0: (z,y,x) -> (y,x,z'); 1: (y,x,z) -> (x,z,y'); 2: (x,z,y) -> (z,y,x')
    int mode;   // 0 plain; 1 divide by lambda; 2 add into out (the start x)
};

// grid (pairs, DS_TG): workgroup y takes column tiles y, y + DS_TG, ... of
// its pair, with S_A staged once; the next tile's input is loaded into
// registers while the current one is multiplied.
constexpr int DS_TG = 16;

// One pass on the FP64 matrix cores (v_mfma_f64_16x16x4f64): A = S
// (j x k, read as S[k][j], S being symmetric), B = the tile (k x columns),
// the axis zero-padded to 64.  Wave w owns output rows j = 16 w .. 16 w + 15
// and the tile's four 16-column blocks.  Operand lanes: row/column = lane %
// 16, k = lane / 16; result item v of a lane is row lane / 16 + 4 v, column
// lane % 16.
typedef double dst_f64x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_dst_mfma(DstArgs d) {
    __shared__ double sS[DS_N * DS_N];    // sS[k * 64 + j] = S[k][j]
    __shared__ double tin[DS_N * DS_TC];  // tin[k * 64 + c]
    constexpr int BS = 256, LD = DS_N * DS_N / BS;
    const int pid = blockIdx.x;
    const sea_pair P = d.pairs[pid];
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    if (nx > DS_N || ny > DS_N || nz > DS_N) return;   // keeps the multipole start
    int A, B, C;
    if (d.pass == 0) { A = nz; B = ny; C = nx; }
    else if (d.pass == 1) { A = ny; B = nx; C = nz; }
    else { A = nx; B = nz; C = ny; }
    const int ncol = B * C;
    if ((int)blockIdx.y * DS_TC >= ncol) return;
    const double* in = d.in + (size_t)pid * d.stride;
    double* out = d.out + (size_t)pid * d.stride;
    {
        const double* Sa = d.S + tab_off(A);
        double t[LD];
#pragma unroll
        for (int u = 0; u < LD; ++u) {
            const int q = threadIdx.x + u * BS, k = q / DS_N, j = q % DS_N;
            t[u] = (k < A && j < A) ? Sa[k * A + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < LD; ++u) sS[threadIdx.x + u * BS] = t[u];
    }
    const DevCell& Cl = d.cells[d.pair_cell[pid]];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane & 15, g = lane >> 4;
    double nxt[LD];
    auto load_tile = [&](int c0) {
#pragma unroll
        for (int u = 0; u < LD; ++u) {
            const int q = threadIdx.x + u * BS, a = q / DS_TC, c = q % DS_TC;
            nxt[u] = (a < A && c0 + c < ncol) ? in[(size_t)a * ncol + c0 + c] : 0.0;
        }
    };
    load_tile(blockIdx.y * DS_TC);
    for (int col0 = blockIdx.y * DS_TC; col0 < ncol; col0 += DS_TG * DS_TC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < LD; ++u) tin[threadIdx.x + u * BS] = nxt[u];
        __syncthreads();
        if (col0 + DS_TG * DS_TC < ncol) load_tile(col0 + DS_TG * DS_TC);
        dst_f64x4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = dst_f64x4{0.0, 0.0, 0.0, 0.0};
        const int kend = (A + 3) & ~3;
        for (int k0 = 0; k0 < kend; k0 += 4) {
            const double av = sS[(k0 + g) * DS_N + 16 * w + r];
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) {
                const double bv = tin[(k0 + g) * DS_TC + 16 * ct + r];
                acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
            }
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = col0 + 16 * ct + r;
            if (col >= ncol) continue;
            double lam_col = 0.0;
            if (d.mode == 1) {
                const int zz = col / C, yy = col % C;
                lam_col = d.mu[mu_off(nz) + zz] / (Cl.h[2] * Cl.h[2]) + d.mu[mu_off(ny) + yy] / (Cl.h[1] * Cl.h[1]);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int j = 16 * w + g + 4 * v;
                if (j >= A) continue;
                const double val = acc[ct][v];
                const size_t o = (size_t)col * A + j;
                if (d.mode == 1) out[o] = val / (lam_col + d.mu[mu_off(nx) + j] / (Cl.h[0] * Cl.h[0]));
                else if (d.mode == 2) out[o] += val;
                else out[o] = val;
            }
        }
    }
}

}  // namespace

size_t dst_table_doubles() { return (size_t)tab_off(DS_N + 1); }
size_t dst_mu_doubles() { return (size_t)mu_off(DS_N + 1); }

// x += S^-1 ((S r) ./ lambda) for every pair whose axes are all <= 64:
// r (n_pairs x stride) is overwritten, tmp is scratch of the same size.
hipError_t launch_spectral_start(const ExxArgs& a, int ncol_max, double* r, double* tmp, double* tab, double* mu,
                                 hipStream_t s, const std::function<void(bool)>& mark) {
    if (a.n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dst_tables, dim3(DS_N), dim3(DS_BS), 0, s, tab, mu);
    DstArgs d{};
    d.pairs = a.pairs;
    d.cells = a.cells;
    d.pair_cell = a.pair_cell;
    d.stride = a.stride;
    d.S = tab;
    d.mu = mu;
    const int tiles = (ncol_max + DS_TC - 1) / DS_TC;
    const dim3 grid((unsigned)a.n_pairs, (unsigned)(tiles < DS_TG ? tiles : DS_TG));
    // forward: r -> tmp -> r -> tmp (divided by lambda); inverse: tmp -> r -> tmp -> x (added)
    const double* ins[6] = {r, tmp, r, tmp, r, tmp};
    double* outs[6] = {tmp, r, tmp, r, tmp, a.v};
    mark(true);
    for (int q = 0; q < 6; ++q) {
        d.in = ins[q];
        d.out = outs[q];
        d.pass = q % 3;
        d.mode = q == 2 ? 1 : (q == 5 ? 2 : 0);
        hipLaunchKernelGGL(k_dst_mfma, grid, dim3(256), 0, s, d);
    }
    mark(false);
    return hipGetLastError();
}
