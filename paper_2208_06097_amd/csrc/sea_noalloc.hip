// The allocation-free entry point: K psi = -xi (dV xi^T psi) (Eq. 18) with
// its device scratch (the K-slice partials of dV xi^T psi and that small
// product itself) in a static array of the code object instead of a caller
// workspace, for callers that cannot allocate device memory.  Each GPU the
// library runs on holds its own copy of the array from module load until
// the process ends; its device address is looked up once per device at
// set-up (sea_create, with the device current) and only that address is
// used from host code.  Every call on one GPU shares the array: calls that
// overlap on one GPU race.  Every element the products read is written by
// the same call first, so nothing needs clearing between calls.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "k_ace.h"
#include "sea_internal.h"

namespace {

sea_status fail(sea_ctx* ctx, sea_status st, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
sea_status fail(sea_ctx* ctx, sea_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
    return st;
}

constexpr size_t kScratchBytes = SEA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

static __device__ __align__(256) unsigned char scratch[SEA_NOALLOC_SCRATCH_BYTES];

void* noalloc_scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[dev] = p;
        else (void)hipGetLastError();
    }
    return g_scratch_ptr[dev];
}

extern "C" sea_status sea_ace_apply_noalloc(sea_ctx* ctx, int64_t n_grid, int n_occ, double dV, const void* xi_dev,
                                            int n_vec, const void* psi_dev, void* out_dev) {
    if (!ctx) return SEA_E_ARG;
    if (n_grid < 1) return fail(ctx, SEA_E_ARG, "n_grid < 1");
    if (n_occ < 1 || n_occ > 4096) return fail(ctx, SEA_E_ARG, "n_occ out of range");
    if (n_vec < 1) return fail(ctx, SEA_E_ARG, "n_vec < 1");
    if (!(dV > 0.0) || !std::isfinite(dV)) return fail(ctx, SEA_E_ARG, "dV must be positive and finite");
    if (!xi_dev || !psi_dev || !out_dev) return fail(ctx, SEA_E_ARG, "NULL array argument");
    // the small product C (n_occ x n_vec) and at least one K slice of partials
    const size_t mn = (size_t)n_occ * (size_t)n_vec * sizeof(double);
    const size_t c_bytes = align256(mn);
    if (c_bytes >= kScratchBytes || (kScratchBytes - c_bytes) / mn < 1)
        return fail(ctx, SEA_E_NOMEM,
                        "n_occ x n_vec = %d x %d needs %zu bytes of scratch; the allocation-free call has %zu",
                        n_occ, n_vec, c_bytes + mn, kScratchBytes);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device)
        return fail(ctx, SEA_E_ARG, "the current device is not the context's device");
    char* base = (char*)ctx->noalloc_scratch;
    if (!base) return fail(ctx, SEA_E_HIP, "the scratch array's device address is not available");
    const int max_splits = (int)((kScratchBytes - c_bytes) / mn);
    double* Cm = (double*)base;
    double* part = (double*)(base + c_bytes);
    hipStream_t s = (hipStream_t)ctx->opts.hip_stream;
    hipError_t e;
    // C (n_occ x n_vec) = dV xi psi^T ; out (n_vec x n_grid) = -C^T xi
    if (ctx->opts.ace_dtype == SEA_F64) {
        e = ace_mm_nt<ACE_F64, double, double>((const double*)xi_dev, (const double*)psi_dev, n_occ, n_vec, n_grid, dV,
                                               part, Cm, s, max_splits);
        if (e == hipSuccess)
            e = ace_mm_nn<ACE_F64, double, double>(Cm, 1, n_vec, (const double*)xi_dev, n_vec, n_occ, n_grid, -1.0,
                                                   (double*)out_dev, s);
    } else if (ctx->opts.ace_dtype == SEA_F32) {
        e = ace_mm_nt<ACE_F32, float, float>((const float*)xi_dev, (const float*)psi_dev, n_occ, n_vec, n_grid, dV,
                                             part, Cm, s, max_splits);
        if (e == hipSuccess)
            e = ace_mm_nn<ACE_F32, float, float>(Cm, 1, n_vec, (const float*)xi_dev, n_vec, n_occ, n_grid, -1.0,
                                                 (float*)out_dev, s);
    } else {
        e = ace_mm_nt<ACE_BF16, uint16_t, uint16_t>((const uint16_t*)xi_dev, (const uint16_t*)psi_dev, n_occ, n_vec,
                                                    n_grid, dV, part, Cm, s, max_splits);
        if (e == hipSuccess)
            e = ace_mm_nn<ACE_BF16, uint16_t, float>(Cm, 1, n_vec, (const uint16_t*)xi_dev, n_vec, n_occ, n_grid, -1.0,
                                                     (float*)out_dev, s);
    }
    if (e != hipSuccess) return fail(ctx, SEA_E_HIP, "HIP error: %s", hipGetErrorString(e));
    return SEA_OK;
}
