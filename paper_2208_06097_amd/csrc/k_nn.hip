// Learned CG warm start: a 3-D U-Net that maps the pair density (resampled
// to a D^3 grid, D = 32 in production) to the correction of the multipole
// guess, plus its backward pass and Adam, all as hand-written kernels.
//
// Network (16 channels; levels D, D/2, D/4, D/8; every 3x3x3 convolution
// but the head followed by ReLU; zero padding 1):
//   e0a(1->16) e0b -> s0, avgpool2, e1a e1b -> s1, avgpool2, e2a e2b -> s2,
//   avgpool2, e3a e3b, up2, [up, s2] d2a(32->16) d2b, up2, [up, s1] d1a d1b,
//   up2, [up, s0] d0a d0b, head(16->1).
//
// Activations: FP32, layout [B][C][D][D][D].  Parameters: one flat FP32
// master array (per layer: weights [O][C][27], then bias [O]); a BF16 copy
// of it is what the convolutions read when BF16 weights are selected.
// Accumulation is FP32 everywhere.
#include <hip/hip_bf16.h>

#include "nn_internal.h"
#include "sea_internal.h"

namespace {

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// round-to-nearest-even FP32 -> BF16 bits (finite inputs)
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

constexpr int CV_BS = 256;
constexpr int CV_MAXW = 16 * 32 * 27;  // largest weight block (either orientation)

// out[b, o, p] = bias[o] + sum_c sum_t W(o, c, t) in[b, c, p + d(t) - 1]
// Input channels 0..cA-1 come from inA, cA..cA+cB-1 from inB.  Output
// channels 0..oA-1 go to outA, the rest to outB.  W is read as
//   flip = 0:  w[(o*Cin + c)*27 + t]              (forward)
//   flip = 1:  w[(c*O + o)*27 + 26 - t]           (gradient w.r.t. the input)
template <int O>
__global__ __launch_bounds__(CV_BS) void k_conv3d(const float* __restrict__ inA, int cA, const float* __restrict__ inB,
                                                  int cB, const float* __restrict__ w32,
                                                  const uint16_t* __restrict__ w16, const float* __restrict__ bias,
                                                  float* __restrict__ outA, int oA, float* __restrict__ outB, int D,
                                                  int relu, int flip) {
    __shared__ float wl[CV_MAXW];
    const int Cin = cA + cB;
    for (int i = threadIdx.x; i < O * Cin * 27; i += CV_BS) {
        const int o = i / (Cin * 27), c = (i / 27) % Cin, t = i % 27;
        const int src = flip ? (c * O + o) * 27 + 26 - t : i;
        wl[i] = w16 ? bf16_bits_to_f32(w16[src]) : w32[src];
    }
    __syncthreads();
    const int b = blockIdx.y;
    const int D3 = D * D * D;
    const int p = blockIdx.x * CV_BS + threadIdx.x;
    if (p >= D3) return;
    const int x = p % D, y = (p / D) % D, z = p / (D * D);
    float acc[O];
#pragma unroll
    for (int o = 0; o < O; ++o) acc[o] = bias ? bias[o] : 0.0f;
#pragma unroll 1
    for (int c = 0; c < Cin; ++c) {
        const float* src = c < cA ? inA + ((size_t)b * cA + c) * D3 : inB + ((size_t)b * cB + (c - cA)) * D3;
#pragma unroll 1
        for (int tzy = 0; tzy < 9; ++tzy) {
            const int zz = z + tzy / 3 - 1, yy = y + tzy % 3 - 1;
            const bool rowin = (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)D;
            const float* row = src + (zz * D + yy) * D;
            float v[3];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                const int xx = x + dx - 1;
                v[dx] = (rowin && (unsigned)xx < (unsigned)D) ? row[xx] : 0.0f;
            }
            const float* wc = wl + c * 27 + tzy * 3;
#pragma unroll
            for (int o = 0; o < O; ++o)
                acc[o] += wc[o * Cin * 27] * v[0] + wc[o * Cin * 27 + 1] * v[1] + wc[o * Cin * 27 + 2] * v[2];
        }
    }
#pragma unroll
    for (int o = 0; o < O; ++o) {
        float r = acc[o];
        if (relu) r = fmaxf(r, 0.0f);
        if (o < oA)
            outA[((size_t)b * oA + o) * D3 + p] = r;
        else
            outB[((size_t)b * (O - oA) + (o - oA)) * D3 + p] = r;
    }
}

// Partial weight/bias gradients over a chunk of (batch, position):
// part[chunk][o][c][27] = sum g[b,o,p] in[b,c,p+d-1];  partb[chunk][o] = sum g.
constexpr int WG_BS = 256;
constexpr int WG_CHUNK = 8192;

__global__ __launch_bounds__(WG_BS) void k_conv3d_wgrad(const float* __restrict__ inA, int cA,
                                                       const float* __restrict__ inB, int cB,
                                                       const float* __restrict__ g, int O, int B, int D,
                                                       float* __restrict__ part, float* __restrict__ partb) {
    __shared__ float red[WG_BS / 64][28];
    const int chunk = blockIdx.x, c = blockIdx.y, o = blockIdx.z;
    const int Cin = cA + cB;
    const int D3 = D * D * D;
    const long total = (long)B * D3;
    const long beg = (long)chunk * WG_CHUNK, end = min(total, beg + WG_CHUNK);
    float acc[28];
#pragma unroll
    for (int t = 0; t < 28; ++t) acc[t] = 0.0f;
    for (long q = beg + threadIdx.x; q < end; q += WG_BS) {
        const int b = (int)(q / D3), p = (int)(q % D3);
        const int x = p % D, y = (p / D) % D, z = p / (D * D);
        const float gv = g[((size_t)b * O + o) * D3 + p];
        const float* src = c < cA ? inA + ((size_t)b * cA + c) * D3 : inB + ((size_t)b * cB + (c - cA)) * D3;
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            const int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
            const bool in = (unsigned)zz < (unsigned)D && (unsigned)yy < (unsigned)D && (unsigned)xx < (unsigned)D;
            acc[t] += gv * (in ? src[(zz * D + yy) * D + xx] : 0.0f);
        }
        acc[27] += gv;
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < 28; ++t) {
        float v = acc[t];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[wid][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < 28) {
        float s = 0.0f;
        for (int w = 0; w < WG_BS / 64; ++w) s += red[w][threadIdx.x];
        if (threadIdx.x < 27)
            part[(((size_t)chunk * O + o) * Cin + c) * 27 + threadIdx.x] = s;
        else if (c == 0)
            partb[(size_t)chunk * O + o] = s;
    }
}

// gw[o][c][t] = sum over chunks (fixed order); gb[o] likewise.
__global__ void k_wgrad_reduce(const float* __restrict__ part, const float* __restrict__ partb, int nchunk, int O,
                               int Cin, float* __restrict__ gw, float* __restrict__ gb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = O * Cin * 27;
    if (i < nw) {
        float s = 0.0f;
        for (int k = 0; k < nchunk; ++k) s += part[(size_t)k * nw + i];
        gw[i] = s;
    } else if (i < nw + O) {
        const int o = i - nw;
        float s = 0.0f;
        for (int k = 0; k < nchunk; ++k) s += partb[(size_t)k * O + o];
        gb[o] = s;
    }
}

__global__ void k_relu_mask(float* __restrict__ g, const float* __restrict__ y, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !(y[i] > 0.0f)) g[i] = 0.0f;
}

// average over 2x2x2 blocks: in [BC][D^3] -> out [BC][(D/2)^3]
__global__ void k_avgpool2(const float* __restrict__ in, float* __restrict__ out, int BC, int D) {
    const int h = D / 2;
    const long n = (long)BC * h * h * h;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = i % h, y = (i / h) % h, z = (i / (h * h)) % h;
    const long bc = i / ((long)h * h * h);
    const float* s = in + bc * D * D * D;
    float acc = 0.0f;
    for (int k = 0; k < 8; ++k) acc += s[((2 * z + (k >> 2)) * D + 2 * y + ((k >> 1) & 1)) * D + 2 * x + (k & 1)];
    out[i] = 0.125f * acc;
}

// gradient of avgpool2 (out [BC][D^3]); add = 1 accumulates into out
__global__ void k_avgpool2_bwd(const float* __restrict__ g, float* __restrict__ out, int BC, int D, int add) {
    const long n = (long)BC * D * D * D;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int h = D / 2;
    const int x = i % D, y = (i / D) % D, z = (i / (D * D)) % D;
    const long bc = i / ((long)D * D * D);
    const float v = 0.125f * g[((bc * h + z / 2) * h + y / 2) * h + x / 2];
    out[i] = add ? out[i] + v : v;
}

// nearest x2 upsampling: in [BC][h^3] -> out [BC][(2h)^3]
__global__ void k_up2(const float* __restrict__ in, float* __restrict__ out, int BC, int h) {
    const int D = 2 * h;
    const long n = (long)BC * D * D * D;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = i % D, y = (i / D) % D, z = (i / (D * D)) % D;
    const long bc = i / ((long)D * D * D);
    out[i] = in[((bc * h + z / 2) * h + y / 2) * h + x / 2];
}

// gradient of up2: out [BC][h^3] = sum of the 2x2x2 block of g [BC][(2h)^3]
__global__ void k_up2_bwd(const float* __restrict__ g, float* __restrict__ out, int BC, int h) {
    const int D = 2 * h;
    const long n = (long)BC * h * h * h;
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = i % h, y = (i / h) % h, z = (i / (h * h)) % h;
    const long bc = i / ((long)h * h * h);
    const float* s = g + bc * D * D * D;
    float acc = 0.0f;
    for (int k = 0; k < 8; ++k) acc += s[((2 * z + (k >> 2)) * D + 2 * y + ((k >> 1) & 1)) * D + 2 * x + (k & 1)];
    out[i] = acc;
}

// MSE: g = 2 (y - t) / n; partial sums of (y - t)^2 per block
constexpr int MS_BS = 256;
__global__ __launch_bounds__(MS_BS) void k_mse(const float* __restrict__ y, const float* __restrict__ t, long n,
                                                float* __restrict__ g, double* __restrict__ part) {
    __shared__ double red[MS_BS / 64];
    const long i = (long)blockIdx.x * MS_BS + threadIdx.x;
    double s = 0.0;
    if (i < n) {
        const float d = y[i] - t[i];
        g[i] = 2.0f * d / (float)n;
        s = (double)d * d;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tt = 0.0;
        for (int w = 0; w < MS_BS / 64; ++w) tt += red[w];
        part[blockIdx.x] = tt;
    }
}

__global__ void k_sum_to(const double* __restrict__ part, int n, double scale, double* __restrict__ out) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < n; ++k) s += part[k];
    out[0] = s * scale;
}

// Adam with bias correction; refreshes the BF16 copy of the parameters.
__global__ void k_adam(float* __restrict__ p, uint16_t* __restrict__ p16, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, long n, float lr, float c1, float c2) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pn = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
    p[i] = pn;
    p16[i] = f32_to_bf16_bits(pn);
}

__global__ void k_to_bf16(const float* __restrict__ p, uint16_t* __restrict__ p16, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p16[i] = f32_to_bf16_bits(p[i]);
}

__global__ void k_add(float* __restrict__ a, const float* __restrict__ b, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] += b[i];
}

inline unsigned nblk(long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ---------------------------------------------------------------------------
// host-side network description and launch sequences

const NnLayer kNnLayers[kNnNumLayers] = {
    {"e0a", 1, 16, 1, 0},  {"e0b", 16, 16, 1, 0}, {"e1a", 16, 16, 1, 1}, {"e1b", 16, 16, 1, 1},
    {"e2a", 16, 16, 1, 2}, {"e2b", 16, 16, 1, 2}, {"e3a", 16, 16, 1, 3}, {"e3b", 16, 16, 1, 3},
    {"d2a", 32, 16, 1, 2}, {"d2b", 16, 16, 1, 2}, {"d1a", 32, 16, 1, 1}, {"d1b", 16, 16, 1, 1},
    {"d0a", 32, 16, 1, 0}, {"d0b", 16, 16, 1, 0}, {"head", 16, 1, 0, 0},
};

size_t nn_param_offset(int layer) {
    size_t off = 0;
    for (int k = 0; k < layer; ++k) off += (size_t)kNnLayers[k].co * (kNnLayers[k].ci * 27 + 1);
    return off;
}

size_t nn_param_count() { return nn_param_offset(kNnNumLayers); }

// Activation buffers (floats) for batch B at input size D.
NnActLayout nn_act_layout(int B, int D) {
    NnActLayout L{};
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = off;
        off += (n + 63) / 64 * 64;
        return o;
    };
    for (int k = 0; k < kNnNumLayers; ++k) {
        const int d = D >> kNnLayers[k].level;
        L.out[k] = take((size_t)B * kNnLayers[k].co * d * d * d);
    }
    for (int lv = 1; lv <= 3; ++lv) {
        const int d = D >> lv;
        L.pool[lv - 1] = take((size_t)B * 16 * d * d * d);
    }
    for (int lv = 0; lv < 3; ++lv) {
        const int d = D >> lv;
        L.up[lv] = take((size_t)B * 16 * d * d * d);
    }
    const size_t big = (size_t)B * 32 * D * D * D;
    L.g0 = take(big);
    L.g1 = take(big);
    L.g2 = take(big);
    L.gskip[0] = take((size_t)B * 16 * D * D * D);
    L.gskip[1] = take((size_t)B * 16 * (D / 2) * (D / 2) * (D / 2));
    L.gskip[2] = take((size_t)B * 16 * (D / 4) * (D / 4) * (D / 4));
    const long npos = (long)B * D * D * D;
    L.nchunk = (int)((npos + WG_CHUNK - 1) / WG_CHUNK);
    L.wpart = take((size_t)L.nchunk * 16 * 32 * 27);
    L.bpart = take((size_t)L.nchunk * 16);
    L.grad = take(nn_param_count());
    L.mse_part = take(2 * (nblk(npos, MS_BS) + 64));  // doubles: 2 floats each
    L.total_floats = off;
    return L;
}

static hipError_t conv_launch(int O, const float* inA, int cA, const float* inB, int cB, const float* w32,
                              const uint16_t* w16, const float* bias, float* outA, int oA, float* outB, int B, int D,
                              int relu, int flip, hipStream_t s) {
    dim3 grid(nblk((long)D * D * D, CV_BS), B);
    switch (O) {
        case 1:
            hipLaunchKernelGGL(k_conv3d<1>, grid, dim3(CV_BS), 0, s, inA, cA, inB, cB, w32, w16, bias, outA, oA, outB,
                               D, relu, flip);
            break;
        case 16:
            hipLaunchKernelGGL(k_conv3d<16>, grid, dim3(CV_BS), 0, s, inA, cA, inB, cB, w32, w16, bias, outA, oA,
                               outB, D, relu, flip);
            break;
        case 32:
            hipLaunchKernelGGL(k_conv3d<32>, grid, dim3(CV_BS), 0, s, inA, cA, inB, cB, w32, w16, bias, outA, oA,
                               outB, D, relu, flip);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Inputs of layer k (A and B sources) given the activation buffers.
static void layer_inputs(int k, float* act, const NnActLayout& L, const float* x, const float** inA, int* cA,
                         const float** inB, int* cB) {
    *inB = nullptr;
    *cB = 0;
    *cA = kNnLayers[k].ci;
    switch (k) {
        case 0: *inA = x; break;                         // e0a <- input
        case 2: *inA = act + L.pool[0]; break;           // e1a <- pool(s0)
        case 4: *inA = act + L.pool[1]; break;           // e2a <- pool(s1)
        case 6: *inA = act + L.pool[2]; break;           // e3a <- pool(s2)
        case 8:                                          // d2a <- [up(e3b), s2]
            *inA = act + L.up[2]; *cA = 16; *inB = act + L.out[5]; *cB = 16; break;
        case 10:                                         // d1a <- [up(d2b), s1]
            *inA = act + L.up[1]; *cA = 16; *inB = act + L.out[3]; *cB = 16; break;
        case 12:                                         // d0a <- [up(d1b), s0]
            *inA = act + L.up[0]; *cA = 16; *inB = act + L.out[1]; *cB = 16; break;
        default: *inA = act + L.out[k - 1]; break;       // chain
    }
}

hipError_t nn_forward(const float* params, const uint16_t* params16, const float* x, float* act, const NnActLayout& L,
                      int B, int D, float* y_out, hipStream_t s) {
    for (int k = 0; k < kNnNumLayers; ++k) {
        const NnLayer& ly = kNnLayers[k];
        const int d = D >> ly.level;
        // the pooled / upsampled inputs this layer needs
        if (k == 2 || k == 4 || k == 6) {
            const int lv = k / 2;
            hipLaunchKernelGGL(k_avgpool2, dim3(nblk((long)B * 16 * d * d * d, 256)), dim3(256), 0, s,
                                         act + L.out[k - 1], act + L.pool[lv - 1], B * 16, 2 * d);
        NN_CHECK(hipGetLastError());
        }
        if (k == 8 || k == 10 || k == 12) {
            const int lv = (12 - k) / 2;  // 8 -> 2, 10 -> 1, 12 -> 0
            hipLaunchKernelGGL(k_up2, dim3(nblk((long)B * 16 * d * d * d, 256)), dim3(256), 0, s,
                                         act + L.out[k - 1], act + L.up[lv], B * 16, d / 2);
        NN_CHECK(hipGetLastError());
        }
        const float *inA, *inB;
        int cA, cB;
        layer_inputs(k, act, L, x, &inA, &cA, &inB, &cB);
        const size_t off = nn_param_offset(k);
        const size_t nw = (size_t)ly.co * ly.ci * 27;
        float* out = (k == kNnNumLayers - 1 && y_out) ? y_out : act + L.out[k];
        NN_CHECK(conv_launch(ly.co, inA, cA, inB, cB, params16 ? nullptr : params + off,
                             params16 ? params16 + off : nullptr, params + off + nw, out, ly.co, nullptr, B, d,
                             ly.relu, 0, s));
    }
    return hipSuccess;
}

// Backward pass from g_out (B x D^3) into L.grad (flat, parameter layout).
hipError_t nn_backward(const float* params, const uint16_t* params16, const float* x, float* act, const NnActLayout& L,
                       int B, int D, const float* g_out, hipStream_t s) {
    float* grad = act + L.grad;
    float* g = act + L.g0;    // gradient w.r.t. the current layer's output
    float* gn = act + L.g1;   // gradient w.r.t. its input (next g)
    float* gt = act + L.g2;
    NN_CHECK(hipMemcpyAsync(g, g_out, sizeof(float) * (size_t)B * D * D * D, hipMemcpyDeviceToDevice, s));
    for (int k = kNnNumLayers - 1; k >= 0; --k) {
        const NnLayer& ly = kNnLayers[k];
        const int d = D >> ly.level;
        const long nout = (long)B * ly.co * d * d * d;
        if (ly.relu)
            hipLaunchKernelGGL(k_relu_mask, dim3(nblk(nout, 256)), dim3(256), 0, s, g, act + L.out[k], nout);
        NN_CHECK(hipGetLastError());
        const float *inA, *inB;
        int cA, cB;
        layer_inputs(k, act, L, x, &inA, &cA, &inB, &cB);
        const size_t off = nn_param_offset(k);
        const size_t nw = (size_t)ly.co * ly.ci * 27;
        // weight and bias gradients
        const int nchunk = (int)(((long)B * d * d * d + WG_CHUNK - 1) / WG_CHUNK);
        hipLaunchKernelGGL(k_conv3d_wgrad, dim3(nchunk, ly.ci, ly.co), dim3(WG_BS), 0, s, inA, cA, inB, cB,
                                     g, ly.co, B, d, act + L.wpart, act + L.bpart);
        NN_CHECK(hipGetLastError());
        hipLaunchKernelGGL(k_wgrad_reduce, dim3(nblk((long)nw + ly.co, 256)), dim3(256), 0, s,
                                     act + L.wpart, act + L.bpart, nchunk, ly.co, ly.ci, grad + off, grad + off + nw);
        NN_CHECK(hipGetLastError());
        if (k == 0) break;  // no gradient needed for the network input
        // gradient w.r.t. the inputs: conv with flipped, transposed weights
        const float* wsrc32 = params16 ? nullptr : params + off;
        const uint16_t* wsrc16 = params16 ? params16 + off : nullptr;
        if (k == 8 || k == 10 || k == 12) {
            // split into the upsampled half and the skip half
            const int lv = (12 - k) / 2;
            float* gsk = act + L.gskip[lv];
            NN_CHECK(conv_launch(32, g, ly.co, nullptr, 0, wsrc32, wsrc16, nullptr, gt, 16, gsk, B, d, 0, 1, s));
            // up2 backward of the first half -> gradient w.r.t. the lower level output
            hipLaunchKernelGGL(k_up2_bwd, dim3(nblk((long)B * 16 * (d / 2) * (d / 2) * (d / 2), 256)),
                                         dim3(256), 0, s, gt, gn, B * 16, d / 2);
        NN_CHECK(hipGetLastError());
        } else if (k == 2 || k == 4 || k == 6) {
            // through the average pool; add the skip gradient of this level
            const int lv = k / 2 - 1;  // level of s_lv
            NN_CHECK(conv_launch(16, g, ly.co, nullptr, 0, wsrc32, wsrc16, nullptr, gt, 16, nullptr, B, d, 0, 1, s));
            hipLaunchKernelGGL(k_avgpool2_bwd, dim3(nblk((long)B * 16 * 8 * d * d * d, 256)), dim3(256), 0,
                                         s, gt, gn, B * 16, 2 * d, 0);
        NN_CHECK(hipGetLastError());
            const long nsk = (long)B * 16 * 8 * d * d * d;
            hipLaunchKernelGGL(k_add, dim3(nblk(nsk, 256)), dim3(256), 0, s, gn, act + L.gskip[lv], nsk);
        NN_CHECK(hipGetLastError());
        } else {
            NN_CHECK(conv_launch(ly.ci, g, ly.co, nullptr, 0, wsrc32, wsrc16, nullptr, gn, ly.ci, nullptr, B, d, 0, 1,
                                 s));
        }
        float* t = g;
        g = gn;
        gn = t;
    }
    return hipSuccess;
}

hipError_t nn_mse(const float* y, const float* t, long n, float* g, double* part, double* loss_dev, hipStream_t s) {
    const unsigned nb = nblk(n, MS_BS);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(MS_BS), 0, s, y, t, n, g, part);
    NN_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(1), 0, s, part, (int)nb, 1.0 / (double)n, loss_dev);
    return hipGetLastError();
}

hipError_t nn_adam(float* p, uint16_t* p16, float* m, float* v, const float* g, long n, float lr, int step,
                   hipStream_t s) {
    const float c1 = 1.0f - powf(0.9f, (float)step), c2 = 1.0f - powf(0.999f, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n, 256)), dim3(256), 0, s, p, p16, m, v, g, n, lr, c1, c2);
    return hipGetLastError();
}

hipError_t nn_to_bf16(const float* p, uint16_t* p16, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n, 256)), dim3(256), 0, s, p, p16, n);
    return hipGetLastError();
}
