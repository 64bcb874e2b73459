// Inference of the learned-start network on the matrix cores (gfx950).
//
// The 16-channel 3x3x3 convolutions are implicit GEMMs: rows = 16 output
// voxels, columns = the 16 output channels, K = (input channels) x 27 taps.
// They run as v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation):
// one instruction covers two taps of one 16-channel input, so a 16-channel
// input takes 14 instructions per 16-voxel tile (the 28th tap has zero
// weights) and the 32-channel decoder inputs are two 16-channel halves
// accumulated into the same tile.  Activations are channels-last BF16
// ([B][D][D][D][16]: one voxel = 32 bytes); the 2x2x2 average pooling and
// the nearest-neighbour upsampling are fused into the staging of each
// convolution's input tile in LDS, and the skip concatenation is the second
// half of the K loop, so no pooled, upsampled or concatenated tensor is ever
// written.  The first layer (1 input channel) and the head (1 output
// channel) are too narrow for the matrix cores and run on the vector ALUs.
//
// Weights are the network state's BF16 copy; bias, ReLU and the rounding of
// each activation to BF16 happen in the epilogue.  The training path (FP32
// activations, k_nn.hip) is unchanged.
#include "nn_internal.h"
#include "sea_internal.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CH = 16;      // channels of every hidden tensor
constexpr int KS = 14;      // K steps per 16-channel input (27 taps, paired)
constexpr int WHALF = KS * CH * 32;  // packed weights of one input half (bf16)
constexpr int MF_NT = 256;  // threads per convolution workgroup

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                     // round to nearest even
    return (uint16_t)(u >> 16);
}

enum InMode { IN_PLAIN = 0, IN_POOL = 1, IN_UP = 2 };

// Packed weights: for every (layer, input half) a [KS][16 out][32 k] block,
// k = 16 * (tap - 2 ks) + c, i.e. element (ks, n, k) = w[n][16 half + c][2 ks + k / 16].
constexpr int kNumHalves = 16;
constexpr int kHalfLayer[kNumHalves] = {1, 2, 3, 4, 5, 6, 7, 8, 8, 9, 10, 10, 11, 12, 12, 13};
constexpr int kHalfIndex[kNumHalves] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 1, 0};
struct PackArgs {  // per half: offset of the layer's weights, its input channels, which half
    long off[kNumHalves];
    int ci[kNumHalves], half[kNumHalves];
};

__global__ void k_pack_weights(PackArgs pa, const uint16_t* __restrict__ p16, uint16_t* __restrict__ wp) {
    const int h = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= WHALF) return;
    const int k = e & 31, n = (e >> 5) & 15, ks = e >> 9;
    const int tap = 2 * ks + (k >> 4), c = pa.half[h] * CH + (k & 15);
    wp[(size_t)h * WHALF + e] = tap < 27 ? p16[pa.off[h] + ((size_t)n * pa.ci[h] + c) * 27 + tap] : (uint16_t)0;
}

// One 16-channel input of a convolution (channels-last BF16 tensor).
struct ConvIn {
    const uint16_t* t;
    int mode;
};

// Output tile of one workgroup: TZ planes x TY rows x all D columns.
template <int D>
struct TileShape {
    static constexpr int TY = D < 8 ? D : 8;
    static constexpr int TZ = D >= 16 ? 2 : 1;
    static constexpr int HX = D + 2, HY = TY + 2, HZ = TZ + 2;
    static constexpr int NV = HX * HY * HZ;       // halo voxels staged in LDS
    static constexpr int NMT = TZ * TY * D / 16;  // 16-voxel M tiles
    static constexpr int MTW = (NMT + 3) / 4;     // M tiles per wave
    static constexpr int TILES = (D / TY) * (D / TZ);
};

// Stage the halo tile of input `in` around output planes z0.. and rows y0..
// into LDS (zero outside the volume), pooling or upsampling on the way.
template <int D>
__device__ __forceinline__ void stage(const ConvIn& in, int b, int z0, int y0, uint16_t* lds) {
    using T = TileShape<D>;
    for (int idx = threadIdx.x; idx < T::NV * 2; idx += MF_NT) {
        const int hv = idx >> 1, ch = (idx & 1) * 8;
        const int hx = hv % T::HX, hy = (hv / T::HX) % T::HY, hz = hv / (T::HX * T::HY);
        const int x = hx - 1, y = y0 + hy - 1, z = z0 + hz - 1;
        uint4 val = make_uint4(0, 0, 0, 0);
        if (x >= 0 && x < D && y >= 0 && y < D && z >= 0 && z < D) {
            if (in.mode == IN_PLAIN) {
                val = *reinterpret_cast<const uint4*>(in.t + ((((size_t)b * D + z) * D + y) * D + x) * CH + ch);
            } else if (in.mode == IN_UP) {
                constexpr int Dc = D / 2;
                val = *reinterpret_cast<const uint4*>(
                    in.t + ((((size_t)b * Dc + z / 2) * Dc + y / 2) * Dc + x / 2) * CH + ch);
            } else {
                constexpr int Df = 2 * D;
                float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const size_t v = (((size_t)b * Df + 2 * z + (q >> 2)) * Df + 2 * y + ((q >> 1) & 1)) * Df +
                                     2 * x + (q & 1);
                    const uint4 u = *reinterpret_cast<const uint4*>(in.t + v * CH + ch);
                    const uint32_t w4[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        acc[2 * e] += bf2f((uint16_t)(w4[e] & 0xffffu));
                        acc[2 * e + 1] += bf2f((uint16_t)(w4[e] >> 16));
                    }
                }
                uint32_t o[4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    o[e] = (uint32_t)f2bf(0.125f * acc[2 * e]) | ((uint32_t)f2bf(0.125f * acc[2 * e + 1]) << 16);
                val = make_uint4(o[0], o[1], o[2], o[3]);
            }
        }
        *reinterpret_cast<uint4*>(lds + (size_t)hv * CH + ch) = val;
    }
}

// LDS offset (bf16 elements) of tap t relative to the output voxel's slot.
template <int D>
__device__ __forceinline__ int tap_off(int t) {
    using T = TileShape<D>;
    const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
    return ((dz * T::HY + dy) * T::HX + dx) * CH;
}

// 3x3x3 convolution, 16 output channels, one or two 16-channel inputs.
// grid: (tiles of the volume, batch); block MF_NT.
template <int D, int NIN>
__global__ __launch_bounds__(MF_NT) void k_conv_mfma(ConvIn in0, ConvIn in1, const uint16_t* __restrict__ wp0,
                                                     const uint16_t* __restrict__ wp1, const float* __restrict__ bias,
                                                     uint16_t* __restrict__ out, int relu) {
    using T = TileShape<D>;
    __shared__ __attribute__((aligned(16))) uint16_t lds[T::NV * CH];
    const int b = blockIdx.y;
    const int tile = blockIdx.x;
    const int y0 = (tile % (D / T::TY)) * T::TY;
    const int z0 = (tile / (D / T::TY)) * T::TZ;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    // this lane's A rows: voxel i of each of the wave's M tiles
    int base[T::MTW];
#pragma unroll
    for (int m = 0; m < T::MTW; ++m) {
        const int mt = wave * T::MTW + m;
        const int v = (mt < T::NMT ? mt : 0) * 16 + i;
        const int zl = v / (T::TY * D), yl = (v / D) % T::TY, xl = v % D;
        base[m] = ((zl * T::HY + yl) * T::HX + xl) * CH + 8 * (g & 1);
    }
    f32x4 acc[T::MTW];
#pragma unroll
    for (int m = 0; m < T::MTW; ++m) acc[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int h = 0; h < NIN; ++h) {
        const uint16_t* wp = h == 0 ? wp0 : wp1;
        bf16x8 bw[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            bw[ks] = *reinterpret_cast<const bf16x8*>(wp + ((size_t)ks * CH + i) * 32 + 8 * g);
        if (h) __syncthreads();
        stage<D>(h == 0 ? in0 : in1, b, z0, y0, lds);
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int t0 = 2 * ks, t1 = 2 * ks + 1 < 27 ? 2 * ks + 1 : 26;
            const int off = (g >> 1) ? tap_off<D>(t1) : tap_off<D>(t0);
#pragma unroll
            for (int m = 0; m < T::MTW; ++m) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(lds + base[m] + off);
                acc[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[ks], acc[m], 0, 0, 0);
            }
        }
    }
    // epilogue: lane holds output channel i of voxels 4g..4g+3 of each M tile
    const float bv = bias[i];
#pragma unroll
    for (int m = 0; m < T::MTW; ++m) {
        const int mt = wave * T::MTW + m;
        if (mt >= T::NMT) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = mt * 16 + 4 * g + j;
            const int z = z0 + v / (T::TY * D), y = y0 + (v / D) % T::TY, x = v % D;
            float r = acc[m][j] + bv;
            if (relu) r = fmaxf(r, 0.0f);
            out[((((size_t)b * D + z) * D + y) * D + x) * CH + i] = f2bf(r);
        }
    }
}

// First layer: 1 input channel (FP32 network input) -> 16 channels, ReLU.
constexpr int V_BS = 256;
template <int D>
__global__ __launch_bounds__(V_BS) void k_conv_first(const float* __restrict__ x, const uint16_t* __restrict__ w16,
                                                    const float* __restrict__ bias, uint16_t* __restrict__ out,
                                                    long nvox) {
    __shared__ float w[CH * 27 + CH];
    for (int k = threadIdx.x; k < CH * 27; k += V_BS) w[k] = bf2f(w16[k]);
    if (threadIdx.x < CH) w[CH * 27 + threadIdx.x] = bias[threadIdx.x];
    __syncthreads();
    const long id = (long)blockIdx.x * V_BS + threadIdx.x;
    if (id >= nvox) return;
    const int xx = id % D, yy = (id / D) % D, zz = (id / (D * D)) % D;
    const long b = id / ((long)D * D * D);
    const float* xb = x + b * D * D * D;
    float in[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) {
        const int z = zz + t / 9 - 1, y = yy + (t / 3) % 3 - 1, xc = xx + t % 3 - 1;
        in[t] = (z >= 0 && z < D && y >= 0 && y < D && xc >= 0 && xc < D) ? xb[(z * D + y) * D + xc] : 0.0f;
    }
    uint32_t o[8];
#pragma unroll
    for (int n = 0; n < CH; n += 2) {
        float s0 = w[CH * 27 + n], s1 = w[CH * 27 + n + 1];
#pragma unroll
        for (int t = 0; t < 27; ++t) {
            s0 += w[n * 27 + t] * in[t];
            s1 += w[(n + 1) * 27 + t] * in[t];
        }
        o[n / 2] = (uint32_t)f2bf(fmaxf(s0, 0.0f)) | ((uint32_t)f2bf(fmaxf(s1, 0.0f)) << 16);
    }
    uint4* dst = reinterpret_cast<uint4*>(out + id * CH);
    dst[0] = make_uint4(o[0], o[1], o[2], o[3]);
    dst[1] = make_uint4(o[4], o[5], o[6], o[7]);
}

// Head: 16 channels -> 1 output (FP32), no ReLU.
template <int D>
__global__ __launch_bounds__(V_BS) void k_conv_head(const uint16_t* __restrict__ in, const uint16_t* __restrict__ w16,
                                                   const float* __restrict__ bias, float* __restrict__ y, long nvox) {
    __shared__ float w[27 * CH];  // [tap][c]
    for (int k = threadIdx.x; k < CH * 27; k += V_BS) {
        const int c = k / 27, t = k % 27;
        w[t * CH + c] = bf2f(w16[k]);
    }
    __syncthreads();
    const long id = (long)blockIdx.x * V_BS + threadIdx.x;
    if (id >= nvox) return;
    const int xx = id % D, yy = (id / D) % D, zz = (id / (D * D)) % D;
    const long b = id / ((long)D * D * D);
    float s = bias[0];
    for (int t = 0; t < 27; ++t) {
        const int z = zz + t / 9 - 1, yv = yy + (t / 3) % 3 - 1, xc = xx + t % 3 - 1;
        if (z < 0 || z >= D || yv < 0 || yv >= D || xc < 0 || xc >= D) continue;
        const uint4* src = reinterpret_cast<const uint4*>(in + ((((size_t)b * D + z) * D + yv) * D + xc) * CH);
        const uint4 u0 = src[0], u1 = src[1];
        const uint32_t q[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            s += w[t * CH + 2 * e] * bf2f((uint16_t)(q[e] & 0xffffu));
            s += w[t * CH + 2 * e + 1] * bf2f((uint16_t)(q[e] >> 16));
        }
    }
    y[id] = s;
}

template <int D, int NIN>
hipError_t conv_mfma(ConvIn a, ConvIn b, const uint16_t* wp0, const uint16_t* wp1, const float* bias, uint16_t* out,
                     int B, hipStream_t s) {
    using T = TileShape<D>;
    hipLaunchKernelGGL((k_conv_mfma<D, NIN>), dim3(T::TILES, B), dim3(MF_NT), 0, s, a, b, wp0, wp1, bias, out, 1);
    return hipGetLastError();
}

}  // namespace

// ---------------------------------------------------------------------------

NnInferLayout nn_infer_layout(int B) {
    NnInferLayout L{};
    size_t off = 0;
    auto take = [&](size_t elems) {  // bf16 elements, 256-byte aligned
        const size_t o = off;
        off += (elems + 127) / 128 * 128;
        return o;
    };
    L.wpack = take((size_t)kNumHalves * WHALF);
    for (int lv = 0; lv < 4; ++lv) {
        const size_t d = (size_t)kNnGrid >> lv;
        const size_t n = (size_t)B * d * d * d * CH;
        L.ta[lv] = take(n);
        L.skip[lv] = take(n);
        L.tb[lv] = take(n);
    }
    L.total_bytes = off * sizeof(uint16_t);
    return L;
}

hipError_t nn_infer(const float* params, const uint16_t* params16, const float* x, void* ws, const NnInferLayout& L,
                    int B, float* y, hipStream_t s) {
    static_assert(kNnGrid == 32, "inference kernels are built for a 32^3 network grid");
    uint16_t* W = reinterpret_cast<uint16_t*>(ws);
    PackArgs pa;
    for (int h = 0; h < kNumHalves; ++h) {
        pa.off[h] = (long)nn_param_offset(kHalfLayer[h]);
        pa.ci[h] = kNnLayers[kHalfLayer[h]].ci;
        pa.half[h] = kHalfIndex[h];
    }
    uint16_t* wp = W + L.wpack;
    hipLaunchKernelGGL(k_pack_weights, dim3((WHALF + 255) / 256, kNumHalves), dim3(256), 0, s, pa, params16, wp);
    NN_CHECK(hipGetLastError());
    auto half = [&](int h) { return wp + (size_t)h * WHALF; };
    auto bias = [&](int k) { return params + nn_param_offset(k) + (size_t)kNnLayers[k].co * kNnLayers[k].ci * 27; };
    auto T = [&](size_t o) { return W + o; };
    const ConvIn none{nullptr, IN_PLAIN};
    const long n0 = (long)B * 32 * 32 * 32;
    // encoder
    hipLaunchKernelGGL(k_conv_first<32>, dim3((unsigned)((n0 + V_BS - 1) / V_BS)), dim3(V_BS), 0, s, x,
                       params16 + nn_param_offset(0), bias(0), T(L.ta[0]), n0);
    NN_CHECK(hipGetLastError());
    NN_CHECK((conv_mfma<32, 1>(ConvIn{T(L.ta[0]), IN_PLAIN}, none, half(0), nullptr, bias(1), T(L.skip[0]), B, s)));
    NN_CHECK((conv_mfma<16, 1>(ConvIn{T(L.skip[0]), IN_POOL}, none, half(1), nullptr, bias(2), T(L.ta[1]), B, s)));
    NN_CHECK((conv_mfma<16, 1>(ConvIn{T(L.ta[1]), IN_PLAIN}, none, half(2), nullptr, bias(3), T(L.skip[1]), B, s)));
    NN_CHECK((conv_mfma<8, 1>(ConvIn{T(L.skip[1]), IN_POOL}, none, half(3), nullptr, bias(4), T(L.ta[2]), B, s)));
    NN_CHECK((conv_mfma<8, 1>(ConvIn{T(L.ta[2]), IN_PLAIN}, none, half(4), nullptr, bias(5), T(L.skip[2]), B, s)));
    NN_CHECK((conv_mfma<4, 1>(ConvIn{T(L.skip[2]), IN_POOL}, none, half(5), nullptr, bias(6), T(L.ta[3]), B, s)));
    NN_CHECK((conv_mfma<4, 1>(ConvIn{T(L.ta[3]), IN_PLAIN}, none, half(6), nullptr, bias(7), T(L.tb[3]), B, s)));
    // decoder: [up(previous), skip]
    NN_CHECK((conv_mfma<8, 2>(ConvIn{T(L.tb[3]), IN_UP}, ConvIn{T(L.skip[2]), IN_PLAIN}, half(7), half(8), bias(8),
                              T(L.ta[2]), B, s)));
    NN_CHECK((conv_mfma<8, 1>(ConvIn{T(L.ta[2]), IN_PLAIN}, none, half(9), nullptr, bias(9), T(L.tb[2]), B, s)));
    NN_CHECK((conv_mfma<16, 2>(ConvIn{T(L.tb[2]), IN_UP}, ConvIn{T(L.skip[1]), IN_PLAIN}, half(10), half(11),
                               bias(10), T(L.ta[1]), B, s)));
    NN_CHECK((conv_mfma<16, 1>(ConvIn{T(L.ta[1]), IN_PLAIN}, none, half(12), nullptr, bias(11), T(L.tb[1]), B, s)));
    NN_CHECK((conv_mfma<32, 2>(ConvIn{T(L.tb[1]), IN_UP}, ConvIn{T(L.skip[0]), IN_PLAIN}, half(13), half(14),
                               bias(12), T(L.ta[0]), B, s)));
    NN_CHECK((conv_mfma<32, 1>(ConvIn{T(L.ta[0]), IN_PLAIN}, none, half(15), nullptr, bias(13), T(L.tb[0]), B, s)));
    hipLaunchKernelGGL(k_conv_head<32>, dim3((unsigned)((n0 + V_BS - 1) / V_BS)), dim3(V_BS), 0, s, T(L.tb[0]),
                       params16 + nn_param_offset(14), bias(14), y, n0);
    NN_CHECK(hipGetLastError());
    return hipSuccess;
}
