// Network description and launch helpers of the learned warm start (k_nn.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

struct NnLayer {
    const char* name;
    int ci, co;   // input / output channels
    int relu;     // ReLU after the convolution
    int level;    // resolution level: size D >> level
};

constexpr int kNnNumLayers = 15;
constexpr int kNnGrid = 32;         // network grid of the learned start
constexpr int kNnInferBatch = 128;  // pairs per inference launch sequence
extern const NnLayer kNnLayers[kNnNumLayers];

size_t nn_param_offset(int layer);  // floats before layer's weights (weights, then bias)
size_t nn_param_count();

// Offsets (floats) into one activation/gradient workspace for batch B.
struct NnActLayout {
    size_t out[kNnNumLayers];
    size_t pool[3], up[3];
    size_t g0, g1, g2, gskip[3];
    size_t wpart, bpart, grad, mse_part;
    int nchunk;
    size_t total_floats;
};
NnActLayout nn_act_layout(int B, int D);

// params16 == nullptr selects FP32 weights; otherwise the BF16 copy is read.
hipError_t nn_forward(const float* params, const uint16_t* params16, const float* x, float* act,
                      const NnActLayout& L, int B, int D, float* y_out, hipStream_t s);
hipError_t nn_backward(const float* params, const uint16_t* params16, const float* x, float* act,
                       const NnActLayout& L, int B, int D, const float* g_out, hipStream_t s);
hipError_t nn_mse(const float* y, const float* t, long n, float* g, double* part, double* loss_dev,
                  hipStream_t s);
hipError_t nn_adam(float* p, uint16_t* p16, float* m, float* v, const float* g, long n, float lr, int step,
                   hipStream_t s);
hipError_t nn_to_bf16(const float* p, uint16_t* p16, long n, hipStream_t s);

// Inference on the matrix cores (BF16 weights and activations, FP32
// accumulation), network grid kNnGrid: offsets (bf16 elements) into its
// workspace for batch B: packed weights, and per level three channels-last
// tensors (ta, skip, tb) of B x d^3 x 16.
constexpr int kNnMfmaBatch = 512;   // pairs per inference launch sequence
struct NnInferLayout {
    size_t wpack;
    size_t ta[4], skip[4], tb[4];
    size_t total_bytes;
};
NnInferLayout nn_infer_layout(int B);
hipError_t nn_infer(const float* params, const uint16_t* params16, const float* x, void* ws, const NnInferLayout& L,
                    int B, float* y, hipStream_t s);

#define NN_CHECK(x)                        \
    do {                                   \
        hipError_t e_ = (x);               \
        if (e_ != hipSuccess) return e_;   \
    } while (0)
