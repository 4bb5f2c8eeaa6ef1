// Types shared by the surrogate network's kernels and its host API.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace mlp {

// C[m, n] = sum_k A[m, k] B[k, n] with A[m, k] at A[m * sam + k * sak] and B[k, n] at
// B[k * sbk + n * sbn] (BF16); the epilogue adds bias[n], applies ReLU, zeroes where
// mask[m, n] <= 0, and writes FP32 to Cf and/or BF16 to Cb (row stride ldc).
struct GemmArgs {
    const uint16_t* A;
    int64_t sam, sak;
    const uint16_t* B;
    int64_t sbk, sbn;
    int M, N, K;
    int relu;
    const float* bias;
    const uint16_t* mask;
    float* Cf;
    uint16_t* Cb;
    int64_t ldc;
    int vec_a, vec_b;   // staging mode, chosen by launch_gemm
    float* ws;          // split-K workspace (may be null: no split)
    int64_t ws_elems;
};

constexpr int kColPartsHost = 64;   // partial sums per column of launch_colsum

// The whole forward pass in one launch (inference): every layer for a tile of samples per
// workgroup, activations kept in LDS.  Supported shapes: n_in <= 32, width a multiple of 32
// and <= kFusedMaxWidth, at most kFusedMaxLayers affine layers.
constexpr int kFusedMaxWidth = 256;
constexpr int kFusedMaxLayers = 8;
struct FusedArgs {
    const float* x;            // [batch x n_in] FP32
    float* y;                  // [batch x n_out] FP32
    int64_t batch;
    int n_in, width, layers, n_out;
    const uint16_t* W[kFusedMaxLayers];   // BF16 weights of layer l, [out x in]
    const float* bias[kFusedMaxLayers];   // FP32 biases of layer l
};
bool fused_forward_supported(int n_in, int width, int layers);
hipError_t launch_forward_fused(const FusedArgs& a, hipStream_t st);

hipError_t launch_gemm(const GemmArgs& g, hipStream_t st);
hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t st);
hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st);
hipError_t launch_loss_grad(const float* y, const float* t, int64_t n, float* df, uint16_t* db, float* loss,
                            hipStream_t st);
// part: scratch of kColPartsHost x cols floats
hipError_t launch_colsum(const float* dz, int64_t rows, int cols, float* part, float* db, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st);

}  // namespace mlp
