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
