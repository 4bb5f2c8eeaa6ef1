// Kernels of the warm-start surrogate: a multilayer perceptron trained and evaluated in
// BF16 on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation), with FP32
// master weights and Adam (Kingma & Ba 2015, Algorithm 1).
//
// Every layer product is one GEMM  C[M x N] = A[M x K] B[K x N]  with element strides
// (so the transposed products of the backward pass need no transposed copies) and a
// fused epilogue: + bias[n], ReLU, a ReLU-derivative mask, FP32 and/or BF16 output.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mlp_types.hpp"

namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN stays a quiet NaN): one v_cvt_pk_bf16_f32.
__device__ __forceinline__ uint16_t to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Two FP32 -> two BF16 in one 32-bit word (a in the low half), one v_cvt_pk_bf16_f32.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2{a, b}), bf16x2));
}

__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Workgroup tile 64 x 64, K staged 32 at a time through LDS; four waves in a 2 x 2
// arrangement, each owning 32 x 32 of C as 2 x 2 MFMA blocks of 16 x 16.  LDS holds the A
// tile m-major and the B tile n-major, both with K contiguous, so that a lane's eight
// K-consecutive operands are one 16-byte LDS read: for the 16x16x32 BF16 MFMA, lane l
// supplies A[l % 16][8 (l / 16) + i] and B[8 (l / 16) + i][l % 16] (i = 0..7) and receives
// D[4 (l / 16) + q][l % 16] (q = 0..3).
constexpr int kBM = 64, kBN = 64, kBK = 32, kLDK = kBK + 8;

__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g, int k_split, float* __restrict__ part) {
    __shared__ __align__(16) uint16_t As[kBM * kLDK];
    __shared__ __align__(16) uint16_t Bs[kBN * kLDK];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int64_t kb = (int64_t)blockIdx.z * k_split;
    const int64_t ke = kb + k_split < g.K ? kb + k_split : g.K;
    for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
        // Stage the 64 x 32 tiles: 16-byte loads of 8 operands where a tile row (or column)
        // is contiguous in memory and 8-aligned (one load per thread per tile), else one
        // element at a time.  Out-of-range operands are zero.
        if (g.vec_a == 1) {   // contiguous along k
            const int r = tid >> 2, c = (tid & 3) * 8;
            const int64_t m = m0 + r, k = k0 + c;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (m < g.M && k < ke) v = *reinterpret_cast<const uint4*>(g.A + m * g.sam + k);
            *reinterpret_cast<uint4*>(&As[r * kLDK + c]) = v;
        } else if (g.vec_a == 2) {   // contiguous along m
            const int c = tid >> 3, r = (tid & 7) * 8;
            const int64_t m = m0 + r, k = k0 + c;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (m < g.M && k < ke) v = *reinterpret_cast<const uint4*>(g.A + m + k * g.sak);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
            for (int j = 0; j < 8; ++j) As[(r + j) * kLDK + c] = h[j];
        } else {
            for (int e = tid; e < kBM * kBK; e += 256) {
                const int r = e / kBK, c = e % kBK;
                const int64_t m = m0 + r, k = k0 + c;
                As[r * kLDK + c] = (m < g.M && k < ke) ? g.A[m * g.sam + k * g.sak] : (uint16_t)0;
            }
        }
        if (g.vec_b == 1) {   // contiguous along k
            const int r = tid >> 2, c = (tid & 3) * 8;
            const int64_t n = n0 + r, k = k0 + c;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (n < g.N && k < ke) v = *reinterpret_cast<const uint4*>(g.B + k + n * g.sbn);
            *reinterpret_cast<uint4*>(&Bs[r * kLDK + c]) = v;
        } else if (g.vec_b == 2) {   // contiguous along n
            const int c = tid >> 3, r = (tid & 7) * 8;
            const int64_t n = n0 + r, k = k0 + c;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (n < g.N && k < ke) v = *reinterpret_cast<const uint4*>(g.B + k * g.sbk + n);
            const uint16_t* h = reinterpret_cast<const uint16_t*>(&v);
            for (int j = 0; j < 8; ++j) Bs[(r + j) * kLDK + c] = h[j];
        } else {
            for (int e = tid; e < kBN * kBK; e += 256) {
                const int r = e / kBK, c = e % kBK;
                const int64_t n = n0 + r, k = k0 + c;
                Bs[r * kLDK + c] = (n < g.N && k < ke) ? g.B[k * g.sbk + n * g.sbn] : (uint16_t)0;
            }
        }
        __syncthreads();
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) {
            a[i] = *reinterpret_cast<const bf16x8*>(&As[(wm + 16 * i + (lane & 15)) * kLDK + 8 * (lane >> 4)]);
            b[i] = *reinterpret_cast<const bf16x8*>(&Bs[(wn + 16 * i + (lane & 15)) * kLDK + 8 * (lane >> 4)]);
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int q = 0; q < 4; ++q) {
                const int64_t m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
                const int64_t n = n0 + wn + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                if (part) {
                    part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][q];
                    continue;
                }
                float v = acc[i][j][q];
                if (g.bias) v += g.bias[n];
                if (g.relu) v = fmaxf(v, 0.0f);
                if (g.mask && !(from_bf16(g.mask[m * g.ldc + n]) > 0.0f)) v = 0.0f;
                if (g.Cf) g.Cf[m * g.ldc + n] = v;
                if (g.Cb) g.Cb[m * g.ldc + n] = to_bf16(v);
            }
}

// The epilogue of one output element: bias, ReLU, mask, FP32 and/or BF16 store.
__device__ __forceinline__ void gemm_store(const GemmArgs& g, int64_t m, int64_t n, float v) {
    if (g.bias) v += g.bias[n];
    if (g.relu) v = fmaxf(v, 0.0f);
    if (g.mask && !(from_bf16(g.mask[m * g.ldc + n]) > 0.0f)) v = 0.0f;
    if (g.Cf) g.Cf[m * g.ldc + n] = v;
    if (g.Cb) g.Cb[m * g.ldc + n] = to_bf16(v);
}

// Large tiles for operands that both stage with 16-byte loads (vec_a, vec_b != 0): a
// workgroup computes 128 x 128 of C, each wave 64 x 64 as 4 x 4 MFMA blocks, K in steps of
// 32 through two LDS buffers: the next step's tiles are loaded into registers while the
// current step's 16 MFMAs per wave run, then stored to the other buffer, one barrier per
// step.  blockIdx.z splits K into chunks of k_split (a multiple of 32): with more than one
// chunk, raw sums go to part[z][M][N] and gemm_reduce_kernel finishes them.
constexpr int kTM = 128, kTN = 128, kTLD = kBK + 8;

__device__ __forceinline__ void stage_load(const uint16_t* base, int vec, int64_t s_outer, int64_t s_inner,
                                           int64_t o0, int64_t k0, int64_t O, int64_t ke, int c, uint4& v,
                                           int& ro, int& rk) {
    // chunk c of the 128 x 32 tile: vec 1 -> 8 consecutive k of row ro; vec 2 -> 8
    // consecutive rows from ro at column rk
    if (vec == 1) {
        ro = c >> 2;
        rk = (c & 3) * 8;
    } else {
        rk = c >> 4;
        ro = (c & 15) * 8;
    }
    const int64_t o = o0 + ro, k = k0 + rk;
    v = make_uint4(0u, 0u, 0u, 0u);
    if (o < O && k < ke)
        v = *reinterpret_cast<const uint4*>(base + (vec == 1 ? o * s_outer + k : o + k * s_inner));
}

__device__ __forceinline__ void stage_store(uint16_t* lds, int vec, const uint4& v, int ro, int rk) {
    if (vec == 1) {
        *reinterpret_cast<uint4*>(&lds[ro * kTLD + rk]) = v;
    } else {
        const uint32_t wd[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int j = 0; j < 8; ++j) lds[(ro + j) * kTLD + rk] = (uint16_t)(wd[j >> 1] >> (16 * (j & 1)));
    }
}

__global__ void __launch_bounds__(256) gemm_bf16_big_kernel(GemmArgs g, int k_split, float* __restrict__ part) {
    // staging buffers, reused for the output tile after the K loop
    __shared__ __align__(16) uint16_t lds[2 * 2 * kTM * kTLD];
    uint16_t(*As)[kTM * kTLD] = reinterpret_cast<uint16_t(*)[kTM * kTLD]>(lds);
    uint16_t(*Bs)[kTN * kTLD] = reinterpret_cast<uint16_t(*)[kTN * kTLD]>(lds + 2 * kTM * kTLD);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.y * kTM, n0 = (int64_t)blockIdx.x * kTN;
    const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
    const int64_t kb = (int64_t)blockIdx.z * k_split;
    const int64_t ke = kb + k_split < g.K ? kb + k_split : g.K;
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    // A is (outer m, inner k): m stride sam, k stride sak; B^T is (outer n, inner k)
    uint4 ra[2], rb[2];
    int rao[2], rak[2], rbo[2], rbk[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        stage_load(g.A, g.vec_a, g.sam, g.sak, m0, kb, g.M, ke, tid + 256 * u, ra[u], rao[u], rak[u]);
        stage_load(g.B, g.vec_b, g.sbn, g.sbk, n0, kb, g.N, ke, tid + 256 * u, rb[u], rbo[u], rbk[u]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        stage_store(As[0], g.vec_a, ra[u], rao[u], rak[u]);
        stage_store(Bs[0], g.vec_b, rb[u], rbo[u], rbk[u]);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += kBK) {
        const bool more = k0 + kBK < ke;
        if (more)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                stage_load(g.A, g.vec_a, g.sam, g.sak, m0, k0 + kBK, g.M, ke, tid + 256 * u, ra[u], rao[u], rak[u]);
                stage_load(g.B, g.vec_b, g.sbn, g.sbk, n0, k0 + kBK, g.N, ke, tid + 256 * u, rb[u], rbo[u], rbk[u]);
            }
        bf16x8 a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            a[i] = *reinterpret_cast<const bf16x8*>(&As[buf][(wm + 16 * i + (lane & 15)) * kTLD + 8 * (lane >> 4)]);
            b[i] = *reinterpret_cast<const bf16x8*>(&Bs[buf][(wn + 16 * i + (lane & 15)) * kTLD + 8 * (lane >> 4)]);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        if (more)
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                stage_store(As[buf ^ 1], g.vec_a, ra[u], rao[u], rak[u]);
                stage_store(Bs[buf ^ 1], g.vec_b, rb[u], rbo[u], rbk[u]);
            }
        __syncthreads();
        buf ^= 1;
    }
    if (part) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t m = m0 + wm + 16 * i + 4 * (lane >> 4) + q;
                    const int64_t n = n0 + wn + 16 * j + (lane & 15);
                    if (m < g.M && n < g.N) part[((int64_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][q];
                }
        return;
    }
    // Output through LDS: each wave writes 32 of its 64 rows at a time (8 KiB per wave), then
    // every lane takes runs of 8 consecutive columns of a row, applies the epilogue and
    // stores them with 16-byte vector stores where the run is whole and 8-aligned.
    float* ot = reinterpret_cast<float*>(lds) + w * 32 * 64;
    const bool vec_out = (g.ldc % 8) == 0 && (!g.Cf || (reinterpret_cast<uintptr_t>(g.Cf) & 15u) == 0) &&
                         (!g.Cb || (reinterpret_cast<uintptr_t>(g.Cb) & 15u) == 0) &&
                         (!g.mask || (reinterpret_cast<uintptr_t>(g.mask) & 15u) == 0);
#pragma unroll
    for (int half = 0; half < 2; ++half) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    ot[(16 * i + 4 * (lane >> 4) + q) * 64 + 16 * j + (lane & 15)] = acc[2 * half + i][j][q];
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int idx = t * 64 + lane, r = idx >> 3, c = (idx & 7) * 8;
            const int64_t m = m0 + wm + 32 * half + r, n = n0 + wn + c;
            if (m >= g.M) continue;
            float v[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) v[e] = ot[r * 64 + c + e];
            if (vec_out && n + 8 <= g.N) {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    if (g.bias) v[e] += g.bias[n + e];
                    if (g.relu) v[e] = fmaxf(v[e], 0.0f);
                }
                if (g.mask) {
                    const uint4 mk = *reinterpret_cast<const uint4*>(g.mask + m * g.ldc + n);
                    const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        if (!(from_bf16((uint16_t)(mw[e >> 1] >> (16 * (e & 1)))) > 0.0f)) v[e] = 0.0f;
                }
                if (g.Cf) {
                    float4* dst = reinterpret_cast<float4*>(g.Cf + m * g.ldc + n);
                    dst[0] = make_float4(v[0], v[1], v[2], v[3]);
                    dst[1] = make_float4(v[4], v[5], v[6], v[7]);
                }
                if (g.Cb) {
                    uint32_t pk[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        pk[e] = (uint32_t)to_bf16(v[2 * e]) | ((uint32_t)to_bf16(v[2 * e + 1]) << 16);
                    *reinterpret_cast<uint4*>(g.Cb + m * g.ldc + n) = make_uint4(pk[0], pk[1], pk[2], pk[3]);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (n + e < g.N) gemm_store(g, m, n + e, v[e]);
            }
        }
        __syncthreads();
    }
}

// Split-K finish: each element sums its chunks in order, then the epilogue.
__global__ void gemm_reduce_kernel(GemmArgs g, int splits, const float* __restrict__ part) {
    const int64_t total = (int64_t)g.M * g.N;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.0f;
        for (int z = 0; z < splits; ++z) v += part[(int64_t)z * total + e];
        gemm_store(g, e / g.N, e % g.N, v);
    }
}

__global__ void to_bf16_kernel(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = to_bf16(x[i]);
}

__global__ void fill_kernel(float* __restrict__ p, int64_t n, float v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// dL/dy of L = sum (y - t)^2 / n: 2 (y - t) / n, in FP32 and BF16; the loss sum goes to
// *loss (one atomic per workgroup).
__global__ void __launch_bounds__(256) loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ t,
                                                        int64_t n, float* __restrict__ df,
                                                        uint16_t* __restrict__ db, float* __restrict__ loss) {
    __shared__ float part[4];
    float s = 0.0f;
    const float scale = 2.0f / (float)n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float d = y[i] - t[i];
        s += d * d;
        const float gi = scale * d;
        df[i] = gi;
        db[i] = to_bf16(gi);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, (part[0] + part[1] + part[2] + part[3]) / (float)n);
}

// Column sums db[c] = sum_r dz[r, c] of a row-major [rows x cols] matrix in two
// deterministic passes: workgroup (x, y) sums 64 columns over its share of the rows (four
// row lanes per column, combined in LDS) into part[y][c]; then each column adds its
// kColParts partial sums in order.
constexpr int kColParts = kColPartsHost;

__global__ void __launch_bounds__(256) colsum_part_kernel(const float* __restrict__ dz, int64_t rows, int cols,
                                                          float* __restrict__ part) {
    __shared__ float red[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + tx;
    const int64_t per = (rows + kColParts - 1) / kColParts;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
    float s = 0.0f;
    if (c < cols)
        for (int64_t r = r0 + ty; r < r1; r += 4) s += dz[r * cols + c];
    red[ty][tx] = s;
    __syncthreads();
    if (ty == 0 && c < cols) part[(int64_t)blockIdx.y * cols + c] = red[0][tx] + red[1][tx] + red[2][tx] + red[3][tx];
}

__global__ void colsum_final_kernel(const float* __restrict__ part, int cols, float* __restrict__ db) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int q = 0; q < kColParts; ++q) s += part[(int64_t)q * cols + c];
    db[c] = s;
}

// One Adam update of every parameter; also refreshes the BF16 copy the GEMMs read.
// c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, uint16_t* __restrict__ pb, int64_t n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.0f - b1) * gi;
        const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
        p[i] = pi;
        pb[i] = to_bf16(pi);
    }
}

namespace {
unsigned grid_for(int64_t n, int threads) {
    const int64_t b = (n + threads - 1) / threads;
    return (unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}
}  // namespace

// ----------------------------------------------------------------------------------
// The forward pass in one launch.  A workgroup of four waves takes kFT samples and runs
// every layer on them; the activations stay in LDS (one BF16 buffer) and never reach HBM,
// so the pass reads the FP32 input and writes the FP32 output only.  A layer's product is
// split over the waves by 64-column slices of its output; a wave computes all kFT rows of
// its slice as 8 x 4 MFMA blocks (v_mfma_f32_16x16x32_bf16, K in steps of 32, in order, as
// the layer-by-layer GEMMs do), with its A operands read from LDS and its B operands
// (weight rows, K contiguous) straight from memory, where every workgroup finds them in
// L2; the next K step's weights are loaded while the current step multiplies.  Each
// weight load thus serves kFT = 128 rows.  A hidden layer (at most 256 columns: one slice
// per wave) keeps its results in registers until every wave has read the layer input,
// then writes ReLU(acc + bias) rounded to BF16 over that input; the last layer adds the
// bias and stores FP32.
// ----------------------------------------------------------------------------------
constexpr int kFT = 128;                         // samples per workgroup
constexpr int kFLd = kFusedMaxWidth + 8;         // LDS row stride (BF16), 16-byte aligned rows

bool fused_forward_supported(int n_in, int width, int layers) {
    return n_in >= 1 && n_in <= 32 && width >= 32 && width <= kFusedMaxWidth && width % 32 == 0 && layers >= 2 &&
           layers <= kFusedMaxLayers;
}

namespace {
// B operands of one K step for the four 16-column blocks from column nc: lane holds
// W[n][kk .. kk + 7] of n = nc + 16 j + lane % 16 (zero past N or past the row's end).
__device__ __forceinline__ void load_b_step(const uint16_t* Wl, int Kw, int N, int nc, int kk, bool short_rows,
                                            bf16x8* bv) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int n = nc + 16 * j + (lane & 15);
        if (short_rows) {   // layer 0 (n_in < 8 possible): element by element
            uint16_t h[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) h[i] = (n < N && kk + i < Kw) ? Wl[(int64_t)n * Kw + kk + i] : (uint16_t)0;
            bv[j] = *reinterpret_cast<const bf16x8*>(h);
        } else {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (n < N) v = *reinterpret_cast<const uint4*>(Wl + (int64_t)n * Kw + kk);
            bv[j] = *reinterpret_cast<const bf16x8*>(&v);
        }
    }
}

// acc[i][j] = W[rows nc + 16 j ..][0, K) x A[rows 16 i ..][0, K)^T, the transposed block of
// the layer's product (weights as the first MFMA operand, activations as the second), so a
// lane ends with four consecutive outputs of one sample.  b0 holds the first K step's
// weights, loaded by the caller; the next step's weights are in flight while a step
// multiplies.
__device__ __forceinline__ void slice_product(const uint16_t* A, const uint16_t* Wl, int K, int Kw, int N, int nc,
                                              bool short_rows, bf16x8 (&b0)[4], f32x4 (&acc)[8][4]) {
    const int lane = threadIdx.x & 63;
    const int kl = 8 * (lane >> 4);
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int k0 = 0; k0 < K; k0 += 32) {
        const int kk = k0 + kl;
        bf16x8 b1[4];
        if (k0 + 32 < K) load_b_step(Wl, Kw, N, nc, kk + 32, short_rows, b1);
        bf16x8 av[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) av[i] = *reinterpret_cast<const bf16x8*>(&A[(16 * i + (lane & 15)) * kFLd + kk]);
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b0[j], av[i], acc[i][j], 0, 0, 0);
#pragma unroll
        for (int j = 0; j < 4; ++j) b0[j] = b1[j];
    }
}
}  // namespace

__global__ void __launch_bounds__(256, 2) forward_fused_kernel(FusedArgs a) {
    __shared__ __align__(16) uint16_t act[kFT * kFLd];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * kFT;
    // input rows as BF16, K zero-padded to 32: every load issued before the first is used
    constexpr int kInPerThread = kFT * 32 / 256;
    float xin[kInPerThread];
#pragma unroll
    for (int u = 0; u < kInPerThread; ++u) {
        const int e = tid + 256 * u, r = e >> 5, k = e & 31;
        const int64_t m = m0 + r;
        xin[u] = (m < a.batch && k < a.n_in) ? a.x[m * a.n_in + k] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kInPerThread; ++u) {
        const int e = tid + 256 * u;
        act[(e >> 5) * kFLd + (e & 31)] = to_bf16(xin[u]);
    }
    __syncthreads();
    // hidden layers: one slice per wave (width <= 256); the last layer: as many as it needs.
    // The first K step of every slice is loaded while the slice before it finishes.
    const int kl = 8 * (lane >> 4);
    bf16x8 bfirst[4];
    if (64 * w < a.width) load_b_step(a.W[0], a.n_in, a.width, 64 * w, kl, true, bfirst);
    for (int l = 0; l < a.layers; ++l) {
        const bool last = l + 1 == a.layers;
        const int K = l == 0 ? 32 : a.width;          // K of the stored operands (layer 0 padded)
        const int Kw = l == 0 ? a.n_in : a.width;     // row length of the weight matrix
        const uint16_t* Wl = a.W[l];
        const float* bl = a.bias[l];
        const int N = last ? a.n_out : a.width;
        const int rounds = last ? (N + 255) / 256 : 1;
        for (int t = 0; t < rounds; ++t) {
            const int nc = 64 * w + 256 * t;
            // block (i, j): lane holds outputs nq + 16 j + q (q < 4) of sample 16 i + lane % 16
            const int nq = nc + 4 * (lane >> 4);
            f32x4 acc[8][4];
            float bias[4][4];   // loaded before the product, used after it
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) bias[j][q] = nq + 16 * j + q < N ? bl[nq + 16 * j + q] : 0.0f;
            if (nc < N) slice_product(act, Wl, K, Kw, N, nc, l == 0, bfirst, acc);
            {   // the next slice's first K step: (l, t + 1), else (l + 1, 0)
                const bool same = t + 1 < rounds;
                const int l2 = same ? l : l + 1;
                if (l2 < a.layers) {
                    const int N2 = l2 + 1 == a.layers ? a.n_out : a.width;
                    const int nc2 = same ? nc + 256 : 64 * w;
                    if (nc2 < N2) load_b_step(a.W[l2], l2 == 0 ? a.n_in : a.width, N2, nc2, kl, l2 == 0, bfirst);
                }
            }
            if (!last) __syncthreads();   // every wave has read the layer input: overwrite it
            if (nc < N) {
                const int ml = lane & 15;
                if (!last) {   // N = width, a multiple of 32: a block's four outputs are all in range
#pragma unroll
                    for (int i = 0; i < 8; ++i)
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int n0 = nq + 16 * j;
                            if (n0 >= N) continue;
                            uint2 pk;
                            pk.x = pack_bf16(fmaxf(acc[i][j][0] + bias[j][0], 0.0f), fmaxf(acc[i][j][1] + bias[j][1], 0.0f));
                            pk.y = pack_bf16(fmaxf(acc[i][j][2] + bias[j][2], 0.0f), fmaxf(acc[i][j][3] + bias[j][3], 0.0f));
                            *reinterpret_cast<uint2*>(&act[(16 * i + ml) * kFLd + n0]) = pk;
                        }
                } else {
                    // rows of four outputs 16-byte aligned
                    const bool vec = (a.n_out & 3) == 0 && (reinterpret_cast<uintptr_t>(a.y) & 15) == 0;
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int64_t m = m0 + 16 * i + ml;
                        if (m >= a.batch) continue;
                        float* yr = a.y + m * a.n_out;
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const int n0 = nq + 16 * j;
                            const float4 v = make_float4(acc[i][j][0] + bias[j][0], acc[i][j][1] + bias[j][1],
                                                         acc[i][j][2] + bias[j][2], acc[i][j][3] + bias[j][3]);
                            if (vec && n0 + 3 < N) {
                                *reinterpret_cast<float4*>(yr + n0) = v;
                            } else {
                                if (n0 < N) yr[n0] = v.x;
                                if (n0 + 1 < N) yr[n0 + 1] = v.y;
                                if (n0 + 2 < N) yr[n0 + 2] = v.z;
                                if (n0 + 3 < N) yr[n0 + 3] = v.w;
                            }
                        }
                    }
                }
            }
            if (!last) __syncthreads();
        }
    }
}

hipError_t launch_forward_fused(const FusedArgs& a, hipStream_t st) {
    if (!fused_forward_supported(a.n_in, a.width, a.layers) || a.batch < 1) return hipErrorInvalidValue;
    const int64_t blocks = (a.batch + kFT - 1) / kFT;
    hipLaunchKernelGGL(forward_fused_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g0, hipStream_t st) {
    if (g0.M <= 0 || g0.N <= 0 || g0.K <= 0) return hipErrorInvalidValue;
    GemmArgs g = g0;
    // vector staging needs 8-aligned starts of every 8-operand chunk and whole chunks in or
    // out of range: the contiguous extent a multiple of 8, the other stride too, 16-byte
    // aligned base
    auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    g.vec_a = 0;
    if (aligned(g.A) && g.sak == 1 && g.K % 8 == 0 && g.sam % 8 == 0) g.vec_a = 1;
    else if (aligned(g.A) && g.sam == 1 && g.M % 8 == 0 && g.sak % 8 == 0) g.vec_a = 2;
    g.vec_b = 0;
    if (aligned(g.B) && g.sbk == 1 && g.K % 8 == 0 && g.sbn % 8 == 0) g.vec_b = 1;
    else if (aligned(g.B) && g.sbn == 1 && g.N % 8 == 0 && g.sbk % 8 == 0) g.vec_b = 2;
    const bool big = g.vec_a && g.vec_b;
    const int64_t tm = (g.M + (big ? kTM : kBM) - 1) / (big ? kTM : kBM);
    const int64_t tn = (g.N + (big ? kTN : kBN) - 1) / (big ? kTN : kBN);
    // split K when the tiles alone cannot fill the device: chunks of at least 512, at most
    // 256 workgroups in all, within the workspace
    int splits = 1;
    if (g.ws && tm * tn < 128 && g.K >= 1024) {
        int64_t s = std::min<int64_t>(g.K / 512, 256 / (tm * tn));
        s = std::min<int64_t>(s, g.ws_elems / ((int64_t)g.M * g.N));
        splits = (int)std::max<int64_t>(1, s);
    }
    int64_t k_split = (g.K + splits - 1) / splits;
    k_split = (k_split + kBK - 1) / kBK * kBK;
    splits = (int)((g.K + k_split - 1) / k_split);
    const dim3 grid((unsigned)tn, (unsigned)tm, (unsigned)splits);
    float* part = splits > 1 ? g.ws : nullptr;
    if (big) hipLaunchKernelGGL(gemm_bf16_big_kernel, grid, dim3(256), 0, st, g, (int)k_split, part);
    else hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, st, g, (int)k_split, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || splits == 1) return e;
    hipLaunchKernelGGL(gemm_reduce_kernel, dim3(grid_for((int64_t)g.M * g.N, 256)), dim3(256), 0, st, g, splits, g.ws);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, x, y, n);
    return hipGetLastError();
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_loss_grad(const float* y, const float* t, int64_t n, float* df, uint16_t* db, float* loss,
                            hipStream_t st) {
    if (n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(loss_grad_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, y, t, n, df, db, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* dz, int64_t rows, int cols, float* part, float* db, hipStream_t st) {
    hipLaunchKernelGGL(colsum_part_kernel, dim3((unsigned)((cols + 63) / 64), kColParts), dim3(256), 0, st, dz, rows,
                       cols, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(colsum_final_kernel, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, st, part, cols, db);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, uint16_t* pb, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, g, m, v, pb, n, lr, b1, b2, eps, c1,
                       c2);
    return hipGetLastError();
}

}  // namespace mlp
