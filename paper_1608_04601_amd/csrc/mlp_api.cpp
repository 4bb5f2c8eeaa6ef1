// Host side of the surrogate network (include/surrogate.h): buffers, the forward pass,
// reverse-mode gradients and Adam, all as kernel launches on the handle's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mlp_types.hpp"
#include "pic1d.h"
#include "surrogate.h"

struct mlp_handle {
    int n_in = 0, width = 0, depth = 0, n_out = 0, max_batch = 0;
    hipStream_t stream = nullptr;
    std::vector<int> out_dim, in_dim;   // per affine layer
    std::vector<int64_t> w_off, b_off;  // offsets into the flat parameter vector
    int64_t n_params = 0;
    float* p = nullptr;        // FP32 master parameters
    uint16_t* pb = nullptr;    // BF16 copy read by the GEMMs
    float* g = nullptr;        // gradients
    float* m = nullptr;        // Adam moments
    float* v = nullptr;
    std::vector<uint16_t*> act;   // BF16 activations: act[0] input, act[l] output of hidden layer l
    float* y = nullptr;           // FP32 output of the last forward pass [max_batch x n_out]
    float* dzf[2] = {nullptr, nullptr};      // FP32 and BF16 dL/dz, ping-pong
    uint16_t* dzb[2] = {nullptr, nullptr};
    float* loss = nullptr;
    float* part = nullptr;   // column-sum partials [kColPartsHost x max(width, n_out)]
    float* ws = nullptr;     // split-K workspace of the weight-gradient products
    int64_t ws_elems = 0;
    int64_t t = 0;   // Adam steps taken
    int status = PIC_OK;
    std::string err;
    std::vector<void*> allocs;
};

namespace {
thread_local std::string g_mlp_error;

int mfail(mlp_handle* h, int code, const std::string& msg) {
    if (!h) {
        g_mlp_error = msg;
        return code;
    }
    if (h->status == PIC_OK) {
        h->status = code;
        h->err = msg;
    }
    return h->status;
}

bool mok(mlp_handle* h, hipError_t e, const char* what) {
    if (e == hipSuccess) return true;
    mfail(h, e == hipErrorOutOfMemory ? PIC_ENOMEM : PIC_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return false;
}

template <typename T>
bool alloc(mlp_handle* h, T** out, int64_t count) {
    void* q = nullptr;
    if (!mok(h, hipMalloc(&q, (size_t)count * sizeof(T)), "hipMalloc")) return false;
    h->allocs.push_back(q);
    *out = static_cast<T*>(q);
    return true;
}

uint64_t splitmix64(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int n_layers(const mlp_handle* h) { return h->depth + 1; }

// Forward pass of `batch` samples from the BF16 input act[0]; hidden outputs to act[l],
// the linear output to y (FP32).
int forward_from_act0(mlp_handle* h, int64_t batch, float* y) {
    const int L = n_layers(h);
    for (int l = 0; l < L; ++l) {
        mlp::GemmArgs g{};
        g.A = h->act[l];
        g.sam = h->in_dim[l];
        g.sak = 1;
        g.B = h->pb + h->w_off[l];   // B[k, n] = W[n, k]
        g.sbk = 1;
        g.sbn = h->in_dim[l];
        g.M = (int)batch;
        g.N = h->out_dim[l];
        g.K = h->in_dim[l];
        g.bias = h->p + h->b_off[l];
        g.ldc = h->out_dim[l];
        if (l + 1 < L) {
            g.relu = 1;
            g.Cb = h->act[l + 1];
        } else {
            g.Cf = y;
        }
        if (!mok(h, mlp::launch_gemm(g, h->stream), "gemm launch")) return h->status;
    }
    return PIC_OK;
}

// Loss gradient and reverse pass for the batch whose forward pass is in act[] and h->y;
// gradients to h->g, the loss (mean over outputs) accumulated into h->loss.
int backward(mlp_handle* h, const float* t, int64_t batch) {
    const int L = n_layers(h);
    if (!mok(h, mlp::launch_fill(h->loss, 1, 0.0f, h->stream), "fill") ||
        !mok(h, mlp::launch_loss_grad(h->y, t, batch * h->n_out, h->dzf[0], h->dzb[0], h->loss, h->stream),
             "loss launch"))
        return h->status;
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int o = h->out_dim[l], i = h->in_dim[l];
        // dW_l[o x i] = dz^T [o x B] . act[l] [B x i]
        mlp::GemmArgs gw{};
        gw.A = h->dzb[cur];
        gw.sam = 1;
        gw.sak = o;
        gw.B = h->act[l];
        gw.sbk = i;
        gw.sbn = 1;
        gw.M = o;
        gw.N = i;
        gw.K = (int)batch;
        gw.Cf = h->g + h->w_off[l];
        gw.ldc = i;
        gw.ws = h->ws;
        gw.ws_elems = h->ws_elems;
        if (!mok(h, mlp::launch_gemm(gw, h->stream), "gemm launch") ||
            !mok(h, mlp::launch_colsum(h->dzf[cur], batch, o, h->part, h->g + h->b_off[l], h->stream), "colsum launch"))
            return h->status;
        if (l == 0) break;
        // dz_{l-1}[B x i] = (dz [B x o] . W_l [o x i]) masked where act[l] (relu output) > 0
        mlp::GemmArgs gd{};
        gd.A = h->dzb[cur];
        gd.sam = o;
        gd.sak = 1;
        gd.B = h->pb + h->w_off[l];
        gd.sbk = i;
        gd.sbn = 1;
        gd.M = (int)batch;
        gd.N = i;
        gd.K = o;
        gd.mask = h->act[l];
        gd.Cf = h->dzf[cur ^ 1];
        gd.Cb = h->dzb[cur ^ 1];
        gd.ldc = i;
        if (!mok(h, mlp::launch_gemm(gd, h->stream), "gemm launch")) return h->status;
        cur ^= 1;
    }
    return PIC_OK;
}

int check_ready(mlp_handle* h) {
    if (!h) return PIC_EINVAL;
    return h->status;
}
}  // namespace

extern "C" {

int mlp_init(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t max_batch, uint64_t seed,
             void* hip_stream, mlp_handle** out) {
    if (!out) return mfail(nullptr, PIC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_in < 1 || n_in > 4096 || n_out < 1 || n_out > 4096 || width < 1 || width > 4096)
        return mfail(nullptr, PIC_EINVAL, "n_in, n_out and width must be in [1, 4096]");
    if (depth < 0 || depth > 16) return mfail(nullptr, PIC_EINVAL, "depth must be in [0, 16]");
    if (max_batch < 1 || max_batch > 65536) return mfail(nullptr, PIC_EINVAL, "max_batch must be in [1, 65536]");
    mlp_handle* h = new (std::nothrow) mlp_handle();
    if (!h) return mfail(nullptr, PIC_ENOMEM, "out of host memory");
    h->n_in = n_in;
    h->width = width;
    h->depth = depth;
    h->n_out = n_out;
    h->max_batch = max_batch;
    h->stream = static_cast<hipStream_t>(hip_stream);
    int prev = n_in;
    for (int l = 0; l <= depth; ++l) {
        const int o = l < depth ? width : n_out;
        h->in_dim.push_back(prev);
        h->out_dim.push_back(o);
        h->w_off.push_back(h->n_params);
        h->n_params += (int64_t)o * prev;
        h->b_off.push_back(h->n_params);
        h->n_params += o;
        prev = o;
    }
    const int64_t P = h->n_params;
    const int dmax = std::max(width, std::max(n_out, n_in));
    bool ok = alloc(h, &h->p, P) && alloc(h, &h->pb, P) && alloc(h, &h->g, P) && alloc(h, &h->m, P) &&
              alloc(h, &h->v, P) && alloc(h, &h->y, (int64_t)max_batch * n_out) && alloc(h, &h->loss, 1) &&
              alloc(h, &h->part, (int64_t)mlp::kColPartsHost * dmax);
    // up to 32 K-chunks of the largest weight gradient
    int64_t wmax = 0;
    for (int l = 0; l <= depth; ++l) wmax = std::max<int64_t>(wmax, (int64_t)h->out_dim[l] * h->in_dim[l]);
    h->ws_elems = 32 * wmax;
    ok = ok && alloc(h, &h->ws, h->ws_elems);
    for (int q = 0; ok && q < 2; ++q)
        ok = alloc(h, &h->dzf[q], (int64_t)max_batch * dmax) && alloc(h, &h->dzb[q], (int64_t)max_batch * dmax);
    h->act.assign(depth + 1, nullptr);
    for (int l = 0; ok && l <= depth; ++l) ok = alloc(h, &h->act[l], (int64_t)max_batch * h->in_dim[l]);
    if (!ok) {
        const std::string msg = h->err;
        mlp_free(h);
        return mfail(nullptr, PIC_ENOMEM, msg);
    }
    // He-uniform weights, zero biases
    std::vector<float> init((size_t)P, 0.0f);
    uint64_t s = seed;
    for (int l = 0; l <= depth; ++l) {
        const double a = std::sqrt(6.0 / (double)h->in_dim[l]);
        const int64_t nw = (int64_t)h->out_dim[l] * h->in_dim[l];
        for (int64_t k = 0; k < nw; ++k) {
            const double u = (double)(splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
            init[(size_t)(h->w_off[l] + k)] = (float)(a * (2.0 * u - 1.0));
        }
    }
    if (mlp_set_params(h, init.data(), P) != PIC_OK) {
        const std::string msg = h->err;
        mlp_free(h);
        return mfail(nullptr, PIC_EHIP, msg);
    }
    *out = h;
    return PIC_OK;
}

int mlp_num_params(const mlp_handle* h, int64_t* n) {
    if (!h || !n) return PIC_EINVAL;
    *n = h->n_params;
    return PIC_OK;
}

int mlp_set_params(mlp_handle* h, const float* host, int64_t n) {
    if (check_ready(h)) return h ? h->status : PIC_EINVAL;
    if (!host || n != h->n_params) return mfail(h, PIC_EINVAL, "host is NULL or n != number of parameters");
    if (!mok(h, hipMemcpyAsync(h->p, host, (size_t)n * sizeof(float), hipMemcpyHostToDevice, h->stream), "copy") ||
        !mok(h, mlp::launch_fill(h->m, n, 0.0f, h->stream), "fill") ||
        !mok(h, mlp::launch_fill(h->v, n, 0.0f, h->stream), "fill") ||
        !mok(h, mlp::launch_to_bf16(h->p, h->pb, n, h->stream), "convert") ||
        !mok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize"))
        return h->status;
    h->t = 0;
    return PIC_OK;
}

int mlp_get_params(mlp_handle* h, float* host, int64_t n) {
    if (check_ready(h)) return h ? h->status : PIC_EINVAL;
    if (!host || n != h->n_params) return mfail(h, PIC_EINVAL, "host is NULL or n != number of parameters");
    if (!mok(h, hipMemcpyAsync(host, h->p, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, h->stream), "copy") ||
        !mok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize"))
        return h->status;
    return PIC_OK;
}

int mlp_forward(mlp_handle* h, const float* x, int64_t batch, float* y) {
    if (check_ready(h)) return h ? h->status : PIC_EINVAL;
    if (!x || !y || batch < 1) return mfail(h, PIC_EINVAL, "x or y is NULL, or batch < 1");
    if (mlp::fused_forward_supported(h->n_in, h->width, n_layers(h))) {
        // one launch for every layer; the same products and roundings as the GEMM path
        mlp::FusedArgs a{};
        a.x = x;
        a.y = y;
        a.batch = batch;
        a.n_in = h->n_in;
        a.width = h->width;
        a.layers = n_layers(h);
        a.n_out = h->n_out;
        for (int l = 0; l < a.layers; ++l) {
            a.W[l] = h->pb + h->w_off[l];
            a.bias[l] = h->p + h->b_off[l];
        }
        if (!mok(h, mlp::launch_forward_fused(a, h->stream), "fused forward launch")) return h->status;
        return PIC_OK;
    }
    for (int64_t b0 = 0; b0 < batch; b0 += h->max_batch) {
        const int64_t nb = std::min<int64_t>(h->max_batch, batch - b0);
        if (!mok(h, mlp::launch_to_bf16(x + b0 * h->n_in, h->act[0], nb * h->n_in, h->stream), "convert"))
            return h->status;
        if (forward_from_act0(h, nb, y + b0 * h->n_out)) return h->status;
    }
    return PIC_OK;
}

int mlp_gradient(mlp_handle* h, const float* x, const float* t, int64_t batch, float* grad_host, double* loss) {
    if (check_ready(h)) return h ? h->status : PIC_EINVAL;
    if (!x || !t || batch < 1 || batch > h->max_batch)
        return mfail(h, PIC_EINVAL, "x or t is NULL, or batch outside [1, max_batch]");
    if (!mok(h, mlp::launch_to_bf16(x, h->act[0], batch * h->n_in, h->stream), "convert") ||
        forward_from_act0(h, batch, h->y) || backward(h, t, batch))
        return h->status;
    if (grad_host &&
        !mok(h, hipMemcpyAsync(grad_host, h->g, (size_t)h->n_params * sizeof(float), hipMemcpyDeviceToHost, h->stream),
             "copy"))
        return h->status;
    float l = 0.0f;
    if (!mok(h, hipMemcpyAsync(&l, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream), "copy") ||
        !mok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize"))
        return h->status;
    if (loss) *loss = l;
    return PIC_OK;
}

int mlp_train_step(mlp_handle* h, const float* x, const float* t, int64_t batch, float lr, float* loss_host) {
    if (check_ready(h)) return h ? h->status : PIC_EINVAL;
    if (!x || !t || batch < 1 || batch > h->max_batch)
        return mfail(h, PIC_EINVAL, "x or t is NULL, or batch outside [1, max_batch]");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return mfail(h, PIC_EINVAL, "lr must be finite and > 0");
    if (!mok(h, mlp::launch_to_bf16(x, h->act[0], batch * h->n_in, h->stream), "convert") ||
        forward_from_act0(h, batch, h->y) || backward(h, t, batch))
        return h->status;
    const float b1 = 0.9f, b2 = 0.999f;
    h->t += 1;
    const float c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)h->t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)h->t)));
    if (!mok(h, mlp::launch_adam(h->p, h->g, h->m, h->v, h->pb, h->n_params, lr, b1, b2, 1e-8f, c1, c2, h->stream),
             "adam launch"))
        return h->status;
    if (loss_host &&
        (!mok(h, hipMemcpyAsync(loss_host, h->loss, sizeof(float), hipMemcpyDeviceToHost, h->stream), "copy") ||
         !mok(h, hipStreamSynchronize(h->stream), "hipStreamSynchronize")))
        return h->status;
    return PIC_OK;
}

void mlp_free(mlp_handle* h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    for (void* q : h->allocs) (void)hipFree(q);
    delete h;
}

const char* mlp_last_error(const mlp_handle* h) {
    if (!h) return g_mlp_error.c_str();
    return h->err.c_str();
}

}  // extern "C"
