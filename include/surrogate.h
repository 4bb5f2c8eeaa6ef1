/* Warm-start surrogate network: a multilayer perceptron from discharge parameters to the
 * cycle-averaged profiles of the periodic state, trained and evaluated on the GPU in BF16
 * on the matrix cores with FP32 accumulation and FP32 master weights.
 *
 * Basis: the periodic state does not depend on the initial density and energy, and a cold
 * start needs ~1000-4000 RF periods to reach it (Sec. 3, on initial values and the number
 * of periods); a prediction of that state is therefore a valid starting point that only
 * shortens the relaxation.  The network itself is not part of the paper's method.
 *
 * Network: depth hidden layers of `width` units with ReLU, then a linear output layer:
 *   h_1 = relu(W_1 x + b_1), ..., y = W_{depth+1} h_depth + b_{depth+1}.
 * Loss: mean squared error over all outputs of all samples, L = sum (y - t)^2 / (B n_out).
 * Optimizer: Adam (Kingma & Ba 2015, Algorithm 1), beta1 0.9, beta2 0.999, eps 1e-8.
 * Parameters are flat FP32, layer by layer: W_l row-major [out x in], then b_l [out].
 *
 * Status codes are those of pic1d.h (PIC_OK, PIC_EINVAL, PIC_ENOMEM, PIC_EHIP); the first
 * error poisons the handle.  x, t and y are DEVICE pointers to row-major FP32 arrays
 * ([batch x n_in], [batch x n_out]) on the handle's device; they are read or written on the
 * handle's stream, and the caller keeps them alive until that work has run. */
#ifndef PAPER_1608_04601_SURROGATE_H
#define PAPER_1608_04601_SURROGATE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlp_handle mlp_handle;

/* 1 <= n_in, n_out, width <= 4096; 0 <= depth <= 16; 1 <= max_batch <= 65536 (the
 * largest batch of one mlp_train_step / mlp_gradient call; mlp_forward takes any batch).
 * Weights: He-uniform, U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)), from a splitmix64 stream
 * of `seed`; biases zero.  hip_stream NULL = the null stream.  On error *out is NULL. */
int mlp_init(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, int32_t max_batch, uint64_t seed,
             void* hip_stream, mlp_handle** out);

/* Number of parameters. */
int mlp_num_params(const mlp_handle* h, int64_t* n);

/* Copy all n parameters from / to host memory (n must equal mlp_num_params); set also
 * resets the Adam moments and step count.  Both synchronise the stream. */
int mlp_set_params(mlp_handle* h, const float* host, int64_t n);
int mlp_get_params(mlp_handle* h, float* host, int64_t n);

/* y = network(x) for batch >= 1 samples; enqueued, returns without waiting. */
int mlp_forward(mlp_handle* h, const float* x, int64_t batch, float* y);

/* Loss and its gradient with respect to every parameter (no update), 1 <= batch <=
 * max_batch; copies n = mlp_num_params gradients to grad_host and the loss to *loss
 * (either may be NULL); synchronises. */
int mlp_gradient(mlp_handle* h, const float* x, const float* t, int64_t batch, float* grad_host, double* loss);

/* One Adam step on the loss of this batch with learning rate lr > 0; 1 <= batch <=
 * max_batch.  When loss_host is not NULL the batch's loss (before the update) is written
 * there and the call synchronises; otherwise it returns without waiting. */
int mlp_train_step(mlp_handle* h, const float* x, const float* t, int64_t batch, float lr, float* loss_host);

void mlp_free(mlp_handle* h);

/* Message for the last error of h (or of the last failed mlp_init when h is NULL). */
const char* mlp_last_error(const mlp_handle* h);

#ifdef __cplusplus
}
#endif

#endif
