"""FP64 CPU oracle of the warm-start surrogate network (TEST INFRASTRUCTURE ONLY).

The paper reports that the periodic state of a discharge does not depend on the initial
density and energy (Sec. 3, remark on initial values) and that reaching it takes ~1000 to
~4000 RF periods.  The surrogate is a plain multilayer perceptron from the discharge
parameters to the cycle-averaged profiles of that periodic state; it is not part of the
paper's method, so this module follows the textbook definitions named in each function.

Network: x -> h_1 = relu(W_1 x + b_1) -> ... -> h_L = relu(W_L h_{L-1} + b_L)
            -> y = W_{L+1} h_L + b_{L+1}   (linear output).
Loss: mean squared error over every output of every sample, L = sum (y - t)^2 / (B n_out).
Parameters are stored flat, layer by layer, W_l row-major [out x in] then b_l [out].
Optimizer: Adam (Kingma & Ba 2015, Algorithm 1) with bias-corrected moments.

Pins (tests/test_oracle_mlp.py, not gpu): central finite differences of the loss against
the backward pass; the first Adam step equals -lr * g / (|g| + eps) elementwise; a network
with no hidden layer reduces to least squares, whose minimiser is numpy's lstsq.
"""
import numpy as np


def layer_shapes(n_in, width, depth, n_out):
    """(out, in) of every affine map: depth hidden layers of `width`, then the output."""
    dims = [n_in] + [width] * depth + [n_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def n_params(shapes):
    return sum(o * i + o for o, i in shapes)


def unpack(theta, shapes):
    """Views (W_l, b_l) into the flat parameter vector."""
    out, k = [], 0
    for o, i in shapes:
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


def forward(theta, shapes, X):
    """Activations of every layer for the batch X [B x n_in]; the last entry is y."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(np.asarray(theta, dtype=np.float64), shapes)
    for li, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(z if li == len(layers) - 1 else np.maximum(z, 0.0))
    return acts


def loss(theta, shapes, X, T):
    y = forward(theta, shapes, X)[-1]
    return float(np.sum((y - T) ** 2) / y.size)


def gradient(theta, shapes, X, T):
    """dL/dtheta by the chain rule, layer by layer from the output back (reverse mode)."""
    theta = np.asarray(theta, dtype=np.float64)
    acts = forward(theta, shapes, X)
    layers = unpack(theta, shapes)
    y = acts[-1]
    dz = 2.0 * (y - T) / y.size            # dL/dz of the linear output layer
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h_in = acts[li]
        grads.append((dz.T @ h_in, dz.sum(axis=0)))
        if li > 0:
            dh = dz @ W
            dz = dh * (acts[li] > 0.0)      # relu passes the gradient where its output is positive
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db)
    return np.concatenate(flat)


class Adam:
    """Adam with bias correction (Kingma & Ba 2015, Algorithm 1), FP64."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)
