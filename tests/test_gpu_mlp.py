"""Surrogate network on the GPU (BF16 MFMA, FP32 accumulation) against the FP64 oracle
network, through the C ABI (include/surrogate.h).

Tolerance: the GPU rounds the inputs, the weights and every hidden activation (and, in the
backward pass, every dL/dz) to BF16, whose unit roundoff is 2^-9 ~ 2e-3.  With four
rounded operands per layer over up to four layers, the result carries a relative error of
a few times 1e-2 at most in the max norm; the tests allow 3e-2 of each tensor's largest
magnitude (forward), a relative L2 error of 3e-2 for the gradient, and require the
gradient's direction (cosine) to agree to 0.999.  The shapes include ragged tiles
(dimensions that are not multiples of the GEMM tiles) and a batch whose weight gradients
split K across workgroups."""
import numpy as np
import pytest
import torch

from gpu_common import log
from oracle import mlp as O
from paper_1608_04601_amd import binding as B

pytestmark = pytest.mark.gpu

SHAPES = {"surrogate_4x256x3x640": (4, 256, 3, 640, 512), "ragged_5x70x2x33": (5, 70, 2, 33, 77),
          # batch 2048: the weight gradients split K over several workgroups
          "surrogate_batch2048": (4, 256, 3, 640, 2048),
          # the one-launch forward pass: a batch that is not a multiple of its 64-sample
          # tile, and a wider input with a narrower network (width 70 above takes the
          # layer-by-layer products)
          "surrogate_batch1001": (4, 256, 3, 640, 1001), "fused_20x64x2x40": (20, 64, 2, 40, 300)}


def _data(n_in, n_out, batch, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(-1.0, 1.0, (batch, n_in)).astype(np.float32)
    T = rng.normal(0.0, 1.0, (batch, n_out)).astype(np.float32)
    return X, T


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("case", list(SHAPES))
def test_forward_and_gradient_match_oracle(case):
    n_in, width, depth, n_out, batch = SHAPES[case]
    log(f"mlp parity: {case}")
    X, T = _data(n_in, n_out, batch, seed=1)
    with B.Mlp(n_in, width, depth, n_out, max_batch=batch, seed=7) as net:
        theta = net.get_params().astype(np.float64)
        shapes = O.layer_shapes(n_in, width, depth, n_out)
        assert net.n_params == O.n_params(shapes)
        y = torch.empty(batch, n_out, device="cuda")
        net.forward(_dev(X), y)
        torch.cuda.synchronize()
        yo = O.forward(theta, shapes, X.astype(np.float64))[-1]
        err = np.abs(y.cpu().numpy() - yo).max()
        assert err <= 3e-2 * np.abs(yo).max(), err
        g, loss = net.gradient(_dev(X), _dev(T))
        go = O.gradient(theta, shapes, X.astype(np.float64), T.astype(np.float64))
        lo = O.loss(theta, shapes, X.astype(np.float64), T.astype(np.float64))
        assert abs(loss - lo) <= 3e-2 * lo
        rel = np.linalg.norm(g - go) / np.linalg.norm(go)
        cos = float(g @ go / (np.linalg.norm(g) * np.linalg.norm(go)))
        log(f"  forward max err {err:.3e}, gradient rel L2 {rel:.3e}, cosine {cos:.6f}")
        assert rel <= 3e-2 and cos >= 0.999
        # every layer's block, not only the whole vector
        k = 0
        for o, i in shapes:
            for n in (o * i, o):
                blk, blko = g[k:k + n], go[k:k + n]
                assert np.linalg.norm(blk - blko) <= 5e-2 * np.linalg.norm(blko) + 1e-7, (o, i, n)
                k += n


def test_first_adam_step_matches_oracle():
    n_in, width, depth, n_out, batch = SHAPES["ragged_5x70x2x33"]
    X, T = _data(n_in, n_out, batch, seed=2)
    lr = 1e-3
    with B.Mlp(n_in, width, depth, n_out, max_batch=batch, seed=3) as net:
        theta = net.get_params().astype(np.float64)
        shapes = O.layer_shapes(n_in, width, depth, n_out)
        net.train_step(_dev(X), _dev(T), lr)
        after = net.get_params().astype(np.float64)
    go = O.gradient(theta, shapes, X.astype(np.float64), T.astype(np.float64))
    expect = O.Adam(theta.size, lr=lr).step(theta, go) - theta   # = -lr g / (|g| + eps)
    # where the gradient is clearly non-zero its sign, hence the first step, is unambiguous
    sure = np.abs(go) > 0.05 * np.abs(go).max()
    assert sure.sum() > 100
    np.testing.assert_allclose((after - theta)[sure], expect[sure], rtol=0, atol=1e-2 * lr)
    assert np.all(np.abs(after - theta) <= lr * (1 + 1e-3))


def test_training_reduces_the_loss_checked_by_the_oracle():
    """A smooth map of 4 inputs to 640 outputs (the surrogate's shapes); after training the
    oracle evaluates the trained parameters independently."""
    rng = np.random.default_rng(5)
    n_in, width, depth, n_out, batch = 4, 256, 3, 640, 512
    X = rng.uniform(-1.0, 1.0, (batch, n_in))
    grid = np.linspace(0.0, 1.0, n_out // 5)
    prof = [np.sin(np.pi * grid[None, :] * (1 + X[:, :1])) * (1 + 0.5 * X[:, 1:2]),
            np.cos(np.pi * grid[None, :]) * X[:, 2:3], np.exp(-grid[None, :] * (2 + X[:, 3:4])),
            grid[None, :] * X[:, :1] * X[:, 1:2], np.tanh(3 * (grid[None, :] - 0.5) * X[:, 2:3])]
    T = np.concatenate(prof, axis=1)
    shapes = O.layer_shapes(n_in, width, depth, n_out)
    with B.Mlp(n_in, width, depth, n_out, max_batch=batch, seed=11) as net:
        l0 = O.loss(net.get_params().astype(np.float64), shapes, X, T)
        xd, td = _dev(X), _dev(T)
        for it in range(600):
            net.train_step(xd, td, 2e-3 if it < 400 else 5e-4)
        l1 = O.loss(net.get_params().astype(np.float64), shapes, X, T)
    log(f"  training loss (oracle-evaluated): {l0:.4e} -> {l1:.4e}")
    assert l1 <= 0.02 * l0


def test_invalid_batches_are_rejected():
    with B.Mlp(4, 16, 1, 8, max_batch=32) as net:
        x = torch.zeros(64, 4, device="cuda")
        t = torch.zeros(64, 8, device="cuda")
        with pytest.raises(B.PicError):
            net.train_step(x, t, 1e-3)
    with B.Mlp(4, 16, 1, 8, max_batch=32) as net:
        y = torch.empty(64, 8, device="cuda")
        net.forward(torch.zeros(64, 4, device="cuda"), y)   # forward takes any batch, in chunks
        torch.cuda.synchronize()
        assert torch.isfinite(y).all()
