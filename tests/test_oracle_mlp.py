"""Pins of the FP64 surrogate-network oracle against what the mathematics fixes: finite
differences of the loss, the closed form of the first Adam step, and least squares for a
network without hidden layers."""
import numpy as np

from oracle import mlp


def _net(seed=0, n_in=4, width=7, depth=2, n_out=5, batch=9):
    rng = np.random.default_rng(seed)
    shapes = mlp.layer_shapes(n_in, width, depth, n_out)
    theta = rng.normal(0.0, 0.6, mlp.n_params(shapes))
    X = rng.normal(size=(batch, n_in))
    T = rng.normal(size=(batch, n_out))
    return shapes, theta, X, T


def test_shapes_and_parameter_count():
    shapes = mlp.layer_shapes(4, 256, 3, 640)
    assert shapes == [(256, 4), (256, 256), (256, 256), (640, 256)]
    assert mlp.n_params(shapes) == 4 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 640 + 640 == 297_344


def test_gradient_matches_central_differences():
    for seed in range(3):
        shapes, theta, X, T = _net(seed)
        g = mlp.gradient(theta, shapes, X, T)
        h = 1e-6
        fd = np.empty_like(theta)
        for k in range(theta.size):
            e = np.zeros_like(theta)
            e[k] = h
            fd[k] = (mlp.loss(theta + e, shapes, X, T) - mlp.loss(theta - e, shapes, X, T)) / (2 * h)
        # relu kinks are measure-zero for these random draws; the FD error is O(h^2)
        assert np.max(np.abs(g - fd)) <= 1e-7 * max(1.0, np.abs(fd).max())


def test_a_dropped_relu_mask_is_caught():
    """The FD pin distinguishes the masked backward from an unmasked one."""
    shapes, theta, X, T = _net(1)
    g = mlp.gradient(theta, shapes, X, T)
    layers = mlp.unpack(theta, shapes)
    acts = mlp.forward(theta, shapes, X)
    dz = 2.0 * (acts[-1] - T) / acts[-1].size
    dh = dz @ layers[-1][0]   # no mask
    wrong = dh.T @ acts[-3]
    o, i = shapes[-2]
    k = mlp.n_params(shapes[:-2])
    assert not np.allclose(g[k:k + o * i].reshape(o, i), wrong)


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(3)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = mlp.Adam(50, lr=0.01, eps=1e-8)
    new = opt.step(theta, g)
    # m_hat = g and v_hat = g^2 after one step
    np.testing.assert_allclose(new, theta - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


def test_linear_network_converges_to_least_squares():
    rng = np.random.default_rng(4)
    X = rng.normal(size=(64, 3))
    A = rng.normal(size=(3, 2))
    T = X @ A + 0.1 * rng.normal(size=(64, 2)) + np.array([0.5, -1.0])
    shapes = mlp.layer_shapes(3, 0, 0, 2)
    theta = np.zeros(mlp.n_params(shapes))
    opt = mlp.Adam(theta.size, lr=0.05)
    for _ in range(3000):
        theta = opt.step(theta, mlp.gradient(theta, shapes, X, T))
    (W, b), = mlp.unpack(theta, shapes)
    sol, *_ = np.linalg.lstsq(np.hstack([X, np.ones((64, 1))]), T, rcond=None)
    np.testing.assert_allclose(W.T, sol[:3], atol=1e-4)
    np.testing.assert_allclose(b, sol[3], atol=1e-4)
