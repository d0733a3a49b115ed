"""Pins of the warm-start network oracle: finite differences and closed forms."""
import numpy as np

from oracle import mlp


def test_silu_closed_form():
    z = np.linspace(-5, 5, 11)
    np.testing.assert_allclose(mlp.silu(z), z * (1 / (1 + np.exp(-z))), rtol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.silu_grad(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), atol=1e-9)


def test_gradient_matches_central_differences():
    d, w, L = 5, 12, 3
    rng = np.random.default_rng(0)
    th = mlp.init_params(d, w, L, seed=1) + 0.01 * rng.standard_normal(mlp.n_params(d, w, L))
    X = rng.standard_normal((40, d))
    T = rng.standard_normal(40)
    loss, g = mlp.loss_and_grad(th, X, T, d, w, L)
    h = 1e-6
    for k in rng.choice(th.size, 40, replace=False):
        e = np.zeros_like(th)
        e[k] = h
        fd = (mlp.loss_and_grad(th + e, X, T, d, w, L)[0] - mlp.loss_and_grad(th - e, X, T, d, w, L)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_linear_network_reduces_to_least_squares_gradient():
    # depth 0: y = X W + b, dL/dW = 2/n X^T (y - t), dL/db = 2/n sum(y - t)
    d = 4
    rng = np.random.default_rng(3)
    th = rng.standard_normal(mlp.n_params(d, 7, 0))
    X = rng.standard_normal((25, d))
    T = rng.standard_normal(25)
    loss, g = mlp.loss_and_grad(th, X, T, d, 7, 0)
    W, b = th[:d], th[d]
    r = X @ W + b - T
    assert abs(loss - np.mean(r ** 2)) < 1e-14
    np.testing.assert_allclose(g[:d], 2 / 25 * X.T @ r, rtol=1e-13)
    assert abs(g[d] - 2 / 25 * r.sum()) < 1e-13


def test_adam_first_step_is_signed_lr():
    # with bias correction the first Adam step is -lr * g / (|g| + eps)
    opt = mlp.Adam(3)
    g = np.array([0.5, -2.0, 1e-3])
    th = opt.step(np.zeros(3), g, 0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_adam_training_fits_a_smooth_function():
    rng = np.random.default_rng(5)
    d, w, L = 2, 16, 2
    X = rng.uniform(-1, 1, (256, d))
    T = np.sin(2 * X[:, 0]) * X[:, 1]
    th = mlp.init_params(d, w, L, seed=2)
    opt = mlp.Adam(th.size)
    l0 = mlp.loss_and_grad(th, X, T, d, w, L)[0]
    for _ in range(400):
        l, g = mlp.loss_and_grad(th, X, T, d, w, L)
        th = opt.step(th, g, 0.01)
    assert l < 0.1 * l0
