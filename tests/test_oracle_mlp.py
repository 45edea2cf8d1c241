"""Pins of the fp64 network oracle (the cost model's reference).

Backpropagation is pinned by central finite differences of the loss, a
one-layer network by the closed-form gradient of linear least squares, and
Adam by its first step, which moves every parameter by lr * sign(g)."""
import numpy as np

from oracle import mlp


def _setup(widths, n=7, seed=3):
    rng = np.random.default_rng(seed)
    n_par = sum(a * b + b for a, b in zip(widths[:-1], widths[1:]))
    return rng.normal(0, 0.5, n_par), rng.normal(0, 1, (n, widths[0])), rng.normal(0, 1, (n, widths[-1]))


def test_gradient_equals_finite_differences():
    widths = (5, 7, 4, 2)
    p, X, Y = _setup(widths)
    loss, g = mlp.loss_and_grad(p, widths, X, Y)
    h = 1e-6
    num = np.empty_like(p)
    for i in range(len(p)):
        e = np.zeros_like(p)
        e[i] = h
        num[i] = (mlp.loss_and_grad(p + e, widths, X, Y)[0] - mlp.loss_and_grad(p - e, widths, X, Y)[0]) / (2 * h)
    assert np.allclose(g, num, rtol=1e-5, atol=1e-8)


def test_one_layer_is_linear_least_squares():
    widths = (6, 1)
    p, X, Y = _setup(widths, n=11)
    W, b = p[:6], p[6]
    r = X @ W + b - Y[:, 0]
    loss, g = mlp.loss_and_grad(p, widths, X, Y)
    assert np.isclose(loss, np.mean(r ** 2))
    assert np.allclose(g[:6], 2.0 / len(r) * X.T @ r)
    assert np.isclose(g[6], 2.0 / len(r) * r.sum())


def test_relu_blocks_gradient_of_inactive_units():
    widths = (3, 4, 1)
    p, X, Y = _setup(widths, n=5)
    layers = mlp.unpack(p, widths)
    # push hidden unit 2 negative for every row: its incoming weights get no gradient
    W0, b0 = layers[0]
    W0[2] = 0.0
    b0[2] = -5.0
    _, g = mlp.loss_and_grad(p, widths, X, Y)
    assert np.all(g[2 * 3:3 * 3] == 0.0) and g[12 + 2] == 0.0


def test_adam_first_step_is_signed_learning_rate():
    p = np.array([0.3, -1.2, 2.0])
    g = np.array([0.5, -2e-3, 7.0])
    q, m, v = mlp.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(q - p, -0.01 * np.sign(g), rtol=1e-5)
