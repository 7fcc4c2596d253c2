"""Pins of the FP64 perceptron reference used to check the device training
kernels: the closed-form gradient of a linear least-squares layer, and
central differences through the tanh layers."""
import numpy as np

from oracle import mlp


def test_linear_layer_gradient_closed_form():
    # one linear layer: loss = |W X + b 1^T - T|^2 / n, so
    # dW = 2 (W X + b - T) X^T / n, db = 2 sum_cols (W X + b - T) / n
    g = np.random.default_rng(3)
    dims = [4, 3]
    p = g.standard_normal(mlp.n_params(dims))
    X = g.standard_normal((4, 7))
    T = g.standard_normal((3, 7))
    W, b = p[:12].reshape(3, 4), p[12:]
    R = W @ X + b[:, None] - T
    n = R.size
    loss, grad = mlp.loss_and_grad(p, dims, X, T)
    assert abs(loss - np.sum(R ** 2) / n) <= 1e-14 * loss
    assert np.allclose(grad[:12], (2 * R @ X.T / n).ravel(), rtol=1e-13, atol=1e-15)
    assert np.allclose(grad[12:], 2 * R.sum(axis=1) / n, rtol=1e-13, atol=1e-15)


def test_deep_gradient_matches_central_differences():
    g = np.random.default_rng(4)
    dims = [3, 6, 5, 4, 2]
    p = 0.5 * g.standard_normal(mlp.n_params(dims))
    X = g.standard_normal((3, 5))
    T = g.standard_normal((2, 5))
    _, grad = mlp.loss_and_grad(p, dims, X, T)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss_and_grad(p + e, dims, X, T)[0] - mlp.loss_and_grad(p - e, dims, X, T)[0]) / (2 * h)
    assert np.abs(grad - fd).max() <= 1e-8 * np.abs(fd).max()


def test_forward_layout_and_activation():
    # a two-layer net with hand-set weights: hidden tanh, linear output
    dims = [2, 2, 1]
    W1 = np.array([[1.0, 0.0], [0.0, 2.0]])
    b1 = np.array([0.5, -0.5])
    W2 = np.array([[3.0, -1.0]])
    b2 = np.array([0.25])
    p = np.concatenate([W1.ravel(), b1, W2.ravel(), b2])
    X = np.array([[1.0], [2.0]])
    y = mlp.forward(p, dims, X)[-1]
    expect = 3.0 * np.tanh(1.5) - np.tanh(3.5) + 0.25
    assert abs(y[0, 0] - expect) <= 1e-15
