"""Pins of the FP64 surrogate-network reference (oracle/mlp.py) against
finite differences and closed forms (CPU only)."""
import numpy as np

import workloads as W
from oracle import mlp as N


def _problem(sizes, B=7, seed=3):
    rng = np.random.default_rng(seed)
    theta = W.mlp_init(sizes, seed) + 0.05 * rng.standard_normal(N.n_params(sizes))
    X = rng.standard_normal((B, sizes[0]))
    T = rng.standard_normal((B, sizes[-1]))
    w = rng.uniform(0.5, 2.0, sizes[-1])
    return theta, X, T, w


def test_parameter_count_of_the_surrogate_architecture():
    assert N.n_params([4, 128, 128, 128, 9]) == 34825
    assert W.mlp_init([4, 128, 128, 128, 9]).size == 34825


def test_forward_of_hand_set_network():
    # y = tanh(x1) + tanh(x2) + 0.5 and y2 = tanh(x1) - 2 tanh(x2)
    theta = np.array([1, 0, 0, 1, 0, 0,        # W0 (2x2), b0
                      1, 1, 1, -2, 0.5, 0.0])  # W1 (2x2), b1
    X = np.array([[0.3, -1.2], [2.0, 0.1]])
    Y, _ = N.forward(theta, [2, 2, 2], X)
    t = np.tanh(X)
    assert np.allclose(Y[:, 0], t[:, 0] + t[:, 1] + 0.5, rtol=0, atol=1e-15)
    assert np.allclose(Y[:, 1], t[:, 0] - 2 * t[:, 1], rtol=0, atol=1e-15)


def test_gradient_against_central_differences():
    sizes = [4, 6, 5, 3]
    theta, X, T, w = _problem(sizes)
    L, g = N.loss_and_grad(theta, sizes, X, T, w)
    assert abs(L - N.loss(theta, sizes, X, T, w)) < 1e-14 * L
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        e = np.zeros_like(theta)
        e[i] = h
        fd[i] = (N.loss(theta + e, sizes, X, T, w) - N.loss(theta - e, sizes, X, T, w)) / (2 * h)
    assert np.abs(fd - g).max() < 1e-8 * np.abs(g).max()


def test_single_linear_layer_gradient_closed_form():
    # no hidden layer: y = W x + b, dL/dW = (2/B) sum_s w (y - t) x^T
    sizes = [3, 2]
    theta, X, T, w = _problem(sizes, B=5)
    Wm, b = theta[:6].reshape(2, 3), theta[6:]
    Y = X @ Wm.T + b
    R = 2.0 * w[None, :] * (Y - T) / 5
    _, g = N.loss_and_grad(theta, sizes, X, T, w)
    assert np.allclose(g[:6].reshape(2, 3), R.T @ X, rtol=1e-14, atol=1e-15)
    assert np.allclose(g[6:], R.sum(axis=0), rtol=1e-14, atol=1e-15)


def test_first_adam_step_is_a_sign_step():
    # zero moments: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
    rng = np.random.default_rng(0)
    theta = rng.standard_normal(10)
    g = rng.standard_normal(10)
    t1, m, v = N.adam_step(theta, g, np.zeros(10), np.zeros(10), 1, lr=1e-2)
    assert np.allclose(t1, theta - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_minimises_a_convex_quadratic():
    A = np.diag([1.0, 10.0, 100.0])
    x = np.array([1.0, -1.0, 0.5])
    m = v = np.zeros(3)
    for t in range(1, 3001):
        x, m, v = N.adam_step(x, A @ x, m, v, t, lr=1e-2)
    assert np.abs(x).max() < 1e-3
