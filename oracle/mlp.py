"""FP64 reference of the surrogate network (test infrastructure).

The surrogate is not part of the paper: it is the learned stand-in for the
RVE response of the nested scheme (Sec. 4.1), mapping a macro strain measure
and a microstructure descriptor to the homogenized stress and tangent.  This
module is the plain definition the GPU kernels are checked against:

* a multilayer perceptron y = W_L h_{L-1} + b_L, h_l = tanh(W_l h_{l-1} + b_l),
  h_0 = x, with W_l of shape (out, in);
* the flat parameter layout: layer after layer, W_l row-major then b_l;
* the loss L = (1/B) sum_s sum_o w_o (y_so - t_so)^2 and its gradient by
  reverse-mode differentiation (the chain rule written out per layer);
* one Adam step (Kingma and Ba, 2015) with bias correction.

Everything is FP64 NumPy; pins against finite differences and closed forms
are in tests/test_mlp_oracle.py.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def n_params(sizes: Sequence[int]) -> int:
    return int(sum(sizes[i + 1] * sizes[i] + sizes[i + 1] for i in range(len(sizes) - 1)))


def unflatten(theta: np.ndarray, sizes: Sequence[int]) -> List[Tuple[np.ndarray, np.ndarray]]:
    """Flat parameter vector -> [(W_l (out, in), b_l (out,)), ...]."""
    out, k = [], 0
    for i in range(len(sizes) - 1):
        n_in, n_out = sizes[i], sizes[i + 1]
        W = theta[k:k + n_out * n_in].reshape(n_out, n_in)
        k += n_out * n_in
        b = theta[k:k + n_out]
        k += n_out
        out.append((W, b))
    assert k == theta.size
    return out


def forward(theta, sizes, X) -> Tuple[np.ndarray, List[np.ndarray]]:
    """X (B, n_in) -> Y (B, n_out) and the activations [h_0, ..., h_{L-1}]."""
    layers = unflatten(np.asarray(theta, dtype=np.float64), sizes)
    h = np.asarray(X, dtype=np.float64)
    acts = [h]
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if i < len(layers) - 1:
            h = np.tanh(z)
            acts.append(h)
        else:
            h = z
    return h, acts


def loss(theta, sizes, X, T, w_out) -> float:
    Y, _ = forward(theta, sizes, X)
    B = Y.shape[0]
    return float(np.sum(np.asarray(w_out)[None, :] * (Y - T) ** 2) / B)


def loss_and_grad(theta, sizes, X, T, w_out) -> Tuple[float, np.ndarray]:
    """Loss and dL/dtheta (flat, same layout as theta)."""
    theta = np.asarray(theta, dtype=np.float64)
    layers = unflatten(theta, sizes)
    Y, acts = forward(theta, sizes, X)
    B = Y.shape[0]
    w_out = np.asarray(w_out, dtype=np.float64)
    L = float(np.sum(w_out[None, :] * (Y - T) ** 2) / B)
    dz = 2.0 * w_out[None, :] * (Y - T) / B          # dL/d(pre-activation of the output layer)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        h_in = acts[i]
        grads[i] = (dz.T @ h_in, dz.sum(axis=0))     # dL/dW_l, dL/db_l
        if i > 0:
            dh = dz @ W                               # dL/dh_{l-1}
            dz = dh * (1.0 - acts[i] ** 2)            # tanh' = 1 - tanh^2
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, g


def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
