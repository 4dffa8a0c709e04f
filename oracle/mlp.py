"""FP64 reference multilayer perceptron for the learned warm start.

TEST INFRASTRUCTURE (oracle). Plain numpy: forward pass, mean-squared-error
loss and its gradient by backpropagation. The GPU network must reproduce
these numbers (forward and gradients) to single-precision accuracy.

Architecture (the learned warm start of the hot path's AI-systems form):
  x (n_in) -> [W_l x + b_l, SiLU] for each hidden layer -> W_out h + b_out (n_out)
SiLU(z) = z / (1 + exp(-z)). Parameters are flattened layer by layer as
W (row-major, n_out_l x n_in_l) then b.
Loss: L = (1 / (B n_out)) sum (y - t)^2.

Pins (tests/test_oracle_mlp.py): gradients vs central finite differences;
a network without hidden layers reduces to linear least squares, whose
gradient has a closed form.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def shapes(n_in: int, width: int, hidden: int, n_out: int) -> List[Tuple[int, int]]:
    dims = [n_in] + [width] * hidden + [n_out]
    return [(dims[k + 1], dims[k]) for k in range(len(dims) - 1)]


def n_params(n_in, width, hidden, n_out) -> int:
    return sum(o * i + o for o, i in shapes(n_in, width, hidden, n_out))


def unflatten(theta: np.ndarray, n_in, width, hidden, n_out):
    out = []
    k = 0
    for o, i in shapes(n_in, width, hidden, n_out):
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x, n_in, width, hidden, n_out):
    """Returns (y, cache) for a batch x (B x n_in)."""
    layers = unflatten(theta, n_in, width, hidden, n_out)
    h = x
    cache = []
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = silu(z) if li < len(layers) - 1 else z
    return h, cache


def loss_and_grad(theta, x, t, n_in, width, hidden, n_out):
    layers = unflatten(theta, n_in, width, hidden, n_out)
    y, cache = forward(theta, x, n_in, width, hidden, n_out)
    B = x.shape[0]
    diff = y - t
    loss = float(np.sum(diff * diff) / (B * n_out))
    g = 2.0 * diff / (B * n_out)            # dL/dy
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        h, z = cache[li]
        if li < len(layers) - 1:
            g = g * dsilu(z)
        grads.append((g.T @ h, g.sum(axis=0)))
        g = g @ W
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def init(n_in, width, hidden, n_out, seed: int) -> np.ndarray:
    """He-style initialisation (normal, std sqrt(2 / fan_in)), zero biases."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for o, i in shapes(n_in, width, hidden, n_out):
        parts.append(g.standard_normal(o * i) * np.sqrt(2.0 / i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)
