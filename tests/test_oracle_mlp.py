"""Pins of the oracle's reference MLP (the warm start's network)."""
import numpy as np

from oracle import mlp


def test_gradient_matches_central_differences():
    n_in, width, hidden, n_out = 7, 9, 3, 5
    g = np.random.Generator(np.random.PCG64(3))
    th = mlp.init(n_in, width, hidden, n_out, 1) + 0.05 * g.standard_normal(mlp.n_params(n_in, width, hidden, n_out))
    x = g.standard_normal((11, n_in))
    t = g.standard_normal((11, n_out))
    L, grad = mlp.loss_and_grad(th, x, t, n_in, width, hidden, n_out)
    h = 1e-6
    idx = g.choice(len(th), 60, replace=False)
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        fd = (mlp.loss_and_grad(th + e, x, t, n_in, width, hidden, n_out)[0]
              - mlp.loss_and_grad(th - e, x, t, n_in, width, hidden, n_out)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-7 * max(1.0, abs(fd)), (k, fd, grad[k])


def test_linear_network_closed_form():
    # no hidden layer: y = W x + b, L = |XW^T + b - T|^2 / (B n_out),
    # dL/dW = 2 (XW^T + b - T)^T X / (B n_out), dL/db = 2 sum_rows(...) / (B n_out)
    n_in, n_out, B = 4, 3, 8
    g = np.random.Generator(np.random.PCG64(9))
    W = g.standard_normal((n_out, n_in))
    b = g.standard_normal(n_out)
    th = np.concatenate([W.ravel(), b])
    X = g.standard_normal((B, n_in))
    T = g.standard_normal((B, n_out))
    L, grad = mlp.loss_and_grad(th, X, T, n_in, 0, 0, n_out)
    R = X @ W.T + b - T
    assert abs(L - np.sum(R * R) / (B * n_out)) < 1e-14
    gW = 2 * R.T @ X / (B * n_out)
    gb = 2 * R.sum(0) / (B * n_out)
    assert np.allclose(grad, np.concatenate([gW.ravel(), gb]), atol=1e-14)


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose(mlp.dsilu(z), (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h), atol=1e-9)


def test_warmstart_last_layer_offsets_match_layout():
    """The offsets the training code uses to fold the output scale into the last
    layer are those of the documented parameter layout (per layer W then b)."""
    from paper_1906_04209_amd import warmstart
    shape = (7, 5, 3, 4)
    n = mlp.n_params(*shape)
    th = np.arange(n, dtype=np.float64)
    layers = mlp.unflatten(th, *shape)
    W, b = layers[-1]
    w0, b0, n_prev, n_out = warmstart._last_layer(shape)
    assert (n_prev, n_out) == (5, 4)
    assert np.array_equal(th[w0:w0 + n_prev * n_out].reshape(n_out, n_prev), W)
    assert np.array_equal(th[b0:b0 + n_out], b)
