"""Pins of the NumPy MLP reference: backpropagation against central finite
differences, the linear special case against least-squares algebra."""
import numpy as np

import mlp_reference as ref


def _net(seed, dims):
    rng = np.random.default_rng(seed)
    n = sum(a * b + b for a, b in zip(dims[:-1], dims[1:]))
    return rng.normal(0, 0.5, n), rng.normal(size=(9, dims[0])), rng.normal(size=(9, dims[-1]))


def test_gradient_matches_finite_differences():
    dims = [6, 7, 5, 4]
    w, x, t = _net(1, dims)
    mask = (np.random.default_rng(2).random(t.shape) > 0.3).astype(np.float64)
    g = ref.gradient(w, dims, x, t, mask)
    fd = np.empty_like(w)
    h = 1e-6
    for i in range(w.size):
        e = np.zeros_like(w)
        e[i] = h
        fd[i] = (ref.loss(w + e, dims, x, t, mask) - ref.loss(w - e, dims, x, t, mask)) / (2 * h)
    assert np.max(np.abs(g - fd)) < 1e-7 * max(1.0, np.max(np.abs(fd)))


def test_single_linear_layer_gradient_is_normal_equations():
    # one linear layer: L = |x W^T + b - t|^2 / (B nout); dL/dW = 2 (xW^T + b - t)^T x / (B nout)
    dims = [3, 2]
    w, x, t = _net(3, dims)
    W, b = w[:6].reshape(2, 3), w[6:]
    r = x @ W.T + b - t
    expect = np.concatenate([(2 * r.T @ x / r.size).ravel(), 2 * r.sum(0) / r.size])
    assert np.allclose(ref.gradient(w, dims, x, t), expect, rtol=1e-13, atol=1e-14)
    # and its zero is the least-squares solution
    A = np.hstack([x, np.ones((x.shape[0], 1))])
    sol = np.linalg.lstsq(A, t, rcond=None)[0]
    w_ls = np.concatenate([sol[:3].T.ravel(), sol[3]])
    assert np.max(np.abs(ref.gradient(w_ls, dims, x, t))) < 1e-12


def test_adam_first_step_moves_by_lr_times_sign():
    # with bias correction the first Adam step is -lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    w1, _, _ = ref.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(w1, -0.01 * np.sign(g), rtol=1e-4)
