"""Pins of the cost-model oracle (oracle/mlp.py) against facts that do not
come from the oracle's own formulas: finite differences, a collapsed linear
map where every unit is active, a disconnected first layer, and the
closed form of bias-corrected Adam under a constant gradient."""

import numpy as np
import pytest

from oracle import mlp


def _params(rng, scale=1.0):
    p = np.zeros(mlp.param_count())
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)  # views into p
    W1[:] = rng.uniform(-1, 1, W1.shape) * np.sqrt(6 / mlp.F) * scale
    W2[:] = rng.uniform(-1, 1, W2.shape) * np.sqrt(6 / mlp.H) * scale
    w3[:] = rng.uniform(-1, 1, w3.shape) * np.sqrt(6 / mlp.H) * scale
    b1[:] = rng.uniform(-0.1, 0.1, b1.shape)
    b2[:] = rng.uniform(-0.1, 0.1, b2.shape)
    p[-1] = 0.3
    return p


def test_layout_views_and_count():
    p = np.arange(mlp.param_count(), dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    assert W1.shape == (64, 26) and W2.shape == (64, 64)
    assert W1[0, 1] == 1 and b1[0] == 64 * 26 and W2[0, 0] == 64 * 26 + 64
    assert b3 == mlp.param_count() - 1 == 5952


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = _params(rng)
    X = rng.uniform(0, 1.5, (16, mlp.F))
    t = rng.normal(1.0, 0.5, 16)
    g = mlp.gradients(p, X, t)
    idx = np.concatenate([rng.choice(p.size, 300, replace=False), [p.size - 1]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_forward_all_active_is_one_linear_map():
    # positive inputs, weights and biases: every ReLU passes its input, so
    # the network is the affine map x -> (W1^T W2^T w3) . x + const
    rng = np.random.default_rng(1)
    p = np.abs(_params(rng))
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    X = rng.uniform(0, 1, (32, mlp.F))
    a = np.linalg.multi_dot([W1.T, W2.T, w3])
    c = w3 @ (W2 @ b1 + b2) + b3
    y, _ = mlp.forward(p, X)
    np.testing.assert_allclose(y, X @ a + c, rtol=1e-12)


def test_zero_second_layer_disconnects_inputs():
    rng = np.random.default_rng(2)
    p = _params(rng)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p)
    W2[:] = 0.0
    X = rng.uniform(0, 2, (8, mlp.F))
    t = rng.normal(size=8)
    y, _ = mlp.forward(p, X)
    assert np.ptp(y) == 0.0
    assert y[0] == pytest.approx(w3 @ np.maximum(b2, 0) + b3)
    g = mlp.gradients(p, X, t)
    assert np.all(g[: 64 * mlp.F + 64] == 0.0)  # nothing reaches W1, b1


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments equal g and g^2
    # exactly, so every step moves each parameter by -lr g / (|g| + eps)
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, eps = 1e-2, 1e-8
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for k in range(1, 6):
        p, m, v = mlp.adam_step(p, m, v, g, lr, k)
        np.testing.assert_allclose(p, p0 - k * lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-14)
