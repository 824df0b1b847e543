"""FP64 reference of the path cost model — TEST INFRASTRUCTURE ONLY.

The learned path selector predicts the log duration of a kernel step with a
two-hidden-layer perceptron,

    z1 = W1 x + b1,  h1 = relu(z1),  z2 = W2 h1 + b2,  h2 = relu(z2),
    y  = w3 . h2 + b3,

trained on the mean squared error L = (1/n) sum_s (y_s - t_s)^2 with Adam
(Kingma & Ba, 2015: first/second moment estimates with bias correction).
This module writes those definitions out in numpy float64, with the
gradients derived by hand through the chain rule, so that the GPU kernels
can be compared with it.  It shares nothing with the library.

Flat parameter layout (same order as the library's):
    W1 [H][F], b1 [H], W2 [H][H], b2 [H], w3 [H], b3 [1].
"""

from __future__ import annotations

import numpy as np

F = 26
H = 64


def unpack(p, f=F, h=H):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + h * f].reshape(h, f); o += h * f
    b1 = p[o:o + h]; o += h
    W2 = p[o:o + h * h].reshape(h, h); o += h * h
    b2 = p[o:o + h]; o += h
    w3 = p[o:o + h]; o += h
    b3 = p[o]; o += 1
    assert o == p.size
    return W1, b1, W2, b2, w3, b3


def param_count(f=F, h=H):
    return h * f + h + h * h + h + h + 1


def forward(p, X):
    """Predictions y [n] and the intermediate values needed by backward."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss(p, X, t):
    y, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def gradients(p, X, t):
    """Gradient of the mean squared error with respect to the flat
    parameters, by the chain rule: dL/dy_s = 2 (y_s - t_s) / n, then back
    through the output layer, the second ReLU (derivative 1 where z2 > 0),
    the second linear layer, the first ReLU and the first linear layer."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / n      # [n]
    g_w3 = h2.T @ dy                                           # [H]
    g_b3 = dy.sum()
    dz2 = np.outer(dy, w3) * (z2 > 0)                          # [n, H]
    g_W2 = dz2.T @ h1                                          # [H, H]
    g_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (z1 > 0)                                # [n, H]
    g_W1 = dz1.T @ X                                           # [H, F]
    g_b1 = dz1.sum(axis=0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def adam_step(p, m, v, g, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
