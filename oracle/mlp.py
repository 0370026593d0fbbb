"""FP64 reference of the placement cost model: a 3-layer perceptron
d -> 64 -> 64 -> 1 with ReLU, mean-squared-error loss and Adam.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Parameter vector layout (flat, as the GPU kernels use it):
  W1 [64][d], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 [1].
Forward:  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3.
Loss:     L = (1/N) sum_s (y_s - t_s)^2.
Adam (Kingma & Ba): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
          p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps).
"""
from __future__ import annotations

import numpy as np

H = 64


def n_params(d: int) -> int:
    return H * d + H + H * H + H + H + 1


def unpack(p, d):
    p = np.asarray(p, dtype=np.float64)
    i = 0
    W1 = p[i:i + H * d].reshape(H, d); i += H * d
    b1 = p[i:i + H]; i += H
    W2 = p[i:i + H * H].reshape(H, H); i += H * H
    b2 = p[i:i + H]; i += H
    w3 = p[i:i + H]; i += H
    b3 = p[i]
    return W1, b1, W2, b2, w3, b3


def forward(p, X):
    X = np.asarray(X, dtype=np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(p, X.shape[1])
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    y = h2 @ w3 + b3
    return h1, h2, y


def loss(p, X, t):
    _, _, y = forward(p, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, X, t):
    """Gradient of the loss with respect to the flat parameter vector."""
    X = np.asarray(X, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    N, d = X.shape
    W1, b1, W2, b2, w3, b3 = unpack(p, d)
    h1, h2, y = forward(p, X)
    dy = 2.0 * (y - t) / N                  # dL/dy_s
    g_w3 = h2.T @ dy
    g_b3 = dy.sum()
    dh2 = np.outer(dy, w3) * (h2 > 0)       # through relu
    g_W2 = dh2.T @ h1
    g_b2 = dh2.sum(0)
    dh1 = (dh2 @ W2) * (h1 > 0)
    g_W1 = dh1.T @ X
    g_b1 = dh1.sum(0)
    return np.concatenate([g_W1.ravel(), g_b1, g_W2.ravel(), g_b2, g_w3, [g_b3]])


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
