"""Pins of the FP64 cost-model reference: its gradient against central finite
differences of its own loss, its forward pass against a plain per-sample loop,
and Adam's first step against its closed form."""
import numpy as np

from oracle import mlp
from paper_2609_28179_amd.inputs import mlp_init


def data(N=37, d=14, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((N, d)), rng.standard_normal(N)


def test_forward_matches_per_sample_loop():
    X, _ = data()
    p = mlp_init(14, 1)
    _, _, y = mlp.forward(p, X)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(p, 14)
    for s in range(len(X)):
        h1 = [max(0.0, sum(W1[j, i] * X[s, i] for i in range(14)) + b1[j]) for j in range(64)]
        h2 = [max(0.0, sum(W2[j, k] * h1[k] for k in range(64)) + b2[j]) for j in range(64)]
        ys = sum(w3[j] * h2[j] for j in range(64)) + b3
        assert abs(ys - y[s]) <= 1e-12 * max(1.0, abs(ys))


def test_gradient_matches_central_differences():
    X, t = data(N=23)
    p = mlp_init(14, 2)
    p[14 * 64: 14 * 64 + 64] = 0.05       # nonzero biases so every block is exercised
    g = mlp.grad(p, X, t)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(len(p), 60, replace=False), [len(p) - 1, 0, 14 * 64]])
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        fd = (mlp.loss(p + e, X, t) - mlp.loss(p - e, X, t)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    p1, m, v = mlp.adam_step(p, g, np.zeros(100), np.zeros(100), 1, lr=1e-3)
    # after one step the bias-corrected moments are g and g^2
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert mlp.n_params(14) == 5185
