"""Pins of the FP64 adjoint of the Cholesky solve (the differentiation part)
against central finite differences of the oracle's own forward solve, against
torch's float64 autograd of a dense solve, and against the closed form for a
diagonal A."""
import numpy as np
import pytest

import oracle
from paper_2609_28179_amd import inputs


def loss_and_grads(A, B, W):
    L, X, info = oracle.posv(A, B)
    assert (info == 0).all()
    dB, dA = oracle.posv_adjoint(L, X, W)
    return X, dB, dA


@pytest.mark.parametrize("n,r", [(1, 1), (3, 2), (12, 1), (7, 4)])
def test_adjoint_matches_central_differences(n, r):
    rng = np.random.default_rng(10 * n + r)
    A = inputs.spd64(rng, 2, n)
    B = rng.uniform(-1, 1, size=(2, n, r))
    W = rng.standard_normal(size=(2, n, r))
    X, dB, dA = loss_and_grads(A, B, W)
    eps = 1e-6

    def f(Ap, Bp):
        _, Xp, _ = oracle.posv(Ap, Bp)
        return np.sum(W * Xp, axis=(1, 2))

    for q in range(2):
        for i in range(n):
            for c in range(r):
                Bp, Bm = B.copy(), B.copy()
                Bp[:, i, c] += eps
                Bm[:, i, c] -= eps
                fd = (f(A, Bp) - f(A, Bm))[q] / (2 * eps)
                assert abs(fd - dB[q, i, c]) <= 1e-7 * max(1.0, abs(fd))
        for i in range(n):
            for j in range(i + 1):
                S = np.zeros((n, n))
                S[i, j] = S[j, i] = 1.0  # symmetric perturbation direction
                Ap, Am = A.copy(), A.copy()
                Ap[q] += eps * S
                Am[q] -= eps * S
                fd = (f(Ap, B) - f(Am, B))[q] / (2 * eps)
                an = np.sum(dA[q] * S)
                assert abs(fd - an) <= 1e-7 * max(1.0, abs(fd)), (i, j, fd, an)


def test_adjoint_matches_torch_autograd_symmetrized():
    import torch
    rng = np.random.default_rng(3)
    n, r = 9, 3
    A = inputs.spd64(rng, 4, n)
    B = rng.uniform(-1, 1, size=(4, n, r))
    W = rng.standard_normal(size=(4, n, r))
    X, dB, dA = loss_and_grads(A, B, W)
    At = torch.tensor(A, requires_grad=True)
    Bt = torch.tensor(B, requires_grad=True)
    (torch.linalg.solve(At, Bt) * torch.tensor(W)).sum().backward()
    gA = At.grad.numpy()
    assert np.max(np.abs(Bt.grad.numpy() - dB)) <= 1e-12
    assert np.max(np.abs(0.5 * (gA + np.swapaxes(gA, 1, 2)) - dA)) <= 1e-12


def test_adjoint_diagonal_closed_form():
    d = np.array([[2.0, 4.0, 8.0]])
    A = np.stack([np.diag(d[0])])
    b = np.array([[[1.0], [2.0], [-3.0]]])
    w = np.array([[[0.5], [1.0], [2.0]]])
    X, dB, dA = loss_and_grads(A, b, w)
    # x_i = b_i / d_i, db_i = w_i / d_i, dA_ii = -db_i x_i, dA_ij = -(db_i x_j + x_i db_j)/2
    x = b[0, :, 0] / d[0]
    g = w[0, :, 0] / d[0]
    assert np.allclose(dB[0, :, 0], g, rtol=0, atol=1e-15)
    exp = -0.5 * (np.outer(g, x) + np.outer(x, g))
    assert np.allclose(dA[0], exp, rtol=0, atol=1e-15)
