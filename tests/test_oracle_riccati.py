"""Pins of the FP64 oracle's LQR gain K = (R + B^T P B)^{-1} B^T P A and of
its transposed GEMM: closed forms, a decoupled diagonal case, exact rational
arithmetic on a tiny integer case, the discrete algebraic Riccati equation
with P from scipy's Schur-method solver, and the stationarity residual."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2609_28179_amd import inputs


def test_gemm_t_integer_exact_and_transposed_copies():
    rng = np.random.default_rng(0)
    for ta in (0, 1):
        for tb in (0, 1):
            m, n, k = 5, 7, 3
            A = rng.integers(-2, 3, size=(4, k, m) if ta else (4, m, k)).astype(np.float64)
            B = rng.integers(-2, 3, size=(4, n, k) if tb else (4, k, n)).astype(np.float64)
            opA = np.swapaxes(A, 1, 2) if ta else A
            opB = np.swapaxes(B, 1, 2) if tb else B
            want = np.einsum("bik,bkj->bij", opA, opB)
            got = oracle.gemm_t(A, B, ta, tb)
            assert np.array_equal(got, want)
            C = rng.integers(-2, 3, size=(4, m, n)).astype(np.float64)
            assert np.array_equal(oracle.gemm_t(A, B, ta, tb, alpha=2.0, beta=-1.0, C=C), 2 * want - C)


def test_scalar_closed_form():
    rng = np.random.default_rng(1)
    a, b = rng.uniform(0.5, 2, 20), rng.uniform(-1, 1, 20)
    p, r = rng.uniform(0.5, 2, 20), rng.uniform(0.5, 2, 20)
    K, info = oracle.riccati_gain(a.reshape(-1, 1, 1), b.reshape(-1, 1, 1), p.reshape(-1, 1, 1), r.reshape(-1, 1, 1))
    assert (info == 0).all()
    assert np.allclose(K[:, 0, 0], b * p * a / (r + b * b * p), rtol=1e-14, atol=0)


def test_decoupled_diagonal_case():
    rng = np.random.default_rng(2)
    n = 6
    a, b, p, r = (rng.uniform(0.5, 2, n) for _ in range(4))
    K, info = oracle.riccati_gain(np.diag(a)[None], np.diag(b)[None], np.diag(p)[None], np.diag(r)[None])
    assert info[0] == 0
    assert np.allclose(np.diag(K[0]), b * p * a / (r + b * b * p), rtol=1e-14, atol=0)
    assert (K[0][~np.eye(n, dtype=bool)] == 0).all()


def test_exact_rationals_tiny_integer_case():
    A = [[1, 1], [0, 1]]
    B = [[0], [1]]
    P = [[2, 1], [1, 3]]
    R = [[1]]
    F = lambda M: [[Fraction(v) for v in row] for row in M]
    A_, B_, P_, R_ = F(A), F(B), F(P), F(R)
    mul = lambda X, Y: [[sum(X[i][q] * Y[q][j] for q in range(len(Y))) for j in range(len(Y[0]))]
                        for i in range(len(X))]
    T = lambda X: [list(r) for r in zip(*X)]
    S = mul(T(B_), mul(P_, B_))[0][0] + R_[0][0]
    BPA = mul(T(B_), mul(P_, A_))[0]
    want = [float(v / S) for v in BPA]
    K, info = oracle.riccati_gain(np.array([A], float), np.array([B], float), np.array([P], float),
                                  np.array([R], float))
    assert info[0] == 0
    assert np.allclose(K[0, 0], want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("nx,nu", [(2, 1), (4, 2), (12, 4), (14, 7)])
def test_dare_fixed_point(nx, nu):
    """With P the stabilising solution of the discrete algebraic Riccati
    equation (scipy, Schur method), the oracle's K satisfies
    P = Q + A^T P A - A^T P B K."""
    rng = np.random.default_rng(nx * 10 + nu)
    A = np.eye(nx) + 0.1 * rng.uniform(-1, 1, (nx, nx))
    B = rng.uniform(-1, 1, (nx, nu))
    Q = np.eye(nx)
    R = np.eye(nu) + 0.1 * np.diag(rng.uniform(0, 1, nu))
    P = scipy.linalg.solve_discrete_are(A, B, Q, R)
    P = 0.5 * (P + P.T)
    K, info = oracle.riccati_gain(A[None], B[None], P[None], R[None])
    assert info[0] == 0
    resid = Q + A.T @ P @ A - A.T @ P @ B @ K[0] - P
    assert np.max(np.abs(resid)) <= 1e-8 * np.max(np.abs(P))


@pytest.mark.parametrize("nx,nu", [(1, 1), (3, 2), (12, 4), (14, 7), (32, 8), (48, 16)])
def test_stationarity_and_numpy_solve(nx, nu):
    c = inputs.make_riccati(5, nx, nu)
    K, info = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
    assert (info == 0).all()
    A, B, P, R = (c[k].astype(np.float64) for k in "ABPR")
    Bt = np.swapaxes(B, 1, 2)
    S = R + Bt @ P @ B
    T = Bt @ P @ A
    res = S @ K - T
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(T))
    assert np.allclose(K, np.linalg.solve(S, T), rtol=0, atol=1e-12 * np.max(np.abs(K)))


def test_info_for_indefinite_s():
    # R = -I with B = 0: S = -I fails at the first pivot
    nx, nu = 3, 2
    A = np.eye(nx)[None]
    B = np.zeros((1, nx, nu))
    P = np.eye(nx)[None]
    R = -np.eye(nu)[None]
    _, info = oracle.riccati_gain(A, B, P, R)
    assert info[0] == 1
