"""Pins of the FP64 oracle against facts fixed by mathematics, not by itself.

Every check here is independent of the oracle's code: exact integer or
rational brute force, closed forms, invariants, or special cases that reduce
to a textbook routine.  They are chosen so that a dropped term, a wrong sign,
a wrong index or a transposed operand in the oracle fails at least one.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2609_28179_amd import inputs

RNG = np.random.default_rng(12345)


# ------------------------------------------------------------------ helpers
def int_mat(shape, lo=-2, hi=2):
    return RNG.integers(lo, hi + 1, size=shape).astype(np.float64)


def brute_matmul(a, b):
    m, k = len(a), len(a[0])
    n = len(b[0])
    return [[sum(Fraction(int(a[i][p])) * Fraction(int(b[p][j])) for p in range(k)) for j in range(n)]
            for i in range(m)]


def frac_det(M):
    """Exact determinant by fraction-valued Gaussian elimination."""
    M = [[Fraction(x) for x in row] for row in M]
    n = len(M)
    det = Fraction(1)
    for c in range(n):
        piv = next((r for r in range(c, n) if M[r][c] != 0), None)
        if piv is None:
            return Fraction(0)
        if piv != c:
            M[c], M[piv] = M[piv], M[c]
            det = -det
        det *= M[c][c]
        for r in range(c + 1, n):
            f = M[r][c] / M[c][c]
            for cc in range(c, n):
                M[r][cc] -= f * M[c][cc]
    return det


def frac_solve(M, b):
    """Cramer's rule in exact fractions."""
    n = len(M)
    D = frac_det(M)
    out = []
    for i in range(n):
        Mi = [row[:] for row in M]
        for r in range(n):
            Mi[r][i] = b[r]
        out.append(frac_det(Mi) / D)
    return out


# --------------------------------------------------------------------- GEMM
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 2), (7, 4, 6), (6, 6, 6), (5, 1, 9)])
def test_gemm_integer_exact(m, n, k):
    b = 3
    A = int_mat((b, m, k))
    B = int_mat((b, k, n))
    C = oracle.gemm(A, B)
    for q in range(b):
        ref = brute_matmul(A[q].tolist(), B[q].tolist())
        assert C[q].tolist() == [[float(x) for x in row] for row in ref]


def test_gemm_alpha_beta_exact_and_beta_zero_ignores_c():
    A = int_mat((2, 4, 3))
    B = int_mat((2, 3, 5))
    C0 = int_mat((2, 4, 5))
    C = oracle.gemm(A, B, C0, alpha=3.0, beta=-2.0)
    for q in range(2):
        ref = brute_matmul(A[q].tolist(), B[q].tolist())
        exp = [[3 * ref[i][j] - 2 * Fraction(int(C0[q, i, j])) for j in range(5)] for i in range(4)]
        assert C[q].tolist() == [[float(x) for x in row] for row in exp]
    Cnan = np.full((2, 4, 5), np.nan)
    out = oracle.gemm(A, B, Cnan, alpha=1.0, beta=0.0)
    assert np.isfinite(out).all()


def test_gemm_identity_and_library_matmul():
    X = RNG.uniform(-1, 1, size=(4, 7, 7))
    I = np.broadcast_to(np.eye(7), X.shape)
    assert np.array_equal(oracle.gemm(I, X), X)
    assert np.array_equal(oracle.gemm(X, I), X)
    A = RNG.uniform(-1, 1, size=(8, 12, 9))
    B = RNG.uniform(-1, 1, size=(8, 9, 11))
    assert np.max(np.abs(oracle.gemm(A, B) - np.matmul(A, B))) <= 1e-13


# --------------------------------------------------------------------- GEMV
@pytest.mark.parametrize("m,n", [(1, 1), (4, 7), (9, 3), (6, 6)])
def test_gemv_integer_exact(m, n):
    A = int_mat((3, m, n))
    x = int_mat((3, n))
    y0 = int_mat((3, m))
    y = oracle.gemv(A, x, y0, alpha=2.0, beta=-1.0)
    for q in range(3):
        exp = [2 * sum(Fraction(int(A[q, i, j])) * int(x[q, j]) for j in range(n)) - int(y0[q, i])
               for i in range(m)]
        assert y[q].tolist() == [float(e) for e in exp]
    ynan = np.full((3, m), np.nan)
    assert np.isfinite(oracle.gemv(A, x, ynan, beta=0.0)).all()


# -------------------------------------------------------------------- POTRF
def test_potrf_diagonal_powers_of_four_exact():
    k = RNG.integers(-6, 7, size=(5, 9))
    A = np.zeros((5, 9, 9))
    for q in range(5):
        A[q] = np.diag(4.0 ** k[q])
    L, info = oracle.potrf(A)
    assert (info == 0).all()
    for q in range(5):
        assert np.array_equal(L[q], np.diag(2.0 ** k[q]))


@pytest.mark.parametrize("n", [1, 2, 5, 16, 64])
def test_potrf_laplacian_closed_form(n):
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    L, info = oracle.potrf(A[None])
    assert info[0] == 0
    kk = np.arange(1, n + 1, dtype=np.float64)
    diag = np.sqrt((kk + 1) / kk)              # L_kk = sqrt((k+1)/k), 1-based
    sub = -np.sqrt(kk[:-1] / (kk[:-1] + 1))    # L_{k+1,k} = -sqrt(k/(k+1))
    exp = np.diag(diag) + np.diag(sub, -1)
    assert np.max(np.abs(L[0] - exp)) <= 1e-14


def test_potrf_small_closed_forms():
    a = 2.25
    L, info = oracle.potrf(np.array([[[a]]]))
    assert info[0] == 0 and L[0, 0, 0] == 1.5
    # n = 2: l11 = sqrt(a), l21 = b / l11, l22 = sqrt(c - l21^2)
    a, b, c = 4.0, 2.0, 5.0
    L, info = oracle.potrf(np.array([[[a, b], [b, c]]]))
    assert info[0] == 0
    assert np.array_equal(L[0], np.array([[2.0, 0.0], [1.0, 2.0]]))


@pytest.mark.parametrize("n", [3, 6, 12, 33, 64])
def test_potrf_reconstruction_and_numpy(n):
    A = inputs.spd64(np.random.default_rng(n), 6, n)
    L, info = oracle.potrf(A)
    assert (info == 0).all()
    R = np.matmul(L, np.swapaxes(L, 1, 2))
    assert np.max(np.abs(R - A)) / np.max(np.abs(A)) <= 1e-12
    assert np.max(np.abs(L - np.linalg.cholesky(A))) <= 1e-12


def test_potrf_strict_upper_is_positive_zero_and_unread():
    A = inputs.spd64(np.random.default_rng(7), 4, 8)
    iu = np.triu_indices(8, 1)
    A_garbage = A.copy()
    A_garbage[:, iu[0], iu[1]] = np.nan
    L1, i1 = oracle.potrf(A)
    L2, i2 = oracle.potrf(A_garbage)
    assert np.array_equal(L1, L2) and np.array_equal(i1, i2)
    up = L1[:, iu[0], iu[1]]
    assert (up == 0).all() and not np.signbit(up).any()


def sylvester_info(M):
    """First k (1-based) whose leading principal minor is <= 0, exactly; 0 if none."""
    n = len(M)
    for k in range(1, n + 1):
        if frac_det([row[:k] for row in M[:k]]) <= 0:
            return k
    return 0


def test_potrf_info_singular_example():
    # l21 = 1 exactly, so the second pivot is 1 - 1 = 0: leading minors 4, 0, -36.
    M = [[4, 2, 0], [2, 1, 3], [0, 3, 5]]
    assert [frac_det([r[:k] for r in M[:k]]) for k in (1, 2, 3)] == [4, 0, -36]
    _, info = oracle.potrf(np.array([M], dtype=np.float64))
    assert info[0] == sylvester_info(M) == 2


def test_potrf_info_brute_force_sylvester():
    rng = np.random.default_rng(99)
    cases = []
    for _ in range(200):
        n = int(rng.integers(1, 5))
        X = rng.integers(-3, 4, size=(n, n))
        M = (X + X.T).tolist()
        cases.append(M)
    for M in cases:
        _, info = oracle.potrf(np.array([M], dtype=np.float64))
        exp = sylvester_info(M)
        # Exactly singular leading minors are decided identically only when the
        # floating-point pivot is exactly zero too; integer inputs of this size
        # keep every pivot exactly representable or clearly signed.
        assert info[0] == exp, (M, info[0], exp)


def test_potrf_info_negative_diagonal():
    for k in range(1, 7):
        d = np.ones(6)
        d[k - 1] = -1.0
        _, info = oracle.potrf(np.diag(d)[None])
        assert info[0] == k
    _, info = oracle.potrf(np.array([[[np.nan]]]))
    assert info[0] == 1


# ------------------------------------------------------------- POTRS / POSV
@pytest.mark.parametrize("n", [1, 3, 8, 31, 64])
def test_posv_laplacian_inverse_closed_form(n):
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    L, X, info = oracle.posv(A[None], np.eye(n)[None])
    assert info[0] == 0
    i = np.arange(1, n + 1)[:, None]
    j = np.arange(1, n + 1)[None, :]
    exp = np.minimum(i, j) * (n + 1 - np.maximum(i, j)) / (n + 1)
    assert np.max(np.abs(X[0] - exp)) <= 1e-12 * n


def test_posv_cramer_exact_small():
    rng = np.random.default_rng(5)
    for _ in range(60):
        n = int(rng.integers(1, 5))
        Mx = rng.integers(-2, 3, size=(n, n))
        A = (Mx @ Mx.T + n * np.eye(n, dtype=np.int64)).tolist()
        b = rng.integers(-4, 5, size=n).tolist()
        exp = frac_solve(A, b)
        _, X, info = oracle.posv(np.array([A], float), np.array([b], float)[:, :, None])
        assert info[0] == 0
        assert np.max(np.abs(X[0, :, 0] - np.array([float(e) for e in exp]))) <= 1e-13


def test_posv_diagonal_powers_bit_exact():
    k = RNG.integers(-5, 6, size=(3, 10))
    A = np.stack([np.diag(4.0 ** k[q]) for q in range(3)])
    e = RNG.integers(-5, 6, size=(3, 10, 2))
    B = 2.0 ** e
    L, X, info = oracle.posv(A, B)
    assert (info == 0).all()
    assert np.array_equal(X, B / (4.0 ** k)[:, :, None])


@pytest.mark.parametrize("n,r", [(6, 1), (12, 3), (64, 8)])
def test_potrs_residual_and_scipy(n, r):
    import scipy.linalg as sla
    rng = np.random.default_rng(n * 10 + r)
    A = inputs.spd64(rng, 5, n)
    B = rng.uniform(-1, 1, size=(5, n, r))
    L, info = oracle.potrf(A)
    X = oracle.potrs(L, B)
    for q in range(5):
        res = np.max(np.abs(A[q] @ X[q] - B[q]))
        assert res / (np.max(np.abs(A[q]).sum(1)) * np.max(np.abs(X[q]))) <= 1e-14
        ref = sla.cho_solve((L[q], True), B[q])
        assert np.max(np.abs(X[q] - ref)) <= 1e-12
    _, X2, info2 = oracle.posv(A, B)
    assert (info2 == 0).all() and np.array_equal(X, X2)


def test_potrs_reads_only_lower():
    rng = np.random.default_rng(3)
    L = np.tril(inputs.lower_factor(rng, 3, 7).astype(np.float64))
    G = L.copy()
    iu = np.triu_indices(7, 1)
    G[:, iu[0], iu[1]] = np.nan
    B = rng.uniform(-1, 1, size=(3, 7, 2))
    assert np.array_equal(oracle.potrs(L, B), oracle.potrs(G, B))


# --------------------------------------------------------------------- TRSV
def test_trsv_identity_and_power_of_two_diagonal_exact():
    x = RNG.uniform(-1, 1, size=(4, 9))
    I = np.broadcast_to(np.eye(9), (4, 9, 9))
    assert np.array_equal(oracle.trsv(I, x, 0), x)
    assert np.array_equal(oracle.trsv(I, x, 1), x)
    e = RNG.integers(-4, 5, size=(4, 9))
    D = np.stack([np.diag(2.0 ** e[q]) for q in range(4)])
    assert np.array_equal(oracle.trsv(D, x, 0), x / 2.0 ** e)


@pytest.mark.parametrize("n", [2, 7, 64])
def test_trsv_unit_bidiagonal_integer_recurrence(n):
    rng = np.random.default_rng(n)
    s = rng.choice([-1.0, 1.0], size=(3, n - 1))
    L = np.stack([np.eye(n) + np.diag(s[q], -1) for q in range(3)])
    b = rng.integers(-3, 4, size=(3, n)).astype(np.float64)
    # forward: x_i = b_i - l_i x_{i-1}; backward with L^T: x_i = b_i - l_{i+1} x_{i+1}
    fw = np.zeros_like(b)
    bw = np.zeros_like(b)
    for q in range(3):
        acc = 0
        for i in range(n):
            acc = int(b[q, i]) - (int(s[q, i - 1]) * acc if i > 0 else 0)
            fw[q, i] = acc
        acc = 0
        for i in range(n - 1, -1, -1):
            acc = int(b[q, i]) - (int(s[q, i]) * acc if i < n - 1 else 0)
            bw[q, i] = acc
    assert np.array_equal(oracle.trsv(L, b, 0), fw)
    assert np.array_equal(oracle.trsv(L, b, 1), bw)


@pytest.mark.parametrize("n", [3, 16, 64])
def test_trsv_scipy_and_exact_small(n):
    import scipy.linalg as sla
    rng = np.random.default_rng(100 + n)
    L = inputs.lower_factor(rng, 4, n).astype(np.float64)
    b = rng.uniform(-1, 1, size=(4, n))
    x0 = oracle.trsv(L, b, 0)
    x1 = oracle.trsv(L, b, 1)
    for q in range(4):
        assert np.max(np.abs(x0[q] - sla.solve_triangular(L[q], b[q], lower=True))) <= 1e-12
        assert np.max(np.abs(x1[q] - sla.solve_triangular(L[q].T, b[q], lower=False))) <= 1e-12
    # exact rational check of the transposed solve on a small integer triangle
    Li = np.tril(rng.integers(-3, 4, size=(4, 4))).astype(np.float64)
    np.fill_diagonal(Li, [1, 2, 4, -1])
    bi = rng.integers(-5, 6, size=4).astype(np.float64)
    exp = frac_solve(Li.T.tolist(), bi.tolist())
    assert np.max(np.abs(oracle.trsv(Li[None], bi[None], 1)[0] - [float(v) for v in exp])) <= 1e-15


# -------------------------------------------------------------------- SE(3)
def test_se3_generator_rotations_orthonormal():
    R = inputs.rotations64(np.random.default_rng(1), 500)
    RtR = np.matmul(np.swapaxes(R, 1, 2), R)
    assert np.max(np.abs(RtR - np.eye(3))) <= 1e-15 * 10
    assert np.max(np.abs(np.linalg.det(R) - 1)) <= 1e-14


def test_se3_identities():
    rng = np.random.default_rng(2)
    Ta = inputs.se3(rng, 64).astype(np.float64)
    Tb = inputs.se3(rng, 64).astype(np.float64)
    I = np.broadcast_to(np.eye(4), Ta.shape)
    assert np.array_equal(oracle.se3_compose(I, Ta), Ta)
    assert np.array_equal(oracle.se3_compose(Ta, I), Ta)
    Ti = oracle.se3_inverse(Ta)
    # float32-rounded rotations are orthonormal to ~1e-7, so T T^-1 = I to that level
    assert np.max(np.abs(oracle.se3_compose(Ta, Ti) - np.eye(4))) <= 1e-6
    assert np.max(np.abs(oracle.se3_inverse(Ti) - Ta)) <= 1e-6
    # (Ta Tb)^-1 = Tb^-1 Ta^-1 holds for the closed form when R is exactly
    # orthonormal, so use float64 rotations here
    Ua = np.zeros((32, 4, 4)); Ub = np.zeros((32, 4, 4))
    for U in (Ua, Ub):
        U[:, :3, :3] = inputs.rotations64(rng, 32)
        U[:, :3, 3] = rng.uniform(-1, 1, size=(32, 3))
        U[:, 3, 3] = 1
    lhs = oracle.se3_inverse(oracle.se3_compose(Ua, Ub))
    rhs = oracle.se3_compose(oracle.se3_inverse(Ub), oracle.se3_inverse(Ua))
    assert np.max(np.abs(lhs - rhs)) <= 1e-14
    # compose equals the plain 4x4 matrix product when row 3 is (0 0 0 1)
    assert np.max(np.abs(oracle.se3_compose(Ta, Tb) - np.matmul(Ta, Tb))) <= 1e-15
    # inverse equals the general 4x4 inverse for an exactly orthonormal R
    R = inputs.rotations64(rng, 16)
    T = np.zeros((16, 4, 4))
    T[:, :3, :3] = R
    T[:, :3, 3] = rng.uniform(-1, 1, size=(16, 3))
    T[:, 3, 3] = 1
    assert np.max(np.abs(oracle.se3_inverse(T) - np.linalg.inv(T))) <= 1e-13


def test_se3_exact_special_cases_and_row3():
    rng = np.random.default_rng(4)
    # pure integer translations compose exactly: t = ta + tb
    ta = rng.integers(-9, 10, size=(8, 3)).astype(float)
    tb = rng.integers(-9, 10, size=(8, 3)).astype(float)
    Ta = np.broadcast_to(np.eye(4), (8, 4, 4)).copy()
    Tb = Ta.copy()
    Ta[:, :3, 3] = ta
    Tb[:, :3, 3] = tb
    out = oracle.se3_compose(Ta, Tb)
    assert np.array_equal(out[:, :3, 3], ta + tb)
    inv = oracle.se3_inverse(Ta)
    assert np.array_equal(inv[:, :3, 3], -ta)
    # 90-degree rotations about z then x, exact {0, +-1} entries
    Rz = np.array([[0, -1, 0], [1, 0, 0], [0, 0, 1]], float)
    Rx = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], float)
    A = np.eye(4); A[:3, :3] = Rz; A[:3, 3] = [1, 2, 3]
    B = np.eye(4); B[:3, :3] = Rx; B[:3, 3] = [-1, 0, 2]
    out = oracle.se3_compose(A[None], B[None])[0]
    assert np.array_equal(out[:3, :3], Rz @ Rx)
    assert np.array_equal(out[:3, 3], Rz @ np.array([-1, 0, 2.0]) + np.array([1, 2, 3.0]))
    # row 3 of the inputs is not read and row 3 of the output is exactly 0 0 0 1
    Ag = A.copy(); Ag[3] = np.nan
    Bg = B.copy(); Bg[3] = [5, 6, 7, 8]
    out2 = oracle.se3_compose(Ag[None], Bg[None])[0]
    assert np.array_equal(out2, out)
    assert np.array_equal(out2[3], [0, 0, 0, 1])
    assert np.array_equal(oracle.se3_inverse(Ag[None])[0], oracle.se3_inverse(A[None])[0])
