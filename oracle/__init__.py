"""FP64 CPU oracle for the batched small dense linear algebra path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU
baseline leg of the benchmark are the only callers.  The product library never
imports, links or calls anything in this directory, and this directory uses
nothing from the product library.

Each function takes numpy arrays (any float dtype; promoted exactly to float64)
in the row-major batch-contiguous layout X[batch][rows][cols] and returns new
float64 arrays; inputs are never modified.  The arithmetic lives in
``glass_oracle.c`` (plain loops, FP64, no BLAS/LAPACK) and is reached through
ctypes.  What each function computes is stated beside it in the C source,
with the paper section it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glass_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile glass_oracle.c into liboracle.so with gcc; returns the path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        d = ctypes.c_double
        i = ctypes.c_int
        p = ctypes.c_void_p
        sig = {
            "oracle_gemm": [i, i, i, i, d, p, p, d, p],
            "oracle_gemv": [i, i, i, d, p, p, d, p],
            "oracle_potrf": [i, i, p, p],
            "oracle_potrs": [i, i, i, p, p],
            "oracle_posv": [i, i, i, p, p, p],
            "oracle_trsv": [i, i, i, p, p],
            "oracle_se3_compose": [i, p, p, p],
            "oracle_se3_inverse": [i, p, p],
            "oracle_posv_adjoint": [i, i, i, p, p, p, p, p],
            "oracle_gemm_t": [i, i, i, i, i, i, d, p, p, d, p],
            "oracle_riccati_gain": [i, i, i, p, p, p, p, p, p],
            "oracle_num_threads": [],
            "oracle_set_num_threads": [i],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int if name == "oracle_num_threads" else None
        _lib = lib
    return _lib


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_num_threads(t: int) -> None:
    _load().oracle_set_num_threads(int(t))


def gemm(A, B, C=None, alpha: float = 1.0, beta: float = 0.0) -> np.ndarray:
    """C = alpha A B + beta C for A [b,m,k], B [b,k,n] (C [b,m,n] read iff beta != 0)."""
    A = _f64(A)
    B = _f64(B)
    b, m, k = A.shape
    n = B.shape[2]
    assert B.shape == (b, k, n)
    out = np.zeros((b, m, n)) if C is None else _f64(C).copy()
    _load().oracle_gemm(m, n, k, b, float(alpha), _ptr(A), _ptr(B), float(beta), _ptr(out))
    return out


def gemv(A, x, y=None, alpha: float = 1.0, beta: float = 0.0) -> np.ndarray:
    """y = alpha A x + beta y for A [b,m,n], x [b,n] (y [b,m] read iff beta != 0)."""
    A = _f64(A)
    x = _f64(x)
    b, m, n = A.shape
    out = np.zeros((b, m)) if y is None else _f64(y).reshape(b, m).copy()
    _load().oracle_gemv(m, n, b, float(alpha), _ptr(A), _ptr(x.reshape(b, n)), float(beta), _ptr(out))
    return out


def potrf(A):
    """Lower Cholesky of SPD A [b,n,n]; returns (L with +0 strict upper, info int32 [b])."""
    L = _f64(A).copy()
    b, n, _ = L.shape
    info = np.zeros(b, dtype=np.int32)
    _load().oracle_potrf(n, b, _ptr(L), _ptr(info))
    return L, info


def potrs(L, B):
    """X = (L L^T)^{-1} B for L [b,n,n] (lower read), B [b,n,r]."""
    L = _f64(L)
    X = _f64(B).copy()
    b, n, r = X.shape
    _load().oracle_potrs(n, r, b, _ptr(L), _ptr(X))
    return X


def posv(A, B):
    """Factor-and-solve; returns (L, X, info).  X unspecified where info != 0."""
    L = _f64(A).copy()
    X = _f64(B).copy()
    b, n, r = X.shape
    info = np.zeros(b, dtype=np.int32)
    _load().oracle_posv(n, r, b, _ptr(L), _ptr(X), _ptr(info))
    return L, X, info


def trsv(L, x, trans: int = 0):
    """Solve L x = b (trans=0) or L^T x = b (trans=1); L [b,n,n] lower, x [b,n]."""
    L = _f64(L)
    b, n, _ = L.shape
    X = _f64(x).reshape(b, n).copy()
    _load().oracle_trsv(n, b, int(trans), _ptr(L), _ptr(X))
    return X


def se3_compose(Ta, Tb):
    """T = Ta Tb for homogeneous transforms [b,4,4] (row 3 written as 0 0 0 1)."""
    Ta = _f64(Ta)
    Tb = _f64(Tb)
    b = Ta.shape[0]
    out = np.empty((b, 4, 4))
    _load().oracle_se3_compose(b, _ptr(Ta), _ptr(Tb), _ptr(out))
    return out


def se3_inverse(Ta):
    """Closed-form rigid-motion inverse [R^T, -R^T t; 0 0 0 1] of Ta [b,4,4]."""
    Ta = _f64(Ta)
    b = Ta.shape[0]
    out = np.empty((b, 4, 4))
    _load().oracle_se3_inverse(b, _ptr(Ta), _ptr(out))
    return out


def posv_adjoint(L, X, G):
    """(dB, dA) of the Cholesky solve X = A^{-1} B for upstream gradient G:
    dB = A^{-1} G with A = L L^T, dA = -(dB X^T + X dB^T) / 2."""
    L = _f64(L)
    X = _f64(X)
    G = _f64(G)
    b, n, r = X.shape
    dB = np.empty((b, n, r))
    dA = np.empty((b, n, n))
    _load().oracle_posv_adjoint(n, r, b, _ptr(L), _ptr(X), _ptr(G), _ptr(dB), _ptr(dA))
    return dB, dA


def gemm_t(A, B, transa=0, transb=0, alpha=1.0, beta=0.0, C=None):
    """alpha op(A) op(B) + beta C with op = transpose where the flag is set."""
    A = _f64(A)
    B = _f64(B)
    b = A.shape[0]
    m = A.shape[2] if transa else A.shape[1]
    k = A.shape[1] if transa else A.shape[2]
    n = B.shape[1] if transb else B.shape[2]
    out = np.zeros((b, m, n)) if C is None else _f64(C).copy()
    _load().oracle_gemm_t(int(transa), int(transb), m, n, k, b, float(alpha), _ptr(A), _ptr(B), float(beta),
                          _ptr(out))
    return out


def riccati_gain(A, B, P, R):
    """K = (R + B^T P B)^{-1} B^T P A per problem; returns (K, info)."""
    A, B, P, R = _f64(A), _f64(B), _f64(P), _f64(R)
    b, nx, nu = B.shape
    K = np.zeros((b, nu, nx))
    info = np.zeros(b, dtype=np.int32)
    _load().oracle_riccati_gain(nx, nu, b, _ptr(A), _ptr(B), _ptr(P), _ptr(R), _ptr(K), _ptr(info))
    return K, info


def posv_ragged(n, nrhs, offA, offB, A, B):
    """Per-problem factor-and-solve of a packed ragged batch (a loop over the
    problems, grouped by (n, nrhs) only to call the batched routine).
    Returns (A_out, B_out, info) with A_out / B_out packed like the inputs."""
    n = np.asarray(n)
    nrhs = np.asarray(nrhs)
    A_out = _f64(A).copy()
    B_out = _f64(B).copy()
    info = np.zeros(len(n), dtype=np.int32)
    for key in set(zip(n.tolist(), nrhs.tolist())):
        idx = np.nonzero((n == key[0]) & (nrhs == key[1]))[0]
        sa, sb = key[0] * key[0], key[0] * key[1]
        Ab = np.stack([A_out[offA[i]:offA[i] + sa] for i in idx]).reshape(len(idx), key[0], key[0])
        Bb = np.stack([B_out[offB[i]:offB[i] + sb] for i in idx]).reshape(len(idx), key[0], key[1])
        L, X, inf = posv(Ab, Bb)
        for row, i in enumerate(idx):
            A_out[offA[i]:offA[i] + sa] = L[row].reshape(-1)
            B_out[offB[i]:offB[i] + sb] = X[row].reshape(-1)
            info[i] = inf[row]
    return A_out, B_out, info


def ragged_order(n):
    """The problem order of a stable counting sort by size class
    ceil(n / 8) - 1, largest class first (ties keep index order)."""
    n = np.asarray(n, dtype=np.int64)
    cls = np.clip((n - 1) // 8, 0, 7)
    return np.argsort(-cls, kind="stable").astype(np.int32)
