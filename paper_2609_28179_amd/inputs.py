"""Seeded synthetic inputs shaped like the paper's robotics-scale workloads.

This module only draws random numbers and assembles well-posed problem
instances (SPD matrices, well-conditioned triangles, rigid transforms).  It
holds none of the batched operations themselves and is shared, unchanged, by
the tests, the benchmark and the tuner; nothing here calls the GPU library or
the oracle.

Recipes (the paper states no input distribution, Sec. IV-A only asks for a
fresh valid input per launch of a destructive op):
  general matrices / vectors : iid uniform[-1, 1]
  SPD matrices               : A = M M^T + n I, M iid uniform[-1, 1], formed in
                               float64, lower triangle mirrored into the upper
                               (exact symmetry), rounded to float32
  triangular factors          : the float64 Cholesky factor of such an A
                               (LAPACK, through numpy), rounded to float32; a
                               random uniform triangle would have condition
                               numbers near 1e19 at n = 64
  conditioned SPD (tests)     : 2^s Q diag(lam) Q^T, lam log-spaced over
                               [1, kappa], Q Haar orthogonal (QR of a Gaussian
                               matrix), mirrored, rounded to float32
  SE(3) transforms            : R from a Hamilton unit quaternion (w, x, y, z)
                               q = normalize(N(0, 1)^4) (uniform on S^3),
                               t iid uniform[-1, 1]^3, last row (0, 0, 0, 1)

Seeding: ``numpy.random.default_rng(SeedSequence([cfg, op_id, n, batch]))``
for the host generators; the ``*_torch`` variants draw the same recipes from a
seeded ``torch.Generator`` on the target device (used for the multi-GB
benchmark inputs, which are too large to draw on the host).
"""
from __future__ import annotations

import numpy as np

OP_IDS = {
    "gemm": 0, "gemv": 1, "potrf": 2, "potrs": 3, "posv": 4, "trsv": 5,
    "se3_compose": 6, "se3_inverse": 7, "adjoint": 8, "ragged": 9, "riccati": 10,
}


def rng_for(cfg: int, op: str, n: int, batch: int, extra: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([cfg, OP_IDS[op], n, batch, extra]))


def uniform(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=shape).astype(np.float32)


def spd64(rng: np.random.Generator, batch: int, n: int) -> np.ndarray:
    """float64 A = M M^T + n I (exactly symmetric), before rounding."""
    M = rng.uniform(-1.0, 1.0, size=(batch, n, n))
    A = np.matmul(M, np.swapaxes(M, 1, 2))
    A += n * np.eye(n)[None]
    il = np.tril_indices(n, -1)
    A[:, il[1], il[0]] = A[:, il[0], il[1]]
    return A


def spd(rng: np.random.Generator, batch: int, n: int) -> np.ndarray:
    return spd64(rng, batch, n).astype(np.float32)


def lower_factor(rng: np.random.Generator, batch: int, n: int) -> np.ndarray:
    """Well-conditioned lower triangle with zero strict upper part (float32)."""
    A = spd64(rng, batch, n)
    L = np.linalg.cholesky(A)
    return np.tril(L).astype(np.float32)


def spd_conditioned64(rng: np.random.Generator, batch: int, n: int, kappa: float, scale_exp: int = 0) -> np.ndarray:
    """float64 SPD A = 2^scale_exp Q diag(lam) Q^T with lam log-spaced over
    [1, kappa] (condition number kappa) and Q the orthogonal factor of a
    Gaussian matrix (column signs fixed by R's diagonal, so Q is Haar
    distributed); lower triangle mirrored (exact symmetry)."""
    G = rng.standard_normal(size=(batch, n, n))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    lam = np.logspace(0.0, np.log10(kappa), n) if n > 1 else np.ones(1)
    A = np.matmul(Q * lam[None, None, :], np.swapaxes(Q, 1, 2))
    il = np.tril_indices(n, -1)
    A[:, il[1], il[0]] = A[:, il[0], il[1]]
    return A * (2.0 ** scale_exp)


def spd_conditioned(rng: np.random.Generator, batch: int, n: int, kappa: float, scale_exp: int = 0) -> np.ndarray:
    return spd_conditioned64(rng, batch, n, kappa, scale_exp).astype(np.float32)


def lower_factor_conditioned(rng: np.random.Generator, batch: int, n: int, kappa: float,
                             scale_exp: int = 0) -> np.ndarray:
    """The float64 Cholesky factor of ``spd_conditioned64`` (condition number
    sqrt(kappa)), rounded to float32."""
    L = np.linalg.cholesky(spd_conditioned64(rng, batch, n, kappa, scale_exp))
    return np.tril(L).astype(np.float32)


def rotations64(rng: np.random.Generator, batch: int) -> np.ndarray:
    q = rng.standard_normal(size=(batch, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((batch, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def se3(rng: np.random.Generator, batch: int) -> np.ndarray:
    T = np.zeros((batch, 4, 4))
    T[:, :3, :3] = rotations64(rng, batch)
    T[:, :3, 3] = rng.uniform(-1.0, 1.0, size=(batch, 3))
    T[:, 3, 3] = 1.0
    return T.astype(np.float32)


# ---------------------------------------------------------------- problem sets
def make_case(op: str, n: int, batch: int, cfg: int = 1, nrhs: int = 1, extra: int = 0,
              kappa: float | None = None, scale_exp: int = 0) -> dict:
    """Inputs of one (op, n, batch) cell as float32 numpy arrays.  With
    ``kappa`` the SPD matrices (and the factors derived from them) come from
    ``spd_conditioned`` with that condition number and scale 2^scale_exp."""
    rng = rng_for(cfg, op, n, batch, extra)
    if kappa is not None:
        if op in ("potrf", "posv"):
            out = {"A": spd_conditioned(rng, batch, n, kappa, scale_exp)}
            if op == "posv":
                out["B"] = uniform(rng, (batch, n, nrhs))
            return out
        if op in ("potrs", "trsv"):
            L = lower_factor_conditioned(rng, batch, n, kappa, scale_exp)
            if op == "potrs":
                return {"L": L, "B": uniform(rng, (batch, n, nrhs))}
            return {"L": L, "x": uniform(rng, (batch, n))}
        raise ValueError(f"no conditioned recipe for {op}")
    if op == "gemm":
        return {"A": uniform(rng, (batch, n, n)), "B": uniform(rng, (batch, n, n))}
    if op == "gemv":
        return {"A": uniform(rng, (batch, n, n)), "x": uniform(rng, (batch, n))}
    if op == "potrf":
        return {"A": spd(rng, batch, n)}
    if op == "posv":
        A = spd(rng, batch, n)
        return {"A": A, "B": uniform(rng, (batch, n, nrhs))}
    if op == "potrs":
        L = lower_factor(rng, batch, n)
        return {"L": L, "B": uniform(rng, (batch, n, nrhs))}
    if op == "trsv":
        L = lower_factor(rng, batch, n)
        return {"L": L, "x": uniform(rng, (batch, n))}
    if op == "se3_compose":
        return {"Ta": se3(rng, batch), "Tb": se3(rng, batch)}
    if op == "se3_inverse":
        return {"Ta": se3(rng, batch)}
    raise ValueError(op)


# ------------------------------------------------------- device-side variants
def _torch():
    import torch
    return torch


def torch_generator(device, seed: int):
    torch = _torch()
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def uniform_torch(g, shape, device):
    torch = _torch()
    return torch.rand(shape, generator=g, device=device, dtype=torch.float32) * 2.0 - 1.0


def spd_torch(g, batch: int, n: int, device, chunk: int = 16384):
    """Same recipe as ``spd`` drawn on ``device``: float64 M M^T + n I, mirrored, float32."""
    torch = _torch()
    out = torch.empty((batch, n, n), dtype=torch.float32, device=device)
    eye = torch.eye(n, dtype=torch.float64, device=device)
    for s in range(0, batch, chunk):
        e = min(batch, s + chunk)
        M = torch.rand((e - s, n, n), generator=g, device=device, dtype=torch.float64) * 2.0 - 1.0
        A = torch.matmul(M, M.transpose(1, 2).contiguous()) + n * eye
        A = torch.tril(A) + torch.tril(A, -1).transpose(1, 2)
        out[s:e] = A.to(torch.float32)
    return out


def lower_factor_torch(g, batch: int, n: int, device, chunk: int = 16384):
    torch = _torch()
    out = torch.empty((batch, n, n), dtype=torch.float32, device=device)
    eye = torch.eye(n, dtype=torch.float64, device=device)
    for s in range(0, batch, chunk):
        e = min(batch, s + chunk)
        M = torch.rand((e - s, n, n), generator=g, device=device, dtype=torch.float64) * 2.0 - 1.0
        A = torch.matmul(M, M.transpose(1, 2).contiguous()) + n * eye
        A = torch.tril(A) + torch.tril(A, -1).transpose(1, 2)
        out[s:e] = torch.tril(torch.linalg.cholesky(A)).to(torch.float32)
    return out


def se3_torch(g, batch: int, device):
    torch = _torch()
    q = torch.randn((batch, 4), generator=g, device=device, dtype=torch.float64)
    q = q / q.norm(dim=1, keepdim=True)
    w, x, y, z = q.unbind(1)
    T = torch.zeros((batch, 4, 4), dtype=torch.float64, device=device)
    T[:, 0, 0] = 1 - 2 * (y * y + z * z)
    T[:, 0, 1] = 2 * (x * y - w * z)
    T[:, 0, 2] = 2 * (x * z + w * y)
    T[:, 1, 0] = 2 * (x * y + w * z)
    T[:, 1, 1] = 1 - 2 * (x * x + z * z)
    T[:, 1, 2] = 2 * (y * z - w * x)
    T[:, 2, 0] = 2 * (x * z - w * y)
    T[:, 2, 1] = 2 * (y * z + w * x)
    T[:, 2, 2] = 1 - 2 * (x * x + y * y)
    T[:, :3, 3] = torch.rand((batch, 3), generator=g, device=device, dtype=torch.float64) * 2.0 - 1.0
    T[:, 3, 3] = 1.0
    return T.to(torch.float32)


# ------------------------------------------------------------------ LQR gain
def riccati64(rng: np.random.Generator, batch: int, nx: int, nu: int):
    """Float64 inputs of K = (R + B^T P B)^{-1} B^T P A, before rounding:
    A = I + 0.1 U[-1,1] (a discretised dynamics matrix), B = 0.5 U[-1,1],
    P = M M^T / nx + I and R = N N^T / nu + I (symmetric positive definite,
    lower triangle mirrored), M, N iid uniform[-1, 1]."""
    A = np.eye(nx)[None] + 0.1 * rng.uniform(-1.0, 1.0, size=(batch, nx, nx))
    B = 0.5 * rng.uniform(-1.0, 1.0, size=(batch, nx, nu))
    M = rng.uniform(-1.0, 1.0, size=(batch, nx, nx))
    P = np.matmul(M, np.swapaxes(M, 1, 2)) / nx + np.eye(nx)[None]
    N = rng.uniform(-1.0, 1.0, size=(batch, nu, nu))
    R = np.matmul(N, np.swapaxes(N, 1, 2)) / nu + np.eye(nu)[None]
    for S in (P, R):
        il = np.tril_indices(S.shape[1], -1)
        S[:, il[1], il[0]] = S[:, il[0], il[1]]
    return A, B, P, R


def make_riccati(batch: int, nx: int, nu: int, seed: int = 4) -> dict:
    rng = np.random.default_rng(np.random.SeedSequence([seed, OP_IDS["riccati"], nx, nu, batch]))
    A, B, P, R = riccati64(rng, batch, nx, nu)
    return {"A": A.astype(np.float32), "B": B.astype(np.float32), "P": P.astype(np.float32),
            "R": R.astype(np.float32)}


def riccati_torch(g, batch: int, nx: int, nu: int, device):
    """The same recipe drawn on the device (float64, rounded to float32)."""
    torch = _torch()
    f64 = torch.float64
    u = lambda shape: torch.rand(shape, generator=g, device=device, dtype=f64) * 2.0 - 1.0
    A = torch.eye(nx, dtype=f64, device=device) + 0.1 * u((batch, nx, nx))
    B = 0.5 * u((batch, nx, nu))
    M = u((batch, nx, nx))
    P = torch.matmul(M, M.transpose(1, 2).contiguous()) / nx + torch.eye(nx, dtype=f64, device=device)
    N = u((batch, nu, nu))
    R = torch.matmul(N, N.transpose(1, 2).contiguous()) / nu + torch.eye(nu, dtype=f64, device=device)
    P = torch.tril(P) + torch.tril(P, -1).transpose(1, 2)
    R = torch.tril(R) + torch.tril(R, -1).transpose(1, 2)
    return {k: v.to(torch.float32).contiguous() for k, v in (("A", A), ("B", B), ("P", P), ("R", R))}


# ----------------------------------------------------- cost-model initial weights
def mlp_init(d: int, seed: int, hidden: int = 64) -> np.ndarray:
    """He-normal initial weights of the d -> 64 -> 64 -> 1 cost model (std
    sqrt(2 / fan_in), zero biases) as one flat float64 vector in the order
    W1 [64][d], b1, W2 [64][64], b2, w3, b3."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, d, hidden]))
    W1 = rng.standard_normal((hidden, d)) * np.sqrt(2.0 / d)
    W2 = rng.standard_normal((hidden, hidden)) * np.sqrt(2.0 / hidden)
    w3 = rng.standard_normal(hidden) * np.sqrt(2.0 / hidden)
    return np.concatenate([W1.ravel(), np.zeros(hidden), W2.ravel(), np.zeros(hidden), w3, [0.0]])


# ------------------------------------------------------------ ragged batches
RAGGED_SIZES = (6, 7, 12, 14, 18, 24, 36, 48, 64)


def make_ragged(count: int, seed: int = 2, sizes=RAGGED_SIZES, max_rhs: int = 8) -> dict:
    """A ragged batch: n uniform over `sizes`, nrhs uniform over 1..max_rhs,
    A = M M^T + n I per problem (as ``spd``), B iid uniform[-1, 1]; packed
    row-major with int64 element offsets (exclusive prefix sums)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, OP_IDS["ragged"], count]))
    n = rng.choice(np.asarray(sizes, dtype=np.int32), size=count).astype(np.int32)
    nrhs = rng.integers(1, max_rhs + 1, size=count).astype(np.int32)
    sa = n.astype(np.int64) ** 2
    sb = n.astype(np.int64) * nrhs
    offA = np.concatenate([[0], np.cumsum(sa)[:-1]]).astype(np.int64)
    offB = np.concatenate([[0], np.cumsum(sb)[:-1]]).astype(np.int64)
    A = np.empty(int(sa.sum()), dtype=np.float32)
    B = rng.uniform(-1.0, 1.0, size=int(sb.sum())).astype(np.float32)
    for size in np.unique(n):
        idx = np.nonzero(n == size)[0]
        blocks = spd(rng, len(idx), int(size)).reshape(len(idx), -1)
        for row, i in enumerate(idx):
            A[offA[i]:offA[i] + sa[i]] = blocks[row]
    return {"n": n, "nrhs": nrhs, "offA": offA, "offB": offB, "A": A, "B": B}
