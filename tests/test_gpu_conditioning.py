"""GPU parity on ill-conditioned and scaled SPD problems (Sec. III-C: the
tests cover numerical scale and conditioning, and factorization residuals
are one of its checks).

Inputs: A = 2^s Q diag(lam) Q^T with lam log-spaced over [1, kappa],
kappa in {1e2, 1e3, 1e4}, s in {-40, 0, 40}; POTRS / TRSV take the FP64
Cholesky factor of such an A, rounded to FP32.  Orders 8..64 reach the
thread, sub-wave and row-per-lane wave kernels and, from order 25, the
blocked wave kernel with its explicit 16 x 16 diagonal-block inverses.

Bars (u = 2^-24):
  forward error against the FP64 oracle, per problem and normwise:
    L <= 1e-4 at every kappa; x <= 1e-4 where the operator's condition
    number k_op <= 1e2, else <= k_op * n * u (k_op = kappa for POSV/POTRS,
    sqrt(kappa) for TRSV, whose operand is L);
  residuals in FP64 from the FP32 outputs, independent of kappa:
    rho_f = max|L L^T - A| / (max|A| n u) <= 2,
    rho_s = ||b - A x||_inf / (||A||_inf ||x||_inf n u) <= 2
    (A = L L^T for POTRS, op(L) for TRSV);
  info = 0 and the +0 strict upper triangle bit-exact.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from helpers import TOL, guarded, guards_intact, normwise
from paper_2609_28179_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -24
RHO_MAX = 2.0
NS = (8, 16, 24, 32, 48, 64)
KAPPAS = (1e2, 1e3, 1e4)
SCALES = (-40, 0, 40)
BATCH = 67


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2609_28179_amd import glass
    assert torch.cuda.is_available()
    return glass, torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rho_f(L, A):
    L = L.astype(np.float64)
    A = A.astype(np.float64)
    n = A.shape[1]
    R = np.matmul(L, np.swapaxes(L, 1, 2)) - A
    return np.abs(R).max(axis=(1, 2)) / (np.abs(A).max(axis=(1, 2)) * n * U)


def _rho_s(M, X, B):
    """||B - M X||_inf / (||M||_inf ||X||_inf n u) per problem (max over columns)."""
    M = M.astype(np.float64)
    X = X.astype(np.float64)
    B = B.astype(np.float64)
    n = M.shape[1]
    R = B - np.matmul(M, X)
    nm = np.abs(M).sum(axis=2).max(axis=1)
    return np.abs(R).max(axis=(1, 2)) / (nm * np.abs(X).max(axis=(1, 2)) * n * U)


def _x_bar(k_op, n):
    return TOL if k_op <= 1e2 else k_op * n * U


def _upper_pos_zero(L):
    n = L.shape[1]
    iu = np.triu_indices(n, 1)
    up = L[:, iu[0], iu[1]]
    return bool((up == 0).all() and not np.signbit(up).any())


def _run(glass, torch, op, n, kappa, s, scope, nrhs=1):
    case = inputs.make_case(op, n, BATCH, cfg=300, nrhs=nrhs, extra=int(np.log10(kappa)) * 100 + s + 50,
                            kappa=kappa, scale_exp=s)
    dev = "cuda:0"
    force = (scope, 1)
    bufs = []

    def g(name):
        full, view = guarded(torch, case[name], dev)
        bufs.append(full)
        return view

    fails = []
    label = f"{op} n={n} kappa={kappa:.0e} s={s} nrhs={nrhs} {scope}"
    if op in ("potrf", "posv"):
        A = g("A")
        info = torch.full((BATCH,), -7, dtype=torch.int32, device=dev)
        if op == "potrf":
            st = glass.glass_potrf_batched(n, BATCH, A, info, force)
        else:
            B = g("B")
            st = glass.glass_posv_batched(n, nrhs, BATCH, A, B, info, force)
        torch.cuda.synchronize()
        if st != 0:
            return [f"{label}: status {st}"], {}
        Lg = A.cpu().numpy()
        if op == "potrf":
            L_ref, info_ref = oracle.potrf(case["A"])
        else:
            L_ref, X_ref, info_ref = oracle.posv(case["A"], case["B"])
        stats = {"L_fwd": normwise(np.tril(Lg), L_ref).max(), "rho_f": _rho_f(np.tril(Lg), case["A"]).max()}
        if op == "posv":
            Xg = B.cpu().numpy()
            stats["x_fwd"] = normwise(Xg, X_ref).max()
            stats["rho_s"] = _rho_s(case["A"], Xg, case["B"]).max()
            if not stats["x_fwd"] <= _x_bar(kappa, n):
                fails.append(f"{label}: x forward {stats['x_fwd']:.3e} > {_x_bar(kappa, n):.3e}")
        if not stats["L_fwd"] <= TOL:
            fails.append(f"{label}: L forward {stats['L_fwd']:.3e}")
        if not np.array_equal(info.cpu().numpy(), info_ref) or info_ref.any():
            fails.append(f"{label}: info")
        if not _upper_pos_zero(Lg):
            fails.append(f"{label}: strict upper not +0")
    elif op == "potrs":
        L, B = g("L"), g("B")
        st = glass.glass_potrs_batched(n, nrhs, BATCH, L, B, force)
        torch.cuda.synchronize()
        if st != 0:
            return [f"{label}: status {st}"], {}
        Xg = B.cpu().numpy()
        X_ref = oracle.potrs(case["L"], case["B"])
        L64 = case["L"].astype(np.float64)
        A64 = np.matmul(L64, np.swapaxes(L64, 1, 2))
        stats = {"x_fwd": normwise(Xg, X_ref).max(), "rho_s": _rho_s(A64, Xg, case["B"]).max()}
        if not stats["x_fwd"] <= _x_bar(kappa, n):
            fails.append(f"{label}: x forward {stats['x_fwd']:.3e} > {_x_bar(kappa, n):.3e}")
    else:  # trsv, both transposes
        stats = {"x_fwd": 0.0, "rho_s": 0.0}
        for trans in (0, 1):
            L, x = g("L"), g("x")
            st = glass.glass_trsv_batched(n, BATCH, trans, L, x, force)
            torch.cuda.synchronize()
            if st != 0:
                return [f"{label}: trans={trans} status {st}"], {}
            xg = x.cpu().numpy()
            x_ref = oracle.trsv(case["L"], case["x"], trans)
            M = case["L"] if trans == 0 else np.swapaxes(case["L"], 1, 2)
            stats["x_fwd"] = max(stats["x_fwd"], normwise(xg, x_ref).max())
            stats["rho_s"] = max(stats["rho_s"], _rho_s(M, xg[..., None], case["x"][..., None]).max())
        k_op = np.sqrt(kappa)
        if not stats["x_fwd"] <= _x_bar(k_op, n):
            fails.append(f"{label}: x forward {stats['x_fwd']:.3e} > {_x_bar(k_op, n):.3e}")
    for key in ("rho_f", "rho_s"):
        if key in stats and not stats[key] <= RHO_MAX:
            fails.append(f"{label}: {key} {stats[key]:.2f} > {RHO_MAX}")
    if not all(guards_intact(b) for b in bufs):
        fails.append(f"{label}: guard band overwritten")
    return fails, stats


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", ["potrf", "posv", "potrs", "trsv"])
def test_conditioned_and_scaled(env, op, scope):
    glass, torch = env
    fails = []
    worst = {}
    for n in NS:
        if glass.glass_placement_feasible(glass.OPS[op], n, 1, glass.SCOPES[scope], 1) != 1:
            continue
        for kappa in KAPPAS:
            for s in SCALES:
                _say(f"{op} n={n} kappa={kappa:.0e} s={s} {scope}/P=1")
                f, stats = _run(glass, torch, op, n, kappa, s, scope)
                fails += f
                for k, v in stats.items():
                    worst[(k, n, kappa)] = max(worst.get((k, n, kappa), 0.0), float(v))
    for (k, n, kappa), v in sorted(worst.items()):
        _say(f"  worst {k} n={n} kappa={kappa:.0e}: {v:.3e}")
    assert not fails, "\n".join(fails[:40])


@pytest.mark.parametrize("scope", ["wave", "subwave", "thread", "workgroup"])
@pytest.mark.parametrize("op", ["posv", "potrs"])
def test_conditioned_multi_rhs(env, op, scope):
    """Several right-hand sides at kappa = 1e4: the blocked kernel's
    substitutions take 16 columns per pass through the diagonal-block
    inverses."""
    glass, torch = env
    fails = []
    for n in (12, 24, 32, 64):
        for nrhs in (3, 17):
            if glass.glass_placement_feasible(glass.OPS[op], n, nrhs, glass.SCOPES[scope], 1) != 1:
                continue
            _say(f"{op} n={n} nrhs={nrhs} kappa=1e4 {scope}/P=1")
            f, _ = _run(glass, torch, op, n, 1e4, 0, scope, nrhs=nrhs)
            fails += f
    assert not fails, "\n".join(fails)
