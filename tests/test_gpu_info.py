"""GPU: failed factorizations inside a batch, at every scope.

Problems whose matrix is clearly indefinite at a planted column k (A_kk set
to -100, far below any rounding margin) must report info = k + 1 exactly,
and every other problem of the batch -- in particular its neighbours that
share a wavefront at sub-wave scope -- must still match the oracle: a NaN
born in one problem may not leak into another.  B of a failed problem is
unspecified by the contract and is not compared.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from helpers import TOL, guarded, guards_intact, normwise
from paper_2609_28179_amd import inputs

pytestmark = pytest.mark.gpu

# planted failures: (problem, column); neighbours 2..5 share one sub-wave
# wavefront at orders <= 16 (four per wavefront), 32/33 at orders <= 32.
PLANTS = ((2, 0), (3, 5), (5, 1), (32, 3), (66, 2))
BATCH = 67


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2609_28179_amd import glass
    assert torch.cuda.is_available()
    return glass, torch


def _planted(n, seed):
    rng = np.random.default_rng(seed)
    A = inputs.spd(rng, BATCH, n)
    B = inputs.uniform(rng, (BATCH, n, 2))
    want = np.zeros(BATCH, np.int32)
    for p, k in PLANTS:
        k = min(k, n - 1)
        A[p, k, k] = -100.0
        want[p] = k + 1
    return A, B, want


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", ["potrf", "posv"])
def test_planted_failures(env, op, scope):
    glass, torch = env
    fails = []
    for n in (1, 3, 8, 13, 16, 17, 24, 32, 40):
        if glass.glass_placement_feasible(glass.OPS[op], n, 2, glass.SCOPES[scope], 1) != 1:
            continue
        print(f"{op} n={n} {scope} planted failures", flush=True)
        sys.stdout.flush()
        A, B, want = _planted(n, 1000 + n)
        if op == "potrf":
            L_ref, info_ref = oracle.potrf(A)
        else:
            L_ref, X_ref, info_ref = oracle.posv(A, B)
        assert np.array_equal(info_ref, want), "oracle must report the planted pivots"
        Af, Ad = guarded(torch, A, "cuda:0")
        Bf, Bd = guarded(torch, B, "cuda:0")
        info = torch.full((BATCH,), -7, dtype=torch.int32, device="cuda:0")
        if op == "potrf":
            st = glass.glass_potrf_batched(n, BATCH, Ad, info, (scope, 1))
        else:
            st = glass.glass_posv_batched(n, 2, BATCH, Ad, Bd, info, (scope, 1))
        torch.cuda.synchronize()
        label = f"{op} n={n} {scope}"
        if st != 0:
            fails.append(f"{label}: status {st}")
            continue
        got = info.cpu().numpy()
        if not np.array_equal(got, want):
            fails.append(f"{label}: info {got[want != 0]} vs {want[want != 0]}, "
                         f"{int(np.count_nonzero(got[want == 0]))} spurious")
        ok = want == 0
        err = normwise(np.tril(Ad.cpu().numpy())[ok], L_ref[ok]).max()
        if op == "posv":
            err = max(err, normwise(Bd.cpu().numpy()[ok], X_ref[ok]).max())
        if not err <= TOL:
            fails.append(f"{label}: healthy problems err {err:.3e}")
        if not (guards_intact(Af) and guards_intact(Bf)):
            fails.append(f"{label}: guard band written")
    assert not fails, "\n".join(fails)


# a pivot that is exactly zero in any precision: in [[4,2,0],[2,1,3],[0,3,5]]
# l_21 = 1 exactly and the second pivot is 1 - 1 = 0, so info = 2 (leading
# minors 4, 0, -36); placed at offset o inside the identity, info = o + 2
ZERO_PIVOT_BLOCK = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 3.0], [0.0, 3.0, 5.0]])


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", ["potrf", "posv"])
def test_exact_zero_pivot(env, op, scope):
    glass, torch = env
    fails = []
    for n in (3, 8, 16, 24, 32, 40, 64):
        if glass.glass_placement_feasible(glass.OPS[op], n, 1, glass.SCOPES[scope], 1) != 1:
            continue
        for o in sorted({0, n - 3, min(17, n - 3)}):
            label = f"{op} n={n} {scope} zero pivot at {o + 1}"
            print(label, flush=True)
            sys.stdout.flush()
            rng = np.random.default_rng(2000 + n + o)
            batch = 5
            A = inputs.spd(rng, batch, n)
            B = inputs.uniform(rng, (batch, n, 1))
            Z = np.eye(n)
            Z[o:o + 3, o:o + 3] = ZERO_PIVOT_BLOCK
            A[2] = Z.astype(np.float32)
            want = np.zeros(batch, np.int32)
            want[2] = o + 2
            if op == "potrf":
                L_ref, info_ref = oracle.potrf(A)
            else:
                L_ref, X_ref, info_ref = oracle.posv(A, B)
            assert np.array_equal(info_ref, want), "oracle must report the exact zero pivot"
            Af, Ad = guarded(torch, A, "cuda:0")
            Bf, Bd = guarded(torch, B, "cuda:0")
            info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
            if op == "potrf":
                st = glass.glass_potrf_batched(n, batch, Ad, info, (scope, 1))
            else:
                st = glass.glass_posv_batched(n, 1, batch, Ad, Bd, info, (scope, 1))
            torch.cuda.synchronize()
            if st != 0:
                fails.append(f"{label}: status {st}")
                continue
            got = info.cpu().numpy()
            if not np.array_equal(got, want):
                fails.append(f"{label}: info {got.tolist()} vs {want.tolist()}")
            ok = want == 0
            err = normwise(np.tril(Ad.cpu().numpy())[ok], L_ref[ok]).max()
            if op == "posv":
                err = max(err, normwise(Bd.cpu().numpy()[ok], X_ref[ok]).max())
            if not err <= TOL:
                fails.append(f"{label}: healthy problems err {err:.3e}")
            if not (guards_intact(Af) and guards_intact(Bf)):
                fails.append(f"{label}: guard band written")
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", ["potrf", "posv"])
def test_nonfinite_pivots(env, op, scope):
    """info follows !(pivot > 0) exactly for non-finite pivots too: a NaN
    pivot fails (info = k + 1), a +inf pivot does not (info = 0; the
    factor of that problem is not compared).  The row kernels test the
    pivot through 1 / L_kk = rsq(d), which is non-finite exactly for the
    failing pivots, +0 at +inf."""
    glass, torch = env
    fails = []
    for n in (3, 8, 16, 24, 32, 40, 64):
        if glass.glass_placement_feasible(glass.OPS[op], n, 1, glass.SCOPES[scope], 1) != 1:
            continue
        label = f"{op} n={n} {scope} non-finite pivots"
        print(label, flush=True)
        sys.stdout.flush()
        k = min(5, n - 1)
        rng = np.random.default_rng(3000 + n)
        batch = 5
        A = inputs.spd(rng, batch, n)
        B = inputs.uniform(rng, (batch, n, 1))
        A[1, k, k] = np.float32(np.nan)
        A[3, k, k] = np.float32(np.inf)
        want = np.array([0, k + 1, 0, 0, 0], np.int32)
        with np.errstate(invalid="ignore", over="ignore", divide="ignore"):
            if op == "potrf":
                L_ref, info_ref = oracle.potrf(A)
            else:
                L_ref, X_ref, info_ref = oracle.posv(A, B)
        assert np.array_equal(info_ref, want), ("oracle", info_ref)
        Af, Ad = guarded(torch, A, "cuda:0")
        Bf, Bd = guarded(torch, B, "cuda:0")
        info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
        if op == "potrf":
            st = glass.glass_potrf_batched(n, batch, Ad, info, (scope, 1))
        else:
            st = glass.glass_posv_batched(n, 1, batch, Ad, Bd, info, (scope, 1))
        torch.cuda.synchronize()
        if st != 0:
            fails.append(f"{label}: status {st}")
            continue
        got = info.cpu().numpy()
        if not np.array_equal(got, want):
            fails.append(f"{label}: info {got.tolist()} vs {want.tolist()}")
        ok = np.array([True, False, True, False, True])
        err = normwise(np.tril(Ad.cpu().numpy())[ok], L_ref[ok]).max()
        if op == "posv":
            err = max(err, normwise(Bd.cpu().numpy()[ok], X_ref[ok]).max())
        if not err <= TOL:
            fails.append(f"{label}: healthy problems err {err:.3e}")
        if not (guards_intact(Af) and guards_intact(Bf)):
            fails.append(f"{label}: guard band written")
    assert not fails, "\n".join(fails)
