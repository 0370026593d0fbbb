"""GPU parity of the contract paths the header promises beyond the square
alpha = 1, beta = 0 calls (Sec. III-B lists the BLAS L2/L3 forms; Sec. III-C
asks that validation cover layouts and scopes):

  - GEMV with alpha != 1, beta != 0 and m != n, at every scope and pack;
  - GEMM with alpha / beta at every scope, rectangular where the scope allows;
  - beta == 0 with C / y pre-filled with NaN: C / y are not read, so the
    outputs are finite and match the oracle;
  - SE(3) with Tout equal to Ta or to Tb (problems are read before written);
  - the POSV adjoint in place, dB equal to G.

Each case is compared with the FP64 oracle at 1e-4 normwise per problem, with
NaN guard bands around every buffer.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from helpers import PACKS, TOL, guarded, guards_intact, normwise
from paper_2609_28179_amd import inputs

pytestmark = pytest.mark.gpu

SCOPES = ("thread", "wave", "workgroup", "subwave")


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2609_28179_amd import glass
    assert torch.cuda.is_available()
    return glass, torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rng(*key):
    return np.random.default_rng(np.random.SeedSequence([400, *key]))


def _gemv_feasible(glass, scope, m, n, pack):
    """GEMV shapes each scope runs: thread m == n <= 16, sub-wave m, n <= 16,
    wave and workgroup any m, n <= 64; the pack factor through the library's
    own rule for the square order max(m, n)."""
    if scope == "thread" and not (m == n and n <= 16):
        return False
    if scope == "subwave" and max(m, n) > 16:
        return False
    return glass.glass_placement_feasible(glass.OP_GEMV, max(m, n), 1, glass.SCOPES[scope], pack) == 1


def _gemm_feasible(glass, scope, m, n, k, pack):
    if scope == "thread" and not (m == n == k and n <= 12):
        return False
    if scope == "subwave" and max(m, n, k) > 16:
        return False
    return glass.glass_placement_feasible(glass.OP_GEMM, max(m, n, k), 1, glass.SCOPES[scope], pack) == 1


GEMV_SHAPES = [(1, 1), (4, 4), (7, 7), (12, 12), (16, 16), (33, 33), (64, 64),
               (7, 12), (12, 7), (16, 3), (3, 16), (33, 5), (5, 33), (64, 17), (17, 64)]


@pytest.mark.parametrize("scope", SCOPES)
def test_gemv_alpha_beta_rectangular(env, scope):
    glass, torch = env
    fails = []
    for (m, n) in GEMV_SHAPES:
        for pack in PACKS:
            if not _gemv_feasible(glass, scope, m, n, pack):
                continue
            for batch in ((1, 67, 1100) if pack == 1 else (67,)):
                rng = _rng(1, m, n, batch)
                A = inputs.uniform(rng, (batch, m, n))
                x = inputs.uniform(rng, (batch, n))
                y0 = inputs.uniform(rng, (batch, m))
                label = f"gemv m={m} n={n} batch={batch} {scope}/P={pack} alpha=1.5 beta=0.5"
                _say(label)
                bufs = [guarded(torch, a, "cuda:0") for a in (A, x, y0)]
                st = glass.glass_gemv_batched(m, n, batch, 1.5, bufs[0][1], bufs[1][1], 0.5, bufs[2][1],
                                              (scope, pack))
                torch.cuda.synchronize()
                if st != 0:
                    fails.append(f"{label}: status {st}")
                    continue
                ref = oracle.gemv(A, x, y0, alpha=1.5, beta=0.5)
                err = normwise(bufs[2][1].cpu().numpy(), ref).max()
                if not err <= TOL:
                    fails.append(f"{label}: err {err:.3e}")
                if not all(guards_intact(b[0]) for b in bufs):
                    fails.append(f"{label}: guard band")
    assert not fails, "\n".join(fails[:40])


GEMM_SHAPES = [(1, 1, 1), (3, 3, 3), (6, 6, 6), (12, 12, 12), (16, 16, 16), (7, 12, 5), (16, 3, 9),
               (12, 16, 16), (5, 5, 16), (33, 20, 8), (64, 17, 48), (64, 64, 64)]


@pytest.mark.parametrize("scope", SCOPES)
def test_gemm_alpha_beta(env, scope):
    glass, torch = env
    fails = []
    for (m, n, k) in GEMM_SHAPES:
        for pack in PACKS:
            if not _gemm_feasible(glass, scope, m, n, k, pack):
                continue
            for batch in ((1, 67, 1100) if pack == 1 else (67,)):
                rng = _rng(2, m, n, k, batch)
                A = inputs.uniform(rng, (batch, m, k))
                B = inputs.uniform(rng, (batch, k, n))
                C0 = inputs.uniform(rng, (batch, m, n))
                label = f"gemm m={m} n={n} k={k} batch={batch} {scope}/P={pack} alpha=-0.75 beta=1.25"
                _say(label)
                bufs = [guarded(torch, a, "cuda:0") for a in (A, B, C0)]
                st = glass.glass_gemm_batched(m, n, k, batch, -0.75, bufs[0][1], bufs[1][1], 1.25, bufs[2][1],
                                              (scope, pack))
                torch.cuda.synchronize()
                if st != 0:
                    fails.append(f"{label}: status {st}")
                    continue
                ref = oracle.gemm(A, B, C0, alpha=-0.75, beta=1.25)
                err = normwise(bufs[2][1].cpu().numpy(), ref).max()
                if not err <= TOL:
                    fails.append(f"{label}: err {err:.3e}")
                if not all(guards_intact(b[0]) for b in bufs):
                    fails.append(f"{label}: guard band")
    assert not fails, "\n".join(fails[:40])


@pytest.mark.parametrize("scope", SCOPES)
@pytest.mark.parametrize("op", ["gemm", "gemv"])
def test_beta_zero_does_not_read_output(env, op, scope):
    """beta == 0: C (y) is not read, so NaN there must not reach the result."""
    glass, torch = env
    fails = []
    shapes = GEMM_SHAPES if op == "gemm" else GEMV_SHAPES
    for shp in shapes:
        for pack in (1, 2):
            ok = _gemm_feasible(glass, scope, *shp, pack) if op == "gemm" else _gemv_feasible(glass, scope, *shp, pack)
            if not ok:
                continue
            batch = 67
            rng = _rng(3, *shp, pack)
            label = f"{op} {shp} batch={batch} {scope}/P={pack} beta=0 over NaN"
            _say(label)
            if op == "gemm":
                m, n, k = shp
                A = inputs.uniform(rng, (batch, m, k))
                B = inputs.uniform(rng, (batch, k, n))
                Ad, Bd = (guarded(torch, a, "cuda:0") for a in (A, B))
                Cf = torch.full((batch * m * n + 128,), float("nan"), dtype=torch.float32, device="cuda:0")
                C = Cf[64:64 + batch * m * n].view(batch, m, n)
                st = glass.glass_gemm_batched(m, n, k, batch, 1.5, Ad[1], Bd[1], 0.0, C, (scope, pack))
                ref = oracle.gemm(A, B, alpha=1.5)
                bufs = (Ad[0], Bd[0], Cf)
            else:
                m, n = shp
                A = inputs.uniform(rng, (batch, m, n))
                x = inputs.uniform(rng, (batch, n))
                Ad, xd = (guarded(torch, a, "cuda:0") for a in (A, x))
                Cf = torch.full((batch * m + 128,), float("nan"), dtype=torch.float32, device="cuda:0")
                C = Cf[64:64 + batch * m].view(batch, m)
                st = glass.glass_gemv_batched(m, n, batch, 1.5, Ad[1], xd[1], 0.0, C, (scope, pack))
                ref = oracle.gemv(A, x, alpha=1.5)
                bufs = (Ad[0], xd[0], Cf)
            torch.cuda.synchronize()
            if st != 0:
                fails.append(f"{label}: status {st}")
                continue
            got = C.cpu().numpy()
            if not np.isfinite(got).all():
                fails.append(f"{label}: NaN propagated from C")
                continue
            err = normwise(got, ref).max()
            if not err <= TOL:
                fails.append(f"{label}: err {err:.3e}")
            if not all(guards_intact(b) for b in bufs):
                fails.append(f"{label}: guard band")
    assert not fails, "\n".join(fails[:40])


@pytest.mark.parametrize("scope", SCOPES)
def test_se3_output_aliases_input(env, scope):
    """Tout may be exactly Ta or Tb: every problem is read before it is written."""
    glass, torch = env
    fails = []
    for pack in (1, 2, 8):
        if glass.glass_placement_feasible(glass.OP_SE3_COMPOSE, 4, 1, glass.SCOPES[scope], pack) != 1:
            continue
        for batch in (1, 67, 1100):
            case = inputs.make_case("se3_compose", 4, batch, cfg=401)
            ref_c = oracle.se3_compose(case["Ta"], case["Tb"])
            ref_i = oracle.se3_inverse(case["Ta"])
            for which in ("Ta", "Tb", "inverse"):
                label = f"se3 {which} aliased batch={batch} {scope}/P={pack}"
                _say(label)
                Taf, Ta = guarded(torch, case["Ta"], "cuda:0")
                Tbf, Tb = guarded(torch, case["Tb"], "cuda:0")
                if which == "Ta":
                    st = glass.glass_se3_batched(glass.OP_SE3_COMPOSE, batch, Ta, Tb, Ta, (scope, pack))
                    out, ref = Ta, ref_c
                elif which == "Tb":
                    st = glass.glass_se3_batched(glass.OP_SE3_COMPOSE, batch, Ta, Tb, Tb, (scope, pack))
                    out, ref = Tb, ref_c
                else:
                    st = glass.glass_se3_batched(glass.OP_SE3_INVERSE, batch, Ta, None, Ta, (scope, pack))
                    out, ref = Ta, ref_i
                torch.cuda.synchronize()
                if st != 0:
                    fails.append(f"{label}: status {st}")
                    continue
                T = out.cpu().numpy()
                err = normwise(T[:, :3, :], ref[:, :3, :]).max()
                if not err <= TOL:
                    fails.append(f"{label}: err {err:.3e}")
                if not np.array_equal(T[:, 3, :], np.broadcast_to([0, 0, 0, 1], (batch, 4))):
                    fails.append(f"{label}: row 3")
                if not (guards_intact(Taf) and guards_intact(Tbf)):
                    fails.append(f"{label}: guard band")
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("scope", ["thread", "wave", "subwave"])
@pytest.mark.parametrize("n,r,batch", [(1, 1, 5), (6, 1, 67), (12, 3, 1100), (16, 2, 130), (24, 1, 70),
                                       (33, 4, 65), (64, 8, 9)])
def test_adjoint_in_place(env, scope, n, r, batch):
    """dB may be G exactly: the in-place adjoint matches the FP64 oracle."""
    glass, torch = env
    if glass.glass_placement_feasible(glass.OP_POSV_ADJOINT, n, r, glass.SCOPES[scope], 1) != 1:
        pytest.skip("infeasible placement")
    _say(f"adjoint in place n={n} nrhs={r} batch={batch} {scope}")
    rng = inputs.rng_for(3, "adjoint", n, batch, 77 + r)
    L = inputs.lower_factor(rng, batch, n)
    X = inputs.uniform(rng, (batch, n, r))
    W = inputs.uniform(rng, (batch, n, r))
    dB_ref, dA_ref = oracle.posv_adjoint(L, X, W)
    Lf, Ld = guarded(torch, L, "cuda:0")
    Xf, Xd = guarded(torch, X, "cuda:0")
    Gf, Gd = guarded(torch, W, "cuda:0")
    dAf, dAd = guarded(torch, np.zeros((batch, n, n), np.float32), "cuda:0")
    st = glass.glass_posv_adjoint_batched(n, r, batch, Ld, Xd, Gd, Gd, dAd, (scope, 1))
    torch.cuda.synchronize()
    assert st == 0, st
    assert normwise(Gd.cpu().numpy(), dB_ref).max() <= TOL
    assert normwise(dAd.cpu().numpy(), dA_ref).max() <= TOL
    assert all(guards_intact(b) for b in (Lf, Xf, Gf, dAf))
