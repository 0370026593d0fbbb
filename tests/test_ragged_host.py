"""Host-side checks of the ragged batch: generator shape, the CPU reference
permutation, workspace size and argument validation (no device calls)."""
import numpy as np
import pytest

import oracle
from paper_2609_28179_amd import inputs


def test_generator_and_reference_order():
    case = inputs.make_ragged(1000, seed=5)
    n, r = case["n"], case["nrhs"]
    assert set(np.unique(n)) <= set(inputs.RAGGED_SIZES)
    assert r.min() >= 1 and r.max() <= 8
    assert case["offA"][0] == 0 and np.all(np.diff(case["offA"]) == n[:-1].astype(np.int64) ** 2)
    assert case["A"].size == int((n.astype(np.int64) ** 2).sum())
    order = oracle.ragged_order(n)
    cls = (n[order] - 1) // 8
    assert np.all(np.diff(cls) <= 0)                      # largest class first
    for c in np.unique(cls):                              # stable within a class
        idx = order[cls == c]
        assert np.all(np.diff(idx) > 0)
    assert sorted(order.tolist()) == list(range(1000))


def test_oracle_ragged_matches_per_problem_solve():
    case = inputs.make_ragged(40, seed=9)
    A_out, B_out, info = oracle.posv_ragged(case["n"], case["nrhs"], case["offA"], case["offB"], case["A"], case["B"])
    assert (info == 0).all()
    for i in (0, 7, 39):
        n, r = int(case["n"][i]), int(case["nrhs"][i])
        A = case["A"][case["offA"][i]:case["offA"][i] + n * n].reshape(n, n).astype(np.float64)
        b = case["B"][case["offB"][i]:case["offB"][i] + n * r].reshape(n, r).astype(np.float64)
        x = np.linalg.solve(A, b)
        got = B_out[case["offB"][i]:case["offB"][i] + n * r].reshape(n, r)
        assert np.max(np.abs(got - x)) <= 1e-10


def test_oracle_ragged_every_problem_against_numpy():
    """Every problem of a ragged batch (all nine orders, 1..8 right-hand
    sides): the packed L is the lower Cholesky factor (numpy.linalg.cholesky,
    LAPACK) with a +0 strict upper part, and the packed X solves A X = B
    (numpy.linalg.solve, LU), so the oracle's packing and unpacking are
    pinned on every offset, not only on a few problems."""
    case = inputs.make_ragged(300, seed=11)
    n, r, offA, offB = case["n"], case["nrhs"], case["offA"], case["offB"]
    A_out, B_out, info = oracle.posv_ragged(n, r, offA, offB, case["A"], case["B"])
    assert (info == 0).all()
    assert A_out.shape == case["A"].shape and B_out.shape == case["B"].shape
    assert set(np.unique(n)) == set(inputs.RAGGED_SIZES)
    for i in range(len(n)):
        ni, ri = int(n[i]), int(r[i])
        A = case["A"][offA[i]:offA[i] + ni * ni].reshape(ni, ni).astype(np.float64)
        b = case["B"][offB[i]:offB[i] + ni * ri].reshape(ni, ri).astype(np.float64)
        L = A_out[offA[i]:offA[i] + ni * ni].reshape(ni, ni)
        X = B_out[offB[i]:offB[i] + ni * ri].reshape(ni, ri)
        iu = np.triu_indices(ni, 1)
        assert (L[iu] == 0).all() and not np.signbit(L[iu]).any(), i
        Lnp = np.linalg.cholesky(A)
        assert np.max(np.abs(L - Lnp)) <= 1e-12 * np.max(np.abs(Lnp)), i
        Xnp = np.linalg.solve(A, b)
        assert np.max(np.abs(X - Xnp)) <= 1e-11 * max(1.0, np.max(np.abs(Xnp))), i


def test_oracle_ragged_info_and_untouched_neighbours():
    """A planted indefinite problem reports its own 1-based failing column
    (Sylvester: the leading minor of order k+1 turns negative) and leaves the
    other problems' results as in a clean run."""
    case = inputs.make_ragged(30, seed=12)
    n, r, offA, offB = case["n"], case["nrhs"], case["offA"], case["offB"]
    clean = oracle.posv_ragged(n, r, offA, offB, case["A"], case["B"])
    A = case["A"].copy()
    bad, k = 4, 2
    nb = int(n[bad])
    A[offA[bad] + k * nb + k] = -100.0
    A_out, B_out, info = oracle.posv_ragged(n, r, offA, offB, A, case["B"])
    assert info[bad] == k + 1
    assert (np.delete(info, bad) == 0).all()
    for i in range(len(n)):
        if i == bad:
            continue
        sa = slice(offA[i], offA[i] + int(n[i]) ** 2)
        sb = slice(offB[i], offB[i] + int(n[i]) * int(r[i]))
        assert np.array_equal(A_out[sa], clean[0][sa]) and np.array_equal(B_out[sb], clean[1][sb])


def test_ragged_validation_without_device():
    from paper_2609_28179_amd import glass
    F = 0x10000
    assert glass.glass_posv_ragged_workspace_size(0) >= 32 * 4
    w = glass.glass_posv_ragged_workspace_size(50000)
    assert w == 4 * ((50000 + 1023) // 1024 * 8 + 32 + 50000)
    assert glass.glass_posv_ragged_perm_offset(50000) == w - 4 * 50000
    assert glass.glass_posv_ragged(0, None, None, None, None, None, None, None, None, 0, stream=0) == glass.OK
    assert glass.glass_posv_ragged(-1, F, F, F, F, F, F, F, F, w, stream=0) == glass.ERR_INVALID_VALUE
    assert glass.glass_posv_ragged(10, F, F, F, F, F, F, None, F, w, stream=0) == glass.ERR_INVALID_VALUE
    assert glass.glass_posv_ragged(10, F, F, F, F, F, F, F, F, 8, stream=0) == glass.ERR_INVALID_VALUE
    bad = ["wave"] * 8
    bad[3] = "thread"
    assert glass.glass_posv_ragged(10, F, F, F, F, F, F, F, F, w, class_scope=bad, stream=0) == \
        glass.ERR_INFEASIBLE_PLACEMENT
    assert glass.glass_posv_ragged(10, F, F, F, F, F, F, F, F, w, class_scope=[7] * 8, stream=0) == \
        glass.ERR_INVALID_VALUE
    bad = ["wave"] * 8
    bad[3] = "subwave"   # sub-wave segments hold orders up to 24 (classes 0 to 2)
    assert glass.glass_posv_ragged(10, F, F, F, F, F, F, F, F, w, class_scope=bad, stream=0) == \
        glass.ERR_INFEASIBLE_PLACEMENT
    assert glass.glass_ragged_table_provenance().startswith("gfx950")


def test_ragged_noalloc_validation_without_device():
    """Argument errors of the no-allocation ragged call are found on the host
    before any device call (none is made here)."""
    from paper_2609_28179_amd import glass
    F = 0x10000
    mx = glass.glass_posv_ragged_noalloc_max_count()
    assert mx == 1 << 20
    assert glass.glass_posv_ragged_noalloc(0, None, None, None, None, None, None, None, stream=0) == glass.OK
    assert glass.glass_posv_ragged_noalloc(-1, F, F, F, F, F, F, F, stream=0) == glass.ERR_INVALID_VALUE
    assert glass.glass_posv_ragged_noalloc(mx + 1, F, F, F, F, F, F, F, stream=0) == glass.ERR_UNSUPPORTED
    assert glass.glass_posv_ragged_noalloc(10, F, F, F, F, F, F, None, stream=0) == glass.ERR_INVALID_VALUE
    assert glass.glass_posv_ragged_noalloc(10, None, F, F, F, F, F, F, stream=0) == glass.ERR_INVALID_VALUE
    bad = ["wave"] * 8
    bad[1] = "thread"
    assert glass.glass_posv_ragged_noalloc(10, F, F, F, F, F, F, F, class_scope=bad, stream=0) == \
        glass.ERR_INFEASIBLE_PLACEMENT
    assert glass.glass_posv_ragged_noalloc(10, F, F, F, F, F, F, F, class_scope=[9] * 8, stream=0) == \
        glass.ERR_INVALID_VALUE
