"""GPU parity: every op x scope x pack against the FP64 oracle, through the C-ABI.

Bar: max per-problem normwise error <= 1e-4; bit-exact for the integer and
structural outputs (info, the +0 strict upper triangle of L, SE(3) row 3,
guard bands around every buffer); within one scope the outputs are
bit-identical across pack factors (the per-problem arithmetic does not depend
on P, so a difference would expose a race or an indexing error).
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

from helpers import PACKS, TOL, run_case

pytestmark = pytest.mark.gpu

OPS_N = ("gemm", "gemv", "potrf", "potrs", "posv", "trsv")
N_WIDE = (1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 15, 16, 17, 20, 24, 31, 32, 33, 48, 63, 64)
N_THREAD = (1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 14, 16)
N_PACKS = (3, 6, 16, 33, 64)
BATCHES = (1, 67, 1100)


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2609_28179_amd import glass
    assert torch.cuda.is_available()
    return glass, torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _check(res, label, fails):
    if res["status"] != 0:
        fails.append(f"{label}: status {res['status']}")
        return
    if not res["err"] <= TOL:
        fails.append(f"{label}: err {res['err']:.3e}")
    for key in ("upper_pos_zero", "info_exact", "row3_exact", "guards"):
        if key in res and not res[key]:
            fails.append(f"{label}: {key} failed")


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", OPS_N)
def test_parity_square_ops(env, op, scope):
    glass, torch = env
    fails = []
    ns = N_THREAD if scope == "thread" else N_WIDE
    for n in ns:
        for pack in PACKS:
            if pack != 1 and n not in N_PACKS and n not in (4, 12):
                continue
            feas = glass.glass_placement_feasible(glass.OPS[op], n, 1, glass.SCOPES[scope], pack)
            # the last workgroup ends part-way (at sub-wave P = 8, 32
            # problems per workgroup: one partial wavefront at 67, a full and
            # a partial one at 70)
            for batch in BATCHES if pack == 1 else (67, 70):
                label = f"{op} n={n} batch={batch} {scope}/P={pack}"
                if feas != 1:
                    res = run_case(glass, torch, op, n, 1, scope, pack, check_guards=False)
                    if res["status"] != glass.ERR_INFEASIBLE_PLACEMENT:
                        fails.append(f"{label}: infeasible placement returned {res['status']}")
                    break
                _say(label)
                _check(run_case(glass, torch, op, n, batch, scope, pack), label, fails)
    assert not fails, "\n".join(fails[:40])


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", ["se3_compose", "se3_inverse"])
def test_parity_se3(env, op, scope):
    glass, torch = env
    fails = []
    for pack in PACKS:
        feas = glass.glass_placement_feasible(glass.OPS[op], 4, 1, glass.SCOPES[scope], pack)
        for batch in (1, 67, 1100, 5000):
            label = f"{op} batch={batch} {scope}/P={pack}"
            _say(label)
            res = run_case(glass, torch, op, 4, batch, scope, pack, check_guards=feas == 1)
            if feas != 1:
                if res["status"] != glass.ERR_INFEASIBLE_PLACEMENT:
                    fails.append(f"{label}: infeasible placement returned {res['status']}")
                continue
            _check(res, label, fails)
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("scope", ["wave", "workgroup", "thread", "subwave"])
@pytest.mark.parametrize("op,nrhs", [("posv", 2), ("posv", 3), ("posv", 4), ("posv", 8), ("posv", 9), ("posv", 12),
                                     ("potrs", 5), ("potrs", 12), ("potrs", 64), ("posv", 64)])
def test_parity_multi_rhs(env, op, nrhs, scope):
    glass, torch = env
    fails = []
    for n in (1, 5, 8, 12, 16, 24, 28, 40, 64):
        for pack in (1, 2):
            feas = glass.glass_placement_feasible(glass.OPS[op], n, nrhs, glass.SCOPES[scope], pack)
            if feas != 1:
                continue
            label = f"{op} n={n} nrhs={nrhs} batch=67 {scope}/P={pack}"
            _say(label)
            _check(run_case(glass, torch, op, n, 67, scope, pack, nrhs=nrhs), label, fails)
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
def test_parity_trsv_transposed(env, scope):
    glass, torch = env
    fails = []
    for n in (1, 3, 7, 16, 25, 32, 33, 64):
        if glass.glass_placement_feasible(glass.OP_TRSV, n, 1, glass.SCOPES[scope], 1) != 1:
            continue
        label = f"trsv trans=1 n={n} {scope}"
        _say(label)
        _check(run_case(glass, torch, "trsv", n, 130, scope, 1, trans=1), label, fails)
    assert not fails, "\n".join(fails)


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", ["gemm", "potrf", "posv", "trsv", "gemv", "potrs", "se3_compose"])
def test_bit_identical_across_packs(env, op, scope):
    glass, torch = env
    from paper_2609_28179_amd import inputs
    for n in ((4,) if op.startswith("se3") else (6, 12, 33)):
        case = inputs.make_case(op, n, 300, cfg=101)
        outs = []
        for pack in PACKS:
            if glass.glass_placement_feasible(glass.OPS[op], n, 1, glass.SCOPES[scope], pack) != 1:
                continue
            _say(f"{op} n={n} {scope}/P={pack} (cross-pack)")
            res = run_case(glass, torch, op, n, 300, scope, pack, case=case)
            assert res["status"] == 0
            outs.append(res["out"])
        for o in outs[1:]:
            assert np.array_equal(o.view(np.uint32), outs[0].view(np.uint32)), f"{op} n={n} {scope}"


# operands 4, 8 and 12 bytes past a 16-byte boundary: every staging and
# store path that widens to 16 bytes must fall back (contract: 4-byte aligned)
N_SHIFT = {"thread": (3, 4, 6, 7, 8, 10, 16), "wave": (3, 8, 12, 16, 20, 25, 32, 64), "workgroup": (3, 16, 33),
           "subwave": (4, 7, 12, 16, 24, 32)}


@pytest.mark.parametrize("scope", ["thread", "wave", "workgroup", "subwave"])
@pytest.mark.parametrize("op", OPS_N + ("se3_compose", "se3_inverse"))
def test_parity_unaligned_operands(env, op, scope):
    glass, torch = env
    fails = []
    for n in ((4,) if op.startswith("se3") else N_SHIFT[scope]):
        if glass.glass_placement_feasible(glass.OPS[op], n, 1, glass.SCOPES[scope], 1) != 1:
            continue
        for shift in (1, 2, 3):
            label = f"{op} n={n} batch=67 {scope}/P=1 shift={shift}"
            _say(label)
            _check(run_case(glass, torch, op, n, 67, scope, 1, shift=shift), label, fails)
    assert not fails, "\n".join(fails[:40])
