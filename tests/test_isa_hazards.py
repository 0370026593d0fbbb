"""Wait-state hazards and the occupancy cap, checked on the built library's
gfx950 code (no GPU needed).  The inline-asm DPP broadcasts, masked selects
and lane writes get no wait states from the compiler; their own `s_nop`s must
cover every path, whatever the compiler schedules around them, and this is
what guards that across compiler versions.  The checker itself is pinned on
small listings with a planted hazard."""
from __future__ import annotations

import os

import pytest

from tests import isa_hazards as hz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2609_28179_amd", "libglass.so")


@pytest.fixture(scope="module")
def scanned():
    if not os.path.exists(os.path.join(hz.LLVM, "llvm-objdump")):
        pytest.skip("ROCm LLVM tools not installed")
    assert os.path.exists(LIB), "libglass.so is not built"
    funcs, meta = hz.scan_library(LIB)
    return funcs, meta, hz.check(funcs)


def _listing(body: str, name: str = "k") -> list[dict]:
    """A one-function llvm-objdump listing from lines 'mnemonic operands'."""
    lines = [f"0000000000001000 <{name}>:"]
    addr = 0x1000
    for ins in body.strip().splitlines():
        ins, _, tgt = ins.strip().partition(" <")  # a branch target goes after the comment, as objdump prints it
        lines.append(f"\t{ins}  // {addr:012X}: 00000000" + (f" <{tgt}" if tgt else ""))
        addr += 4
    return hz.parse("\n".join(lines))


def _rules(funcs, **kw):
    return sorted(v[0] for v in hz.check(funcs, **kw)["violations"])


# ------------------------------------------------------ the checker itself --
def test_checker_flags_planted_dpp_hazard():
    bad = _listing("""
        v_mul_f32_e32 v3, v1, v2
        v_fmac_f32_dpp v4, v3, v5 row_newbcast:1 row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(bad) == ["dpp_src"]
    one = _listing("""
        v_mul_f32_e32 v3, v1, v2
        s_nop 0
        v_fmac_f32_dpp v4, v3, v5 row_newbcast:1 row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(one) == ["dpp_src"]
    ok = _listing("""
        v_mul_f32_e32 v3, v1, v2
        s_nop 1
        v_fmac_f32_dpp v4, v3, v5 row_newbcast:1 row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(ok) == []
    # src1 is not read across lanes: no hazard
    src1 = _listing("""
        v_mul_f32_e32 v3, v1, v2
        v_fmac_f32_dpp v4, v5, v3 row_newbcast:1 row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(src1) == []
    # register ranges and the self-broadcast form (vdst = src0)
    rng = _listing("""
        v_pk_mov_b32 v[6:7], v[0:1], v[0:1] op_sel:[0,1]
        v_fmac_f32_dpp v7, v7, -v9 row_newbcast:3 row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(rng) == ["dpp_src"]


def test_checker_follows_branches():
    # the write reaches the DPP read through the branch with one wait state
    # (the branch itself); the fall-through path is covered by the s_nop
    funcs = _listing("""
        v_add_f32_e32 v2, v0, v1
        s_cbranch_scc1 2 <k+0x10>
        s_nop 3
        s_nop 3
        v_mov_b32_dpp v3, v2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(funcs) == ["dpp_src"]
    # an unconditional branch ends the fall-through path
    funcs = _listing("""
        v_add_f32_e32 v2, v0, v1
        s_branch 2 <k+0x10>
        v_mov_b32_dpp v3, v2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf
        s_endpgm
        s_nop 1
        v_mov_b32_dpp v3, v2 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(funcs) == []


def test_checker_other_rules():
    trans = _listing("""
        v_rsq_f32_e32 v2, v1
        v_mul_f32_e32 v3, v2, v0
        s_endpgm
    """)
    assert _rules(trans) == ["trans_use"]
    lane = _listing("""
        v_readfirstlane_b32 s4, v1
        s_nop 1
        v_readlane_b32 s5, v2, s4
        s_endpgm
    """)
    assert _rules(lane) == ["lane_select"]
    lane_ok = _listing("""
        v_readfirstlane_b32 s4, v1
        s_nop 3
        v_readlane_b32 s5, v2, s4
        s_endpgm
    """)
    assert _rules(lane_ok) == []
    exec_w = _listing("""
        v_cmpx_gt_f32_e32 vcc, 0, v1
        s_nop 2
        v_mov_b32_dpp v3, v4 quad_perm:[1,0,3,2] row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert "dpp_exec" in _rules(exec_w)
    mfma = _listing("""
        v_mfma_f32_16x16x4_f32 v[0:3], v4, v5, v[0:3]
        s_nop 3
        v_mov_b32_dpp v6, v1 row_newbcast:1 row_mask:0xf bank_mask:0xf
        s_endpgm
    """)
    assert _rules(mfma, mfma_dpp_need=10) == ["mfma_dpp"]


# --------------------------------------------------------- the built code --
def test_scan_is_not_vacuous(scanned):
    funcs, vgprs, res = scanned
    names = " ".join(f["name"] for f in funcs)
    for k in ("chol_blk", "chol_seg", "adjoint", "ragged_solve", "gemv_wave_dpp", "gemm_mfma"):
        assert k in names, k
    assert res["counts"]["dpp"] > 10000
    assert res["counts"]["mfma"] > 1000
    assert res["counts"]["trans"] > 1000
    assert "v_mfma_f32_16x16x4_f32" in res["mfma_valu_min"]


def test_no_wait_state_hazards(scanned):
    _, _, res = scanned
    shown = [f"{rule} in {name}: {w.mn} {w.ops} -> {r.mn} {r.ops} after {d} wait states"
             for rule, name, w, r, d in res["violations"][:10]]
    assert res["violations"] == [], "\n".join(shown)


def test_blocked_potrf_occupancy_cap(scanned):
    # the whole-tile POTRF kernels at three and four tiles per side reserve
    # VGPRs up to v103: four waves per SIMD (512 VGPRs / 104 rounded to 8)
    _, meta, _ = scanned
    caps = {k: m["vgpr_count"] for k, m in meta.items()
            if "8chol_blkILi3ELi0ELb1E" in k or "8chol_blkILi4ELi0ELb1E" in k}
    assert len(caps) == 2, sorted(meta)[:5]
    for k, v in caps.items():
        assert 512 // (-(-v // 8) * 8) == 4, (k, v)


def test_no_kernel_spills_to_scratch(scanned):
    # a VGPR spill or a private segment is per-lane scratch in HBM on every
    # access of the spilled value: none of the kernels needs one
    _, meta, _ = scanned
    assert len(meta) > 400
    spill = {k: (m.get("private_segment_fixed_size", 0), m.get("vgpr_spill_count", 0))
             for k, m in meta.items() if m.get("private_segment_fixed_size", 0) or m.get("vgpr_spill_count", 0)}
    assert spill == {}, sorted(spill.items())[:5]
