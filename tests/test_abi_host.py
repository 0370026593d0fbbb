"""Host-side checks of the C-ABI that need no GPU: the library loads and
exports every function include/glass.h declares, argument validation returns
the documented status without touching the device, the advisor's lookup rule
matches an independent re-implementation over the shipped table, and the
feasibility rule has the documented shape."""
from __future__ import annotations

import os
import re

import pytest

import oracle.placement_ref as pref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glass.h")


@pytest.fixture(scope="module")
def glass():
    from paper_2609_28179_amd import glass as g
    return g


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(glass_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(glass):
    names = declared_functions()
    assert len(names) >= 11
    for name in names:
        assert hasattr(glass._lib, name), name
    assert set(names) == set(glass.EXPORTED)


FAKE = 0x10000  # never dereferenced: every call below fails validation first


def test_validation_paths(glass):
    g = glass
    S = 0  # explicit NULL stream: no torch stream lookup on a machine without GPU
    assert g.glass_posv_batched(0, 1, 4, FAKE, FAKE, None, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_posv_batched(65, 1, 4, FAKE, FAKE, None, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_posv_batched(6, 0, 4, FAKE, FAKE, None, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_posv_batched(6, 65, 4, FAKE, FAKE, None, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_posv_batched(6, 1, -1, FAKE, FAKE, None, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_posv_batched(6, 1, 0, None, None, None, stream=S) == g.OK
    assert g.glass_posv_batched(6, 1, 3, None, FAKE, None, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_potrf_batched(6, 3, None, None, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_potrs_batched(6, 1, 3, FAKE, None, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_trsv_batched(6, 3, 2, FAKE, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_trsv_batched(6, 3, 0, None, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_gemm_batched(6, 70, 6, 3, 1.0, FAKE, FAKE, 0.0, FAKE, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_gemm_batched(6, 6, 6, 3, 1.0, FAKE, None, 0.0, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_gemv_batched(6, 6, 3, 1.0, FAKE, FAKE, 0.0, None, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_se3_batched(g.OP_GEMM, 3, FAKE, FAKE, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_se3_batched(g.OP_SE3_COMPOSE, 3, FAKE, None, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_se3_batched(g.OP_SE3_INVERSE, 0, None, None, None, stream=S) == g.OK
    # forced placements: bad enum values are invalid, impossible ones infeasible
    assert g.glass_potrf_batched(6, 3, FAKE, None, force=(5, 1), stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_potrf_batched(6, 3, FAKE, None, force=("wave", 3), stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_potrf_batched(32, 3, FAKE, None, force=("thread", 1), stream=S) == g.ERR_INFEASIBLE_PLACEMENT
    assert g.glass_gemm_batched(4, 5, 4, 3, 1.0, FAKE, FAKE, 0.0, FAKE, force=("thread", 1), stream=S) \
        == g.ERR_INFEASIBLE_PLACEMENT
    for s in (0, -1, -2, -3, -4):
        assert g.status_string(s).startswith("GLASS_")


def test_riccati_and_gemm_ex_validation_paths(glass):
    g = glass
    S = 0
    assert g.glass_gemm_batched_ex(2, 0, 4, 4, 4, 3, 1.0, FAKE, FAKE, 0.0, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_gemm_batched_ex(0, -1, 4, 4, 4, 3, 1.0, FAKE, FAKE, 0.0, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_gemm_batched_ex(1, 0, 4, 65, 4, 3, 1.0, FAKE, FAKE, 0.0, FAKE, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_gemm_batched_ex(1, 0, 4, 4, 4, 3, 1.0, FAKE, FAKE, 0.0, FAKE, force=("thread", 1), stream=S) \
        == g.ERR_INFEASIBLE_PLACEMENT
    assert g.glass_gemm_batched_ex(1, 1, 4, 4, 4, 0, 1.0, None, None, 0.0, None, stream=S) == g.OK
    for nx, nu in ((0, 1), (1, 0), (57, 1), (8, 17), (49, 9), (50, 15)):
        assert g.glass_riccati_gain_batched(nx, nu, 3, FAKE, FAKE, FAKE, FAKE, FAKE, stream=S) == g.ERR_UNSUPPORTED
        assert g.glass_riccati_feasible(nx, nu, 1) == g.ERR_UNSUPPORTED
    assert g.glass_riccati_gain_batched(12, 4, -1, FAKE, FAKE, FAKE, FAKE, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_riccati_gain_batched(12, 4, 0, None, None, None, None, None, stream=S) == g.OK
    assert g.glass_riccati_gain_batched(12, 4, 3, FAKE, FAKE, None, FAKE, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_riccati_gain_batched(12, 4, 3, FAKE, FAKE, FAKE, FAKE, FAKE, force=("workgroup", 1),
                                        stream=S) == g.ERR_INFEASIBLE_PLACEMENT
    assert g.glass_riccati_feasible(12, 4, 3) == g.ERR_INVALID_VALUE
    assert g.glass_riccati_feasible(12, 4, 8) == 1
    # the matrix-core form (nx >= 9) stages one 16 x 20 block a wavefront and
    # the LDS-staged form (nx <= 8) at most 464 floats: every pack fits
    for nx, nu in ((48, 16), (56, 8), (8, 16), (1, 1)):
        assert all(g.glass_riccati_feasible(nx, nu, p) == 1 for p in (1, 2, 4, 8)), (nx, nu)
    # scope-aware feasibility: thread scope up to nx = 8, nu = 4; wavefront as
    # above; the other scopes never; bad scope / pack and sizes as documented
    T, W = g.SCOPES["thread"], g.SCOPES["wave"]
    for nx, nu in ((1, 1), (4, 2), (8, 4), (5, 3)):
        assert all(g.glass_riccati_placement_feasible(nx, nu, T, p) == 1 for p in (1, 2, 4, 8)), (nx, nu)
    for nx, nu in ((9, 1), (4, 5), (12, 4), (48, 16)):
        assert g.glass_riccati_placement_feasible(nx, nu, T, 1) == 0, (nx, nu)
        assert g.glass_riccati_gain_batched(nx, nu, 3, FAKE, FAKE, FAKE, FAKE, FAKE, force=("thread", 1),
                                            stream=S) == g.ERR_INFEASIBLE_PLACEMENT
    for nx, nu in ((12, 4), (4, 2), (56, 8)):
        for p in (1, 2, 4, 8):
            assert g.glass_riccati_placement_feasible(nx, nu, W, p) == g.glass_riccati_feasible(nx, nu, p)
        assert g.glass_riccati_placement_feasible(nx, nu, g.SCOPES["workgroup"], 1) == 0
    # sub-wave scope up to nx = 16, nu = 8
    SW = g.SCOPES["subwave"]
    for nx, nu in ((1, 1), (4, 2), (12, 4), (14, 7), (16, 8)):
        assert all(g.glass_riccati_placement_feasible(nx, nu, SW, p) == 1 for p in (1, 2, 4, 8)), (nx, nu)
    for nx, nu in ((17, 1), (8, 9), (32, 8), (56, 8)):
        assert g.glass_riccati_placement_feasible(nx, nu, SW, 1) == 0, (nx, nu)
        assert g.glass_riccati_gain_batched(nx, nu, 3, FAKE, FAKE, FAKE, FAKE, FAKE, force=("subwave", 1),
                                            stream=S) == g.ERR_INFEASIBLE_PLACEMENT
    assert g.glass_riccati_placement_feasible(4, 2, 17, 1) == g.ERR_INVALID_VALUE
    assert g.glass_riccati_placement_feasible(4, 2, T, 3) == g.ERR_INVALID_VALUE
    assert g.glass_riccati_placement_feasible(57, 1, T, 1) == g.ERR_UNSUPPORTED


def test_mlp_validation_paths(glass):
    g = glass
    S = 0
    assert g.glass_mlp_num_params(14) == 5185 and g.glass_mlp_num_params(0) == 0 and g.glass_mlp_num_params(33) == 0
    assert g.glass_mlp_backward_workspace_size(64, 14) == 2 * 5185 * 4
    assert g.glass_mlp_backward_workspace_size(65, 14) == 3 * 5185 * 4
    assert g.glass_mlp_forward(4, 0, FAKE, FAKE, None, None, FAKE, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_mlp_forward(4, 33, FAKE, FAKE, None, None, FAKE, stream=S) == g.ERR_UNSUPPORTED
    assert g.glass_mlp_forward(-1, 14, FAKE, FAKE, None, None, FAKE, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_mlp_forward(0, 14, None, None, None, None, None, stream=S) == g.OK
    assert g.glass_mlp_forward(4, 14, FAKE, None, None, None, FAKE, stream=S) == g.ERR_INVALID_VALUE
    ws = g.glass_mlp_backward_workspace_size(4, 14)
    assert g.glass_mlp_backward(0, 14, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, ws, stream=S) \
        == g.ERR_INVALID_VALUE
    assert g.glass_mlp_backward(4, 14, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, FAKE, ws - 4, stream=S) \
        == g.ERR_INVALID_VALUE
    assert g.glass_mlp_backward(4, 14, FAKE, FAKE, None, FAKE, FAKE, FAKE, FAKE, FAKE, ws, stream=S) \
        == g.ERR_INVALID_VALUE
    assert g.glass_mlp_adam(0, None, None, None, None, 1, 1e-3, stream=S) == g.OK
    assert g.glass_mlp_adam(8, FAKE, FAKE, FAKE, FAKE, 0, 1e-3, stream=S) == g.ERR_INVALID_VALUE
    assert g.glass_mlp_adam(8, FAKE, FAKE, None, FAKE, 1, 1e-3, stream=S) == g.ERR_INVALID_VALUE


def test_query_placement_matches_reference_lookup(glass):
    table = pref.load_table(os.path.join(ROOT, "paper_2609_28179_amd", "csrc", "glass_table_gfx950.inc"))
    batches = [1, 2, 3, 4, 5, 8, 15, 16, 17, 63, 64, 65, 255, 256, 257, 1000, 1024, 1025, 4095, 4096,
               4097, 16384, 16385, 30000, 65535, 65536, 65537, 1 << 20]
    for opname, op in glass.OPS.items():
        for n in range(1, 65):
            for b in batches:
                got = glass.glass_query_placement(op, n, b)
                scope, pack = pref.lookup(table, op, n, b)
                if glass.glass_placement_feasible(op, n, 1, scope, pack) != 1:
                    scope, pack = glass.SCOPE_WAVE, 1
                assert (got.scope, got.pack) == (scope, pack), (opname, n, b)
                per = {0: 64 * pack, 3: pack * (4 if n <= 16 else 2)}.get(scope, pack)
                assert got.problems_per_wg == per
    with pytest.raises(glass.GlassError):
        glass.glass_query_placement(glass.OP_POSV, 0, 16)
    with pytest.raises(glass.GlassError):
        glass.glass_query_placement(glass.OP_POSV, 8, 0)


def test_batch_key_rule_examples():
    keys = [1, 16, 256, 4096, 65536]
    # geometric midpoint of 16 and 256 is 64: ties go to the smaller key
    assert pref.batch_key(keys, 64) == 16
    assert pref.batch_key(keys, 65) == 256
    assert pref.batch_key(keys, 4) == 1
    assert pref.batch_key(keys, 5) == 16
    assert pref.batch_key(keys, 1 << 30) == 65536
    assert pref.n_key([3, 4, 6, 7, 12, 16, 32, 64], 1) == 3
    assert pref.n_key([3, 4, 6, 7, 12, 16, 32, 64], 13) == 16
    assert pref.n_key([3, 4, 6, 7, 12, 16, 32, 64], 33) == 64


def test_feasibility_rule_shape(glass):
    g = glass
    for op in ("potrf", "posv", "potrs", "trsv", "gemv"):
        assert g.glass_placement_feasible(g.OPS[op], 16, 1, g.SCOPE_THREAD, 1) == 1
        assert g.glass_placement_feasible(g.OPS[op], 17, 1, g.SCOPE_THREAD, 1) == 0
    assert g.glass_placement_feasible(g.OP_GEMM, 12, 1, g.SCOPE_THREAD, 1) == 1
    assert g.glass_placement_feasible(g.OP_GEMM, 13, 1, g.SCOPE_THREAD, 1) == 0
    for op in g.OPS.values():
        for n in range(1, 65):
            # the table fallback must always be runnable
            assert g.glass_placement_feasible(op, n, 1, g.SCOPE_WAVE, 1) == 1
            assert g.glass_placement_feasible(op, n, 64, g.SCOPE_WAVE, 1) == 1
            assert g.glass_placement_feasible(op, n, 1, g.SCOPE_WORKGROUP, 8) == 1
            # monotone in n: feasible at n implies feasible below n
            for scope in range(4):
                for pack in (1, 2, 4, 8):
                    if n > 1 and g.glass_placement_feasible(op, n, 1, scope, pack) == 1:
                        assert g.glass_placement_feasible(op, n - 1, 1, scope, pack) == 1


def test_subwave_feasibility(glass):
    g = glass
    for op in ("potrf", "posv", "potrs", "trsv"):
        for n in (1, 16, 17, 32):
            assert g.glass_placement_feasible(g.OPS[op], n, 1, g.SCOPE_SUBWAVE, 1) == 1
        assert g.glass_placement_feasible(g.OPS[op], 33, 1, g.SCOPE_SUBWAVE, 1) == 0
        # 2 problems x 32 x 36 floats per wavefront: 8 wavefronts exceed 64 KiB
        assert g.glass_placement_feasible(g.OPS[op], 32, 1, g.SCOPE_SUBWAVE, 4) == 1
        assert g.glass_placement_feasible(g.OPS[op], 32, 1, g.SCOPE_SUBWAVE, 8) == 0
        assert g.glass_placement_feasible(g.OPS[op], 16, 1, g.SCOPE_SUBWAVE, 8) == 1
    for op in ("gemm", "gemv"):
        assert g.glass_placement_feasible(g.OPS[op], 16, 1, g.SCOPE_SUBWAVE, 8) == 1
        assert g.glass_placement_feasible(g.OPS[op], 17, 1, g.SCOPE_SUBWAVE, 1) == 0
    for op in ("se3_compose", "se3_inverse"):
        assert g.glass_placement_feasible(g.OPS[op], 8, 1, g.SCOPE_SUBWAVE, 1) == 0
    assert g.glass_placement_feasible(g.OP_POSV_ADJOINT, 32, 1, g.SCOPE_SUBWAVE, 1) == 1
    assert g.glass_placement_feasible(g.OP_POSV_ADJOINT, 33, 1, g.SCOPE_SUBWAVE, 1) == 0
    assert g.glass_placement_feasible(g.OP_POSV, 8, 1, 4, 1) == g.ERR_INVALID_VALUE


def test_single_hip_runtime_in_process():
    """Importing the binding first must still leave one HIP runtime mapped:
    the library has to share torch's runtime (streams, allocations)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2609_28179_amd import glass\n"
            "import torch\n"
            "print(sorted({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))") % ROOT
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    libs = eval(out.stdout.strip().splitlines()[-1])
    assert len(libs) == 1, libs


def test_stream_probe_validation(glass):
    """The streaming probe rejects bad arguments on the host (no device call)."""
    F = 0x10000
    assert glass.glass_stream_probe(0, F, F, F, 0, 1, 0) == glass.OK
    assert glass.glass_stream_probe(4, F, F, F, 1024, 1, 0) == glass.ERR_INVALID_VALUE
    assert glass.glass_stream_probe(-1, F, F, F, 1024, 1, 0) == glass.ERR_INVALID_VALUE
    assert glass.glass_stream_probe(2, F + 4, F, F, 1024, 1, 0) == glass.ERR_INVALID_VALUE
    assert glass.glass_stream_probe(3, F, None, F, 1024, 1, 0) == glass.ERR_INVALID_VALUE
    assert glass.glass_stream_probe(1, None, None, None, 1024, 1, 0) == glass.ERR_INVALID_VALUE
    assert glass.glass_stream_probe(0, F, F, F, 63, 1, 0) == glass.ERR_INVALID_VALUE
    assert glass.glass_stream_probe(2, F, F, F, 1024, 0, 0) == glass.ERR_INVALID_VALUE
