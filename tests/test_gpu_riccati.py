"""GPU checks of the composition part: GEMM with transposed operands, the
fused LQR gain kernel and the unfused chain of library calls, each against
the FP64 oracle; info bit-exact on failing problems; the unfused chain
captured in a graph and replayed."""
import numpy as np
import pytest

import oracle
from helpers import TOL, normwise
from paper_2609_28179_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2609_28179_amd import glass
    return glass, torch


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("scope", ["wave", "workgroup"])
@pytest.mark.parametrize("m,n,k", [(3, 5, 7), (12, 4, 12), (4, 12, 16), (16, 16, 16), (33, 8, 20), (8, 48, 64),
                                   (64, 64, 64)])
def test_gemm_transposed_parity(env, scope, m, n, k):
    glass, torch = env
    rng = np.random.default_rng(m * 10000 + n * 100 + k)
    batch = 67
    for ta in (0, 1):
        for tb in (0, 1):
            A = rng.uniform(-1, 1, (batch, k, m) if ta else (batch, m, k)).astype(np.float32)
            B = rng.uniform(-1, 1, (batch, n, k) if tb else (batch, k, n)).astype(np.float32)
            C0 = rng.uniform(-1, 1, (batch, m, n)).astype(np.float32)
            for pack in (1, 2):
                for beta in (0.0, 0.5):
                    print(f"gemm_ex ta={ta} tb={tb} m={m} n={n} k={k} {scope}/P={pack} beta={beta}", flush=True)
                    C = dev(torch, C0)
                    st = glass.glass_gemm_batched_ex(ta, tb, m, n, k, batch, 1.5, dev(torch, A), dev(torch, B), beta,
                                                     C, (scope, pack))
                    assert st == 0, st
                    torch.cuda.synchronize()
                    ref = oracle.gemm_t(A, B, ta, tb, alpha=1.5, beta=beta, C=C0)
                    assert normwise(C.cpu().numpy(), ref).max() <= TOL


def test_gemm_transposed_rejects_thread_scope(env):
    glass, torch = env
    z = torch.zeros(4 * 8 * 8, device="cuda:0")
    assert glass.glass_gemm_batched_ex(1, 0, 8, 8, 8, 4, 1.0, z, z, 0.0, z, ("thread", 1)) == \
        glass.ERR_INFEASIBLE_PLACEMENT
    # the table's thread-scope entry falls back to wave scope for a transposed call
    rng = np.random.default_rng(3)
    A = rng.uniform(-1, 1, (4, 8, 8)).astype(np.float32)
    B = rng.uniform(-1, 1, (4, 8, 8)).astype(np.float32)
    C = torch.zeros((4, 8, 8), device="cuda:0")
    assert glass.glass_gemm_batched_ex(1, 1, 8, 8, 8, 4, 1.0, dev(torch, A), dev(torch, B), 0.0, C) == 0
    torch.cuda.synchronize()
    assert normwise(C.cpu().numpy(), oracle.gemm_t(A, B, 1, 1)).max() <= TOL


SIZES = [(1, 1), (4, 2), (7, 3), (12, 4), (14, 7), (20, 16), (32, 8), (33, 9), (48, 16), (56, 8)]


@pytest.mark.parametrize("nx,nu", SIZES)
def test_fused_gain_parity(env, nx, nu):
    glass, torch = env
    for batch in (1, 67, 1000):
        c = inputs.make_riccati(batch, nx, nu, seed=11)
        K_ref, info_ref = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
        assert (info_ref == 0).all()
        for pack in (1, 2, 4, 8):
            if glass.glass_riccati_feasible(nx, nu, pack) != 1:
                continue
            print(f"riccati fused nx={nx} nu={nu} batch={batch} P={pack}", flush=True)
            K = torch.full((batch, nu, nx), float("nan"), device="cuda:0")
            info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
            st = glass.glass_riccati_gain_batched(nx, nu, batch, dev(torch, c["A"]), dev(torch, c["B"]),
                                                  dev(torch, c["P"]), dev(torch, c["R"]), K, info,
                                                  ("wave", pack))
            assert st == 0, st
            torch.cuda.synchronize()
            assert np.array_equal(info.cpu().numpy(), info_ref)
            assert normwise(K.cpu().numpy(), K_ref).max() <= TOL


THREAD_SIZES = [(1, 1), (1, 4), (2, 3), (3, 1), (4, 2), (5, 3), (6, 4), (7, 2), (8, 1), (8, 4)]


SUBWAVE_SIZES = [(1, 1), (3, 2), (4, 2), (9, 1), (12, 4), (13, 5), (14, 7), (16, 1), (16, 8)]


@pytest.mark.parametrize("nx,nu", SUBWAVE_SIZES)
def test_fused_gain_subwave_parity(env, nx, nu):
    """The sub-wave form (four problems per wavefront) at every pack, with
    batches that leave partly filled wavefronts, NaN guard bands around K,
    and indefinite problems among healthy ones in the same wavefronts."""
    glass, torch = env
    assert glass.glass_riccati_placement_feasible(nx, nu, glass.SCOPES["subwave"], 1) == 1
    for batch in (1, 6, 67, 1000):
        c = inputs.make_riccati(batch, nx, nu, seed=18)
        bad = np.arange(1, batch, 5)
        c["R"][bad] = -50.0 * np.eye(nu, dtype=np.float32)
        K_ref, info_ref = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
        assert (info_ref[bad] != 0).all() and (np.delete(info_ref, bad) == 0).all()
        good = np.setdiff1d(np.arange(batch), bad)
        ops = {k: dev(torch, c[k]) for k in ("A", "B", "P", "R")}
        Kbuf = torch.full((batch * nu * nx + 8,), float("nan"), device="cuda:0")
        K = Kbuf[4:4 + batch * nu * nx]
        for pack in (1, 2, 4, 8):
            print(f"riccati fused subwave nx={nx} nu={nu} batch={batch} P={pack}", flush=True)
            K.fill_(float("nan"))
            info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
            st = glass.glass_riccati_gain_batched(nx, nu, batch, ops["A"], ops["B"], ops["P"], ops["R"], K, info,
                                                  ("subwave", pack))
            assert st == 0, st
            torch.cuda.synchronize()
            assert np.array_equal(info.cpu().numpy(), info_ref)
            Kh = K.cpu().numpy().reshape(batch, nu, nx)
            assert normwise(Kh[good], K_ref[good]).max() <= TOL
            assert np.isnan(Kh[bad]).all()  # K is not written where info is nonzero
            kb = Kbuf.cpu().numpy()
            assert np.isnan(kb[:4]).all() and np.isnan(kb[4 + batch * nu * nx:]).all()


@pytest.mark.parametrize("nx,nu", THREAD_SIZES)
def test_fused_gain_thread_parity(env, nx, nu):
    """The thread-scope form (one problem per lane), at every pack, on
    16-byte aligned operands and on operands one float off alignment (the
    4-byte access path), with batches that leave ragged workgroups."""
    glass, torch = env
    assert glass.glass_riccati_placement_feasible(nx, nu, glass.SCOPES["thread"], 1) == 1
    for batch in (1, 67, 1000):
        c = inputs.make_riccati(batch, nx, nu, seed=15)
        K_ref, info_ref = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
        assert (info_ref == 0).all()
        for shift in (0, 1):
            ops = {}
            for key in ("A", "B", "P", "R"):
                flat = np.ascontiguousarray(c[key]).reshape(-1)
                buf = torch.full((flat.size + 4,), float("nan"), device="cuda:0")
                buf[shift:shift + flat.size] = torch.from_numpy(flat).to("cuda:0")
                ops[key] = buf[shift:shift + flat.size]
            Kbuf = torch.full((batch * nu * nx + 8,), float("nan"), device="cuda:0")
            K = Kbuf[shift + 4:shift + 4 + batch * nu * nx]  # 16-byte aligned at shift 0
            for pack in (1, 2, 4, 8):
                print(f"riccati fused thread nx={nx} nu={nu} batch={batch} P={pack} shift={shift}", flush=True)
                K.fill_(float("nan"))
                info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
                st = glass.glass_riccati_gain_batched(nx, nu, batch, ops["A"], ops["B"], ops["P"], ops["R"], K, info,
                                                      ("thread", pack))
                assert st == 0, st
                torch.cuda.synchronize()
                assert np.array_equal(info.cpu().numpy(), info_ref)
                assert normwise(K.cpu().numpy().reshape(batch, nu, nx), K_ref).max() <= TOL
                kb = Kbuf.cpu().numpy()  # nothing written outside K
                assert np.isnan(kb[:shift + 4]).all() and np.isnan(kb[shift + 4 + batch * nu * nx:]).all()


def test_fused_default_placement_small_sizes(env):
    """force = NULL at sizes within the thread scope's range (its default there)."""
    glass, torch = env
    for nx, nu in ((1, 1), (4, 2), (8, 4)):
        batch = 333
        c = inputs.make_riccati(batch, nx, nu, seed=17)
        K_ref, info_ref = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
        print(f"riccati fused default nx={nx} nu={nu} batch={batch}", flush=True)
        K = torch.full((batch, nu, nx), float("nan"), device="cuda:0")
        info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
        assert glass.glass_riccati_gain_batched(nx, nu, batch, dev(torch, c["A"]), dev(torch, c["B"]),
                                                dev(torch, c["P"]), dev(torch, c["R"]), K, info) == 0
        torch.cuda.synchronize()
        assert np.array_equal(info.cpu().numpy(), info_ref)
        assert normwise(K.cpu().numpy(), K_ref).max() <= TOL


def test_fused_thread_info_on_indefinite_problems(env):
    glass, torch = env
    nx, nu, batch = 4, 2, 70
    c = inputs.make_riccati(batch, nx, nu, seed=16)
    bad = np.arange(3, batch, 5)
    c["R"][bad] = -50.0 * np.eye(nu, dtype=np.float32)   # S = R + B^T P B is then negative definite
    K_ref, info_ref = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
    assert (info_ref[bad] == 1).all() and (np.delete(info_ref, bad) == 0).all()
    K = torch.zeros((batch, nu, nx), device="cuda:0")
    info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
    assert glass.glass_riccati_gain_batched(nx, nu, batch, dev(torch, c["A"]), dev(torch, c["B"]),
                                            dev(torch, c["P"]), dev(torch, c["R"]), K, info, ("thread", 1)) == 0
    torch.cuda.synchronize()
    assert np.array_equal(info.cpu().numpy(), info_ref)
    good = np.setdiff1d(np.arange(batch), bad)
    assert normwise(K.cpu().numpy()[good], K_ref[good]).max() <= TOL
    assert (K.cpu().numpy()[bad] == 0).all()  # K is not written where info is nonzero


@pytest.mark.parametrize("nx,nu", SIZES)
def test_unfused_chain_parity(env, nx, nu):
    glass, torch = env
    from paper_2609_28179_amd import riccati
    batch = 300
    c = inputs.make_riccati(batch, nx, nu, seed=12)
    K_ref, _ = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
    print(f"riccati unfused nx={nx} nu={nu} batch={batch}", flush=True)
    K = torch.full((batch, nu, nx), float("nan"), device="cuda:0")
    info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
    ws = riccati.Workspace(torch, nx, nu, batch, "cuda:0")
    riccati.unfused(glass, dev(torch, c["A"]), dev(torch, c["B"]), dev(torch, c["P"]), dev(torch, c["R"]), K, ws,
                    info)
    torch.cuda.synchronize()
    assert (info.cpu().numpy() == 0).all()
    assert normwise(K.cpu().numpy(), K_ref).max() <= TOL


def test_fused_info_on_indefinite_problems(env):
    glass, torch = env
    nx, nu, batch = 12, 4, 40
    c = inputs.make_riccati(batch, nx, nu, seed=13)
    bad = np.arange(0, batch, 7)
    c["R"][bad] = -50.0 * np.eye(nu, dtype=np.float32)   # S = R + B^T P B is then negative definite
    K_ref, info_ref = oracle.riccati_gain(c["A"], c["B"], c["P"], c["R"])
    assert (info_ref[bad] == 1).all() and (np.delete(info_ref, bad) == 0).all()
    K = torch.zeros((batch, nu, nx), device="cuda:0")
    info = torch.full((batch,), -7, dtype=torch.int32, device="cuda:0")
    assert glass.glass_riccati_gain_batched(nx, nu, batch, dev(torch, c["A"]), dev(torch, c["B"]),
                                            dev(torch, c["P"]), dev(torch, c["R"]), K, info) == 0
    torch.cuda.synchronize()
    assert np.array_equal(info.cpu().numpy(), info_ref)
    good = np.setdiff1d(np.arange(batch), bad)
    assert normwise(K.cpu().numpy()[good], K_ref[good]).max() <= TOL


def test_graph_replays_of_both_forms(env):
    glass, torch = env
    from paper_2609_28179_amd import riccati
    nx, nu, batch = 14, 7, 500
    c = {k: dev(torch, v) for k, v in inputs.make_riccati(batch, nx, nu, seed=14).items()}
    ws = riccati.Workspace(torch, nx, nu, batch, "cuda:0")
    K_f = torch.empty((batch, nu, nx), device="cuda:0")
    K_u = torch.empty_like(K_f)
    riccati.fused(glass, c["A"], c["B"], c["P"], c["R"], K_f)
    riccati.unfused(glass, c["A"], c["B"], c["P"], c["R"], K_u, ws)
    torch.cuda.synchronize()
    ef, eu = K_f.clone(), K_u.clone()
    gf, gu = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
    with torch.cuda.graph(gf):
        riccati.fused(glass, c["A"], c["B"], c["P"], c["R"], K_f)
    with torch.cuda.graph(gu):
        riccati.unfused(glass, c["A"], c["B"], c["P"], c["R"], K_u, ws)
    for rep in range(3):
        K_f.fill_(float("nan"))
        K_u.fill_(float("nan"))
        ws.S.fill_(float("nan"))
        torch.cuda.synchronize()
        gf.replay()
        gu.replay()
        torch.cuda.synchronize()
        assert torch.equal(K_f, ef) and torch.equal(K_u, eu), rep


@pytest.mark.parametrize("scope,nx,nu", [("thread", 4, 2), ("subwave", 12, 4), ("subwave", 14, 7)])
def test_graph_replays_of_thread_and_subwave_forms(env, scope, nx, nu):
    """The thread and sub-wave forms captured in a graph: every replay, with
    the output wiped between them, equals the eager call bit for bit."""
    glass, torch = env
    from paper_2609_28179_amd import riccati
    batch = 501
    c = {k: dev(torch, v) for k, v in inputs.make_riccati(batch, nx, nu, seed=19).items()}
    K = torch.empty((batch, nu, nx), device="cuda:0")
    info = torch.empty((batch,), dtype=torch.int32, device="cuda:0")
    print(f"riccati graph {scope} nx={nx} nu={nu} batch={batch}", flush=True)
    riccati.fused(glass, c["A"], c["B"], c["P"], c["R"], K, info, pack=2, scope=scope)
    torch.cuda.synchronize()
    eK, ei = K.clone(), info.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        riccati.fused(glass, c["A"], c["B"], c["P"], c["R"], K, info, pack=2, scope=scope)
    for rep in range(3):
        K.fill_(float("nan"))
        info.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(K, eK) and torch.equal(info, ei), rep
    K_ref, _ = oracle.riccati_gain(*(c[k].cpu().numpy() for k in ("A", "B", "P", "R")))
    assert normwise(eK.cpu().numpy(), K_ref).max() <= TOL
