"""GPU parity past 2^31 elements per operand: batches whose largest operand
holds 2^31 + 3 problems' worth of floats (8 GiB), so the last problems lie
beyond every 32-bit element or byte offset.  Each call runs at the library's
own table placement, one case per kernel family (the thread, sub-wave and
blocked wave Cholesky routines, the MFMA GEMM and the register GEMV); the
first, middle and last problems and a few more past the 2^31-element mark are
checked against the FP64 oracle, and info over the whole batch."""
import numpy as np
import pytest

import oracle
from helpers import TOL, normwise
from paper_2609_28179_amd import inputs

pytestmark = pytest.mark.gpu

ELEMS = 2 ** 31


def big_batch(n):
    return ELEMS // (n * n) + 3


# (op, n): the table's placements at these batches are thread scope for n = 4
# (SE(3): 4 x 4 transforms), sub-wave for n = 16 and the blocked / MFMA /
# register wave kernels for n = 64
CASES = [("gemm", 4), ("posv", 4), ("se3_compose", 4), ("potrf", 16), ("trsv", 16), ("gemm", 64), ("gemv", 64),
         ("posv", 64), ("potrs", 64)]


def sample_index(batch, n):
    past = ELEMS // (n * n)  # first problem that starts past 2^31 elements
    return np.unique(np.array([0, 1, batch // 2, past - 1, past, past + 1, batch - 2, batch - 1]))


@pytest.mark.parametrize("op,n", CASES, ids=[f"{o}-{n}" for o, n in CASES])
def test_past_2g_elements(op, n):
    import torch
    from paper_2609_28179_amd import glass
    dev = torch.device("cuda:0")
    batch = big_batch(n)
    pl = glass.glass_query_placement(glass.OPS[op], n, batch)
    print(f"{op} n={n} batch={batch} table {glass.SCOPE_NAMES[pl.scope]}/P={pl.pack}", flush=True)
    g = inputs.torch_generator(dev, 70_000 + n)
    chunk = max(16384, (1 << 24) // (n * n))
    idx = sample_index(batch, n)
    ti = torch.from_numpy(idx).to(dev)
    h = lambda t: t.index_select(0, ti).cpu().numpy()
    if op == "gemm":
        A = inputs.uniform_torch(g, (batch, n, n), dev)
        B = inputs.uniform_torch(g, (batch, n, n), dev)
        C = torch.full((batch, n, n), float("nan"), dtype=torch.float32, device=dev)  # beta = 0 never reads C
        assert glass.glass_gemm_batched(n, n, n, batch, 1.0, A, B, 0.0, C, None) == 0
        torch.cuda.synchronize()
        err = normwise(h(C), oracle.gemm(h(A), h(B)))
        del A, B, C
    elif op == "gemv":
        A = inputs.uniform_torch(g, (batch, n, n), dev)
        x = inputs.uniform_torch(g, (batch, n), dev)
        y = torch.full((batch, n), float("nan"), dtype=torch.float32, device=dev)
        assert glass.glass_gemv_batched(n, n, batch, 1.0, A, x, 0.0, y, None) == 0
        torch.cuda.synchronize()
        err = normwise(h(y), oracle.gemv(h(A), h(x)))
        del A, x, y
    elif op == "se3_compose":
        Ta = inputs.se3_torch(g, batch, dev)
        Tb = inputs.se3_torch(g, batch, dev)
        T = torch.full((batch, 4, 4), float("nan"), dtype=torch.float32, device=dev)
        assert glass.glass_se3_batched(glass.OP_SE3_COMPOSE, batch, Ta, Tb, T, None) == 0
        torch.cuda.synchronize()
        err = normwise(h(T), oracle.se3_compose(h(Ta), h(Tb)))
        row3 = T.index_select(0, ti)[:, 3, :]
        assert torch.equal(row3, torch.tensor([0.0, 0.0, 0.0, 1.0], device=dev).expand_as(row3))
        del Ta, Tb, T
    elif op in ("potrf", "posv"):
        A = inputs.spd_torch(g, batch, n, dev, chunk=chunk)
        A0 = h(A)
        info = torch.full((batch,), -7, dtype=torch.int32, device=dev)
        if op == "potrf":
            assert glass.glass_potrf_batched(n, batch, A, info, None) == 0
            torch.cuda.synchronize()
            L_ref, info_ref = oracle.potrf(A0)
            err = normwise(np.tril(h(A)), L_ref)
        else:
            B = inputs.uniform_torch(g, (batch, n, 1), dev)
            B0 = h(B)
            assert glass.glass_posv_batched(n, 1, batch, A, B, info, None) == 0
            torch.cuda.synchronize()
            L_ref, X_ref, info_ref = oracle.posv(A0, B0)
            err = np.maximum(normwise(np.tril(h(A)), L_ref), normwise(h(B), X_ref))
            del B
        assert (info_ref == 0).all()
        assert (info.cpu().numpy() == 0).all(), "info must be 0 for every problem"
        up = torch.triu(A.index_select(0, ti), 1)
        assert int(torch.count_nonzero(up)) == 0 and not bool(torch.signbit(up).any()), "strict upper must be +0"
        del A, info
    else:
        L = inputs.lower_factor_torch(g, batch, n, dev, chunk=chunk)
        if op == "potrs":
            B = inputs.uniform_torch(g, (batch, n, 1), dev)
            B0 = h(B)
            assert glass.glass_potrs_batched(n, 1, batch, L, B, None) == 0
            torch.cuda.synchronize()
            err = normwise(h(B), oracle.potrs(h(L), B0))
            del B
        else:
            x = inputs.uniform_torch(g, (batch, n), dev)
            x0 = h(x)
            assert glass.glass_trsv_batched(n, batch, 0, L, x, None) == 0
            torch.cuda.synchronize()
            err = normwise(h(x), oracle.trsv(h(L), x0, 0))
            del x
        del L
    torch.cuda.empty_cache()
    assert err.max() <= TOL, f"max normwise error {err.max():.3e} at problems {idx[err > TOL]}"


def test_adjoint_past_2g_elements():
    """The POSV adjoint at n = 12 with L and dA holding 2^31 + 3 problems'
    worth of floats (14.9 M problems), at the table's placement."""
    import torch
    from paper_2609_28179_amd import glass
    dev = torch.device("cuda:0")
    n = 12
    batch = big_batch(n)
    pl = glass.glass_query_placement(glass.OP_POSV_ADJOINT, n, batch)
    print(f"adjoint n={n} batch={batch} table {glass.SCOPE_NAMES[pl.scope]}/P={pl.pack}", flush=True)
    g = inputs.torch_generator(dev, 70_100)
    L = inputs.lower_factor_torch(g, batch, n, dev, chunk=(1 << 24) // (n * n))
    X = inputs.uniform_torch(g, (batch, n, 1), dev)
    G = inputs.uniform_torch(g, (batch, n, 1), dev)
    dB = torch.full((batch, n, 1), float("nan"), dtype=torch.float32, device=dev)
    dA = torch.full((batch, n, n), float("nan"), dtype=torch.float32, device=dev)
    assert glass.glass_posv_adjoint_batched(n, 1, batch, L, X, G, dB, dA, None) == 0
    torch.cuda.synchronize()
    idx = sample_index(batch, n)
    ti = torch.from_numpy(idx).to(dev)
    h = lambda t: t.index_select(0, ti).cpu().numpy()
    dB_ref, dA_ref = oracle.posv_adjoint(h(L), h(X), h(G))
    err = np.maximum(normwise(h(dB), dB_ref), normwise(h(dA), dA_ref))
    del L, X, G, dB, dA
    torch.cuda.empty_cache()
    assert err.max() <= TOL, f"max normwise error {err.max():.3e} at problems {idx[err > TOL]}"


def test_ragged_past_2g_elements():
    """The ragged solve with int64 problem offsets on both sides of 2^31
    elements: the second half of a mixed batch (thread / sub-wave / row and
    blocked wave classes) is moved up by 2^31 + 7 floats in A and 2^31 + 3 in
    B (odd shifts, so its problems also lose their 16-byte alignment)."""
    import torch
    from paper_2609_28179_amd import glass
    dev = torch.device("cuda:0")
    case = inputs.make_ragged(48, seed=9, sizes=(5, 12, 18, 24, 36, 64))
    half = len(case["n"]) // 2
    shA, shB = ELEMS + 7, ELEMS + 3
    offA = case["offA"].copy()
    offB = case["offB"].copy()
    offA[half:] += shA
    offB[half:] += shB
    print(f"ragged count={len(case['n'])} last offsets A {offA[-1]} B {offB[-1]}", flush=True)
    A = torch.zeros(int(case["A"].size) + shA, dtype=torch.float32, device=dev)
    B = torch.zeros(int(case["B"].size) + shB, dtype=torch.float32, device=dev)
    a0, b0 = int(case["offA"][half]), int(case["offB"][half])
    A[:a0] = torch.from_numpy(case["A"][:a0]).to(dev)
    A[a0 + shA:] = torch.from_numpy(case["A"][a0:]).to(dev)
    B[:b0] = torch.from_numpy(case["B"][:b0]).to(dev)
    B[b0 + shB:] = torch.from_numpy(case["B"][b0:]).to(dev)
    t = lambda a: torch.from_numpy(a).to(dev)
    info = torch.full((len(case["n"]),), -7, dtype=torch.int32, device=dev)
    ws_bytes = glass.glass_posv_ragged_workspace_size(len(case["n"]))
    ws = torch.empty((ws_bytes + 3) // 4, dtype=torch.int32, device=dev)
    assert glass.glass_posv_ragged(len(case["n"]), t(case["n"]), t(case["nrhs"]), t(offA), t(offB), A, B, info, ws,
                                   ws_bytes) == 0
    torch.cuda.synchronize()
    A_ref, B_ref, info_ref = oracle.posv_ragged(case["n"], case["nrhs"], case["offA"], case["offB"], case["A"],
                                                case["B"])
    assert np.array_equal(info.cpu().numpy(), info_ref)
    assert (info_ref == 0).all()
    for i in range(len(case["n"])):
        n, r = int(case["n"][i]), int(case["nrhs"][i])
        L = A[offA[i]:offA[i] + n * n].cpu().numpy().reshape(n, n)
        Lr = A_ref[case["offA"][i]:case["offA"][i] + n * n].reshape(n, n)
        X = B[offB[i]:offB[i] + n * r].cpu().numpy()
        Xr = B_ref[case["offB"][i]:case["offB"][i] + n * r]
        assert np.max(np.abs(L - Lr)) / np.max(np.abs(Lr)) <= TOL, (i, n, r)
        assert np.max(np.abs(X - Xr)) / max(np.max(np.abs(Xr)), 2.0 ** -126) <= TOL, (i, n, r)
        iu = np.triu_indices(n, 1)
        assert (L[iu] == 0).all() and not np.signbit(L[iu]).any(), (i, n)
    del A, B
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scope,nx,nu", [("thread", 4, 2), ("subwave", 16, 4), ("wave", 32, 8)])
def test_riccati_past_2g_elements(scope, nx, nu):
    """The fused LQR gain with P and A holding 2^31 + 3 problems' worth of
    floats, in each of its scopes (thread, sub-wave, and the matrix-core
    wavefront form): P = 2 I (exactly symmetric), R = I, A and B uniform, so
    S = I + 2 B^T B is positive definite; sampled problems against the oracle."""
    import torch
    from paper_2609_28179_amd import glass
    dev = torch.device("cuda:0")
    batch = big_batch(nx)
    print(f"riccati {scope} nx={nx} nu={nu} batch={batch}", flush=True)
    g = inputs.torch_generator(dev, 70_200 + nx)
    A = inputs.uniform_torch(g, (batch, nx, nx), dev)
    B = inputs.uniform_torch(g, (batch, nx, nu), dev) * 0.5
    P = torch.zeros((batch, nx, nx), dtype=torch.float32, device=dev)
    P.diagonal(dim1=1, dim2=2).fill_(2.0)
    R = torch.zeros((batch, nu, nu), dtype=torch.float32, device=dev)
    R.diagonal(dim1=1, dim2=2).fill_(1.0)
    K = torch.full((batch, nu, nx), float("nan"), dtype=torch.float32, device=dev)
    info = torch.full((batch,), -7, dtype=torch.int32, device=dev)
    assert glass.glass_riccati_gain_batched(nx, nu, batch, A, B, P, R, K, info, (scope, 1)) == 0
    torch.cuda.synchronize()
    info_h = info.cpu().numpy()
    badi = np.nonzero(info_h != 0)[0]
    assert badi.size == 0, (badi[:8], info_h[badi[:8]])
    idx = sample_index(batch, nx)
    ti = torch.from_numpy(idx).to(dev)
    h = lambda t: t.index_select(0, ti).cpu().numpy()
    K_ref, info_ref = oracle.riccati_gain(h(A), h(B), h(P), h(R))
    assert (info_ref == 0).all()
    err = normwise(h(K), K_ref)
    del A, B, P, R, K, info
    torch.cuda.empty_cache()
    assert err.max() <= TOL, f"max normwise error {err.max():.3e} at problems {idx[err > TOL]}"
