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


# (op, n): the table's placements at these batches are thread scope for n = 4,
# sub-wave for n = 16 and the blocked / MFMA / register wave kernels for n = 64
CASES = [("gemm", 4), ("posv", 4), ("potrf", 16), ("trsv", 16), ("gemm", 64), ("gemv", 64), ("posv", 64),
         ("potrs", 64)]


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
        assert int(info.abs().max()) == 0, "info must be 0 for every problem"
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
