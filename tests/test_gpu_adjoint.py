"""GPU checks of the differentiation part: the adjoint kernel against the FP64
oracle adjoint, central finite differences of the GPU forward solve, and the
autograd wrapper end to end."""
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


@pytest.mark.parametrize("scope", ["thread", "wave", "subwave"])
@pytest.mark.parametrize("n,r,batch", [(1, 1, 5), (6, 1, 67), (12, 1, 1100), (12, 3, 70), (16, 2, 130),
                                       (17, 1, 33), (33, 4, 65), (64, 1, 40), (64, 8, 9)])
def test_adjoint_parity(env, scope, n, r, batch):
    glass, torch = env
    if glass.glass_placement_feasible(glass.OP_POSV_ADJOINT, n, r, glass.SCOPES[scope], 1) != 1:
        pytest.skip("infeasible placement")
    print(f"adjoint n={n} nrhs={r} batch={batch} {scope}", flush=True)
    rng = inputs.rng_for(3, "adjoint", n, batch, r)
    A = inputs.spd(rng, batch, n)
    B = inputs.uniform(rng, (batch, n, r))
    W = rng.standard_normal(size=(batch, n, r)).astype(np.float32)
    L_ref, X_ref, info = oracle.posv(A, B)
    dB_ref, dA_ref = oracle.posv_adjoint(L_ref, X_ref, W)
    # the kernel consumes the float32 factor and solution of the GPU forward
    dev = "cuda:0"
    Lt = torch.from_numpy(A).to(dev)
    Xt = torch.from_numpy(B).to(dev)
    glass.posv_(Lt, Xt, force=("wave", 1))
    Gt = torch.from_numpy(W).to(dev)
    dB, dA = glass.posv_adjoint(Lt, Xt, Gt, force=(scope, 1))
    torch.cuda.synchronize()
    assert normwise(dB.cpu().numpy(), dB_ref).max() <= TOL
    assert normwise(dA.cpu().numpy(), dA_ref).max() <= TOL
    dAh = dA.cpu().numpy()
    assert np.array_equal(dAh, np.swapaxes(dAh, 1, 2))  # symmetric bit-exactly


def test_adjoint_config3_and_finite_differences(env):
    """16,384 systems, n = 12, FP32 (the differentiation workload): gradients
    match the FP64 reference, and central differences of the GPU forward agree
    with the GPU adjoint on sampled entries."""
    glass, torch = env
    from paper_2609_28179_amd.autograd import cholesky_solve
    n, batch = 12, 16384
    rng = inputs.rng_for(3, "adjoint", n, batch)
    A = inputs.spd(rng, batch, n)
    B = inputs.uniform(rng, (batch, n, 1))
    W = rng.standard_normal(size=(batch, n, 1)).astype(np.float32)
    dev = "cuda:0"
    At = torch.from_numpy(A).to(dev).requires_grad_(True)
    Bt = torch.from_numpy(B).to(dev).requires_grad_(True)
    Wt = torch.from_numpy(W).to(dev)
    X = cholesky_solve(At, Bt)
    (X * Wt).sum().backward()
    L_ref, X_ref, _ = oracle.posv(A, B)
    dB_ref, dA_ref = oracle.posv_adjoint(L_ref, X_ref, W)
    assert normwise(X.detach().cpu().numpy(), X_ref).max() <= TOL
    assert normwise(Bt.grad.cpu().numpy(), dB_ref).max() <= TOL
    assert normwise(At.grad.cpu().numpy(), dA_ref).max() <= TOL
    # central differences of the float32 GPU forward on a few sampled problems
    eps = 1e-2
    idx = [0, 777, 16383]

    def loss(Ap, Bp):
        with torch.no_grad():
            return (cholesky_solve(Ap, Bp) * Wt).sum(dim=(1, 2))

    gA = At.grad
    for q in idx:
        for (i, j) in [(0, 0), (5, 2), (11, 11), (7, 3)]:
            S = torch.zeros_like(At)
            S[q, i, j] = 1.0
            S[q, j, i] = 1.0
            fd = ((loss(At + eps * S, Bt) - loss(At - eps * S, Bt))[q] / (2 * eps)).item()
            an = (gA[q] * S[q]).sum().item()
            assert abs(fd - an) <= 1e-2 * max(1.0, abs(an)), (q, i, j, fd, an)


@pytest.mark.parametrize("n", [1, 3, 4, 5, 6, 7, 8, 12, 15, 16])
def test_adjoint_thread_direct_form_bit_identical(env, n):
    """One right-hand side at thread scope: aligned operands take the direct
    form (no LDS), operands one float off alignment the staged form; both
    must give the same dB and dA bit for bit, within the oracle's tolerance,
    and leave the guard floats around the outputs untouched."""
    glass, torch = env
    batch = 333
    rng = inputs.rng_for(5, "adjoint", n, batch, 1)
    A = inputs.spd(rng, batch, n)
    B = inputs.uniform(rng, (batch, n, 1))
    W = rng.standard_normal(size=(batch, n, 1)).astype(np.float32)
    L_ref, X_ref, _ = oracle.posv(A, B)
    dB_ref, dA_ref = oracle.posv_adjoint(L_ref, X_ref, W)
    Lt = torch.from_numpy(A).to("cuda:0")
    Xt = torch.from_numpy(B).to("cuda:0")
    glass.posv_(Lt, Xt, force=("wave", 1))
    torch.cuda.synchronize()
    out = {}
    for shift in (0, 1):
        print(f"adjoint thread direct n={n} shift={shift}", flush=True)
        ops = {}
        for key, t in (("L", Lt), ("X", Xt), ("G", torch.from_numpy(W).to("cuda:0"))):
            buf = torch.full((t.numel() + 8,), float("nan"), device="cuda:0")
            buf[4 + shift:4 + shift + t.numel()] = t.reshape(-1)
            ops[key] = buf[4 + shift:4 + shift + t.numel()]
        dBb = torch.full((batch * n + 8,), float("nan"), device="cuda:0")
        dAb = torch.full((batch * n * n + 8,), float("nan"), device="cuda:0")
        dB = dBb[4 + shift:4 + shift + batch * n]
        dA = dAb[4 + shift:4 + shift + batch * n * n]
        assert glass.glass_posv_adjoint_batched(n, 1, batch, ops["L"], ops["X"], ops["G"], dB, dA, ("thread", 1)) == 0
        torch.cuda.synchronize()
        for buf in (dBb, dAb):
            h = buf.cpu().numpy()
            assert np.isnan(h[:4 + shift]).all() and np.isnan(h[len(h) - 4 + shift:]).all()
        out[shift] = (dB.cpu().numpy().reshape(batch, n, 1), dA.cpu().numpy().reshape(batch, n, n))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert normwise(out[0][0], dB_ref).max() <= TOL
    assert normwise(out[0][1], dA_ref).max() <= TOL
    assert np.array_equal(out[0][1], np.swapaxes(out[0][1], 1, 2))
