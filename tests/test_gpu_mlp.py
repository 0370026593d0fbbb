"""GPU checks of the cost model's kernels: forward activations, the
deterministic backward pass and the Adam step against the FP64 reference, a
short training run step by step, and GPU inference of the committed weights."""
import os

import numpy as np
import pytest

from helpers import TOL
from oracle import mlp
from paper_2609_28179_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2609_28179_amd import glass
    return glass, torch


def rel(got, ref):
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 2.0 ** -126))


def case(N, d, seed):
    rng = np.random.default_rng(np.random.SeedSequence([seed, N, d]))
    X = rng.standard_normal((N, d)).astype(np.float32)
    t = rng.standard_normal(N).astype(np.float32)
    p = inputs.mlp_init(d, seed)
    # nonzero biases so the bias paths and both ReLU branches are exercised
    p[64 * d:64 * d + 64] = rng.uniform(-0.3, 0.3, 64)
    p[64 * d + 64 + 4096:64 * d + 128 + 4096] = rng.uniform(-0.3, 0.3, 64)
    p[-1] = 0.1
    return X, t, p.astype(np.float32)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def run_forward(glass, torch, X, p):
    N, d = X.shape
    H1 = torch.empty((N, 64), dtype=torch.float32, device="cuda:0")
    H2 = torch.empty_like(H1)
    y = torch.empty(N, dtype=torch.float32, device="cuda:0")
    Xd, pd = dev(torch, X), dev(torch, p)
    assert glass.glass_mlp_forward(N, d, Xd, pd, H1, H2, y) == 0
    return Xd, pd, H1, H2, y


@pytest.mark.parametrize("N,d", [(1, 14), (15, 14), (16, 14), (1000, 14), (33, 1), (77, 5), (301, 32)])
def test_forward_parity(env, N, d):
    glass, torch = env
    print(f"mlp forward N={N} d={d}", flush=True)
    X, _, p = case(N, d, 1)
    _, _, H1, H2, y = run_forward(glass, torch, X, p)
    torch.cuda.synchronize()
    h1, h2, yr = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert rel(H1.cpu().numpy(), h1) <= TOL
    assert rel(H2.cpu().numpy(), h2) <= TOL
    assert rel(y.cpu().numpy(), yr) <= TOL


@pytest.mark.parametrize("N,d", [(1, 14), (31, 14), (32, 14), (33, 14), (2436, 14), (100, 3), (257, 32)])
def test_backward_parity_and_determinism(env, N, d):
    glass, torch = env
    print(f"mlp backward N={N} d={d}", flush=True)
    X, t, p = case(N, d, 2)
    Xd, pd, H1, H2, y = run_forward(glass, torch, X, p)
    T = dev(torch, t)
    P = glass.glass_mlp_num_params(d)
    assert P == mlp.n_params(d)
    wsb = glass.glass_mlp_backward_workspace_size(N, d)
    ws = torch.full(((wsb + 3) // 4,), float("nan"), dtype=torch.float32, device="cuda:0")
    g1 = torch.full((P,), float("nan"), dtype=torch.float32, device="cuda:0")
    g2 = torch.full_like(g1, float("nan"))
    assert glass.glass_mlp_backward(N, d, Xd, pd, H1, H2, y, T, g1, ws, wsb) == 0
    assert glass.glass_mlp_backward(N, d, Xd, pd, H1, H2, y, T, g2, ws, wsb) == 0
    torch.cuda.synchronize()
    a, b = g1.cpu().numpy(), g2.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), "backward pass is not deterministic"
    ref = mlp.grad(p.astype(np.float64), X.astype(np.float64), t.astype(np.float64))
    assert rel(a, ref) <= TOL


def test_backward_rejects_small_workspace(env):
    glass, torch = env
    X, t, p = case(40, 14, 3)
    Xd, pd, H1, H2, y = run_forward(glass, torch, X, p)
    wsb = glass.glass_mlp_backward_workspace_size(40, 14)
    ws = torch.empty(wsb // 4, dtype=torch.float32, device="cuda:0")
    g = torch.empty(glass.glass_mlp_num_params(14), dtype=torch.float32, device="cuda:0")
    assert glass.glass_mlp_backward(40, 14, Xd, pd, H1, H2, y, dev(torch, t), g, ws, wsb - 4) == glass.ERR_INVALID_VALUE
    torch.cuda.synchronize()


@pytest.mark.parametrize("P,step", [(1, 1), (5185, 3), (70000, 1000)])
def test_adam_parity(env, P, step):
    glass, torch = env
    rng = np.random.default_rng(P + step)
    p = rng.standard_normal(P).astype(np.float32)
    g = rng.standard_normal(P).astype(np.float32)
    m = (0.1 * rng.standard_normal(P)).astype(np.float32)
    v = (0.01 * rng.random(P)).astype(np.float32)
    pd, gd, md, vd = dev(torch, p), dev(torch, g), dev(torch, m), dev(torch, v)
    assert glass.glass_mlp_adam(P, pd, gd, md, vd, step, 1e-3) == 0
    torch.cuda.synchronize()
    pr, mr, vr = mlp.adam_step(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                               v.astype(np.float64), step, lr=1e-3)
    assert rel(md.cpu().numpy(), mr) <= TOL
    assert rel(vd.cpu().numpy(), vr) <= TOL
    p1 = pd.cpu().numpy()
    assert rel(p1, pr) <= TOL
    # the update relative to its own size: the new parameter is rounded to
    # FP32, whose half ulp at |p| ~ 4 is 2.4e-7, about 1e-4 of a 2e-3 update
    assert rel(p1.astype(np.float64) - p, pr - p) <= 1e-3


def test_training_steps_follow_reference(env):
    """Ten full-batch training steps; every transition is checked against the
    reference applied to the GPU's own state before the step (so a rounding
    difference cannot grow through the trajectory), and the loss after ten
    steps against the reference's own ten-step run."""
    glass, torch = env
    N, d, steps = 500, 14, 10
    X, t, p = case(N, d, 4)
    X64, t64 = X.astype(np.float64), t.astype(np.float64)
    P = glass.glass_mlp_num_params(d)
    Xd, Td, pd = dev(torch, X), dev(torch, t), dev(torch, p)
    md = torch.zeros(P, dtype=torch.float32, device="cuda:0")
    vd = torch.zeros_like(md)
    gd = torch.empty_like(md)
    H1 = torch.empty((N, 64), dtype=torch.float32, device="cuda:0")
    H2 = torch.empty_like(H1)
    y = torch.empty(N, dtype=torch.float32, device="cuda:0")
    wsb = glass.glass_mlp_backward_workspace_size(N, d)
    ws = torch.empty((wsb + 3) // 4, dtype=torch.float32, device="cuda:0")
    for s in range(1, steps + 1):
        p0, m0, v0 = (a.cpu().numpy().astype(np.float64) for a in (pd, md, vd))
        assert glass.glass_mlp_forward(N, d, Xd, pd, H1, H2, y) == 0
        assert glass.glass_mlp_backward(N, d, Xd, pd, H1, H2, y, Td, gd, ws, wsb) == 0
        g = gd.cpu().numpy().astype(np.float64)
        assert rel(g, mlp.grad(p0, X64, t64)) <= TOL, s
        assert glass.glass_mlp_adam(P, pd, gd, md, vd, s, 1e-3) == 0
        pr, mr, vr = mlp.adam_step(p0, g, m0, v0, s, lr=1e-3)
        p1 = pd.cpu().numpy().astype(np.float64)
        assert rel(p1, pr) <= TOL, s
        assert rel(p1 - p0, pr - p0) <= 1e-3, s      # FP32 rounding of p (see test_adam_parity)
        assert rel(md.cpu().numpy(), mr) <= TOL and rel(vd.cpu().numpy(), vr) <= TOL, s
    pr, mr, vr = p.astype(np.float64), np.zeros(P), np.zeros(P)
    for s in range(1, steps + 1):
        pr, mr, vr = mlp.adam_step(pr, mlp.grad(pr, X64, t64), mr, vr, s, lr=1e-3)
    l_gpu = mlp.loss(pd.cpu().numpy().astype(np.float64), X64, t64)
    l_ref = mlp.loss(pr, X64, t64)
    assert l_gpu < mlp.loss(p.astype(np.float64), X64, t64)
    assert abs(l_gpu - l_ref) <= 1e-3 * l_ref


MODEL = os.path.join(os.path.dirname(__file__), "..", "paper_2609_28179_amd", "tuning", "costmodel_gfx950")


@pytest.mark.skipif(not os.path.exists(MODEL + ".f32"), reason="no trained model committed")
def test_committed_model_inference_matches_reference(env):
    glass, torch = env
    from paper_2609_28179_amd import costmodel, timing
    model = costmodel.CostModel.load(MODEL)
    rows = []
    for (op, n, b) in timing.heldout_cells():
        for (s, k) in timing.feasible_placements(glass, op, n):
            rows.append((op, n, b, s, k))
    got = model.predict_log_us(rows)
    Z = model.standardise(np.array([costmodel.features(*r) for r in rows]))
    _, _, ref = mlp.forward(model.params.astype(np.float64), Z.astype(np.float64))
    assert rel(got, ref) <= TOL
