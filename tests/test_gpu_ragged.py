"""GPU checks of the ragged batch: every problem against the FP64 oracle,
info and the device-side class permutation bit-exact, under every class
placement, and the 50,000-problem workload on sampled problems plus its full
permutation."""
import numpy as np
import pytest

import oracle
from helpers import TOL
from paper_2609_28179_amd import inputs

pytestmark = pytest.mark.gpu


def per_problem_err(case, B_gpu, B_ref, idx):
    worst = 0.0
    for i in idx:
        n, r = int(case["n"][i]), int(case["nrhs"][i])
        s = slice(case["offB"][i], case["offB"][i] + n * r)
        ref = B_ref[s]
        worst = max(worst, np.max(np.abs(B_gpu[s] - ref)) / max(np.max(np.abs(ref)), 2.0 ** -126))
    return worst


@pytest.mark.parametrize("scopes", [None, ["wave"] * 8, ["thread"] + ["wave"] * 7,
                                    ["subwave", "subwave"] + ["wave"] * 6, ["thread", "subwave"] + ["wave"] * 6,
                                    ["subwave"] * 3 + ["wave"] * 5])
@pytest.mark.parametrize("count,seed", [(1, 3), (77, 4), (2500, 5)])
def test_ragged_parity(scopes, count, seed):
    import torch
    from paper_2609_28179_amd import glass
    sizes = (1, 2, 5, 6, 7, 8, 9, 12, 14, 16, 17, 18, 24, 31, 33, 36, 48, 57, 63, 64)
    case = inputs.make_ragged(count, seed=seed, sizes=sizes)
    print(f"ragged count={count} seed={seed} scopes={scopes}", flush=True)
    rg = glass.Ragged(case)
    rg.solve(class_scope=scopes)
    torch.cuda.synchronize()
    A_ref, B_ref, info_ref = oracle.posv_ragged(case["n"], case["nrhs"], case["offA"], case["offB"], case["A"],
                                                case["B"])
    assert np.array_equal(rg.info.cpu().numpy(), info_ref)
    assert np.array_equal(rg.perm().cpu().numpy(), oracle.ragged_order(case["n"]))
    Bg = rg.B.cpu().numpy()
    Ag = rg.A.cpu().numpy()
    assert per_problem_err(case, Bg, B_ref, range(count)) <= TOL
    for i in range(count):
        n = int(case["n"][i])
        L = Ag[case["offA"][i]:case["offA"][i] + n * n].reshape(n, n)
        Lr = A_ref[case["offA"][i]:case["offA"][i] + n * n].reshape(n, n)
        assert np.max(np.abs(L - Lr)) / np.max(np.abs(Lr)) <= TOL
        iu = np.triu_indices(n, 1)
        assert (L[iu] == 0).all() and not np.signbit(L[iu]).any()


def test_ragged_config2_sampled():
    """50,000 systems, n over {6,7,12,14,18,24,36,48,64}, 1-8 right-hand sides."""
    import torch
    from paper_2609_28179_amd import glass
    case = inputs.make_ragged(50000, seed=2)
    rg = glass.Ragged(case)
    rg.solve()
    torch.cuda.synchronize()
    assert np.array_equal(rg.perm().cpu().numpy(), oracle.ragged_order(case["n"]))
    info = rg.info.cpu().numpy()
    assert (info == 0).all()
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(50000, size=600, replace=False))
    sub = {k: v for k, v in case.items()}
    Bg = rg.B.cpu().numpy()
    # oracle on the sampled problems only
    n, r = case["n"][sample], case["nrhs"][sample]
    sa, sb = n.astype(np.int64) ** 2, n.astype(np.int64) * r
    oA = np.concatenate([[0], np.cumsum(sa)[:-1]])
    oB = np.concatenate([[0], np.cumsum(sb)[:-1]])
    A = np.concatenate([case["A"][case["offA"][i]:case["offA"][i] + case["n"][i] ** 2] for i in sample])
    B = np.concatenate([case["B"][case["offB"][i]:case["offB"][i] + case["n"][i] * case["nrhs"][i]] for i in sample])
    _, B_ref, info_ref = oracle.posv_ragged(n, r, oA, oB, A, B)
    assert (info_ref == 0).all()
    got = np.concatenate([Bg[case["offB"][i]:case["offB"][i] + case["n"][i] * case["nrhs"][i]] for i in sample])
    small = {"n": n, "nrhs": r, "offB": oB}
    assert per_problem_err(small, got, B_ref, range(len(sample))) <= TOL


def test_ragged_graph_replays_match_eager():
    """The ragged pipeline captured in a HIP graph: several replays, with
    eager work and synchronisations between them, each bit-identical to the
    eager result."""
    import torch
    from paper_2609_28179_amd import glass
    case = inputs.make_ragged(3000, seed=6)
    rg = glass.Ragged(case)
    A0, B0 = rg.A.clone(), rg.B.clone()
    rg.solve()
    torch.cuda.synchronize()
    A_e, B_e, info_e, perm_e = rg.A.clone(), rg.B.clone(), rg.info.clone(), rg.perm().clone()
    rg.A.copy_(A0)
    rg.B.copy_(B0)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rg.solve()
    for rep in range(3):
        rg.A.copy_(A0)
        rg.B.copy_(B0)
        rg.info.fill_(-7)
        rg.ws.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(rg.A, A_e) and torch.equal(rg.B, B_e), rep
        assert torch.equal(rg.info, info_e) and torch.equal(rg.perm(), perm_e), rep
