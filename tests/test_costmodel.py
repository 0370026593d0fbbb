"""Host-side checks of the learned cost model: the feature encoding, the
evaluation rule on a hand-made case, and the committed model judged by the
committed held-out measurements (the picks recomputed here with the FP64
reference forward pass, so this runs without a GPU)."""
import json
import os

import numpy as np
import pytest

from oracle import mlp
from paper_2609_28179_amd import costmodel, timing


def test_feature_encoding():
    f = costmodel.features("posv", 12, 4096, 1, 4)
    assert f.shape == (15,)
    assert f[4] == 1 and f[:8].sum() == 1
    assert f[8] == pytest.approx(np.log(12)) and f[9] == pytest.approx(np.log(4096))
    assert f[11] == 1 and f[10:14].sum() == 1
    assert f[14] == 2
    s = costmodel.features("se3_inverse", 99, 1, 0, 1)
    assert s[7] == 1 and s[8] == pytest.approx(np.log(4)) and s[9] == 0 and s[10] == 1 and s[14] == 0
    w = costmodel.features("trsv", 20, 256, 3, 8)
    assert w[13] == 1 and w[10:14].sum() == 1 and w[14] == 3


def test_evaluation_rule():
    recs = [{"op": "gemv", "n": 5, "batch": 256, "scope": s, "pack": k, "median_us": us}
            for (s, k, us) in [(0, 1, 10.0), (1, 1, 12.0), (1, 2, 10.5), (2, 1, 30.0)]]
    ranks = {("gemv", 5, 256): [(2, 1), (1, 2), (1, 1), (0, 1)]}
    table = {("gemv", 5, 256): (1, 1)}
    rows, summ = costmodel.evaluate(ranks, table, recs, k=3)
    r = rows[0]
    assert r["best"] == [0, 1] and r["top1_ratio"] == pytest.approx(3.0)
    assert r["topk_ratio"] == pytest.approx(1.05) and r["table_ratio"] == pytest.approx(1.2)
    assert summ["topk_within_10pct"] == 1 and summ["top1_within_10pct"] == 0


HAVE = all(os.path.exists(p) for p in (costmodel.DEFAULT_MODEL + ".f32", costmodel.DEFAULT_HELDOUT,
                                       costmodel.DEFAULT_EVAL))


@pytest.mark.skipif(not HAVE, reason="no trained model / held-out sweep committed")
def test_committed_model_beats_the_table_rule_on_heldout_sizes():
    """The committed model's proposals for n in {5, 9, 20, 48} x batch in
    {256, 65536}, recomputed in FP64 from its weights, judged by exhaustive
    measurements that were not used to train it."""
    model = costmodel.CostModel.load(costmodel.DEFAULT_MODEL)
    recs = costmodel.load_records(costmodel.DEFAULT_HELDOUT)
    with open(costmodel.DEFAULT_EVAL) as f:
        saved = json.load(f)
    cells = {}
    for r in recs:
        cells.setdefault((r["op"], r["n"], r["batch"]), []).append((r["scope"], r["pack"]))
    assert set(cells) == set(timing.heldout_cells())
    ranks, table = {}, {}
    for row in saved["cells"]:
        key = (row["op"], row["n"], row["batch"])
        pls = sorted(cells[key])
        Z = model.standardise(np.array([costmodel.features(*key, s, k) for (s, k) in pls]))
        _, _, y = mlp.forward(model.params.astype(np.float64), Z.astype(np.float64))
        order = sorted(range(len(pls)), key=lambda i: (y[i], pls[i]))
        ranks[key] = [pls[i] for i in order]
        table[key] = tuple(row["table"])
        # the GPU's FP32 ranking agrees with the FP64 one on the proposals,
        # up to swaps of predictions closer than FP32 can separate
        gpu_top = [tuple(p) for p in row["model_top"]]
        pred = dict(zip(pls, y))
        for a, b in zip(gpu_top, ranks[key][:costmodel.TOP_K]):
            assert a == b or abs(pred[a] - pred[b]) <= 1e-4 * max(1.0, abs(pred[b])), (key, gpu_top, ranks[key])
    rows, summ = costmodel.evaluate(ranks, table, recs)
    print(json.dumps(summ, indent=1))
    assert summ["cells"] == 48
    # best of the top-3 within 10 % of the measured best on 47 of the 48
    # cells: it misses GEMM n=48 x 256 (1.23x, the best placement ranked
    # fourth); the table rule misses 9 of them, up to 1.75x
    missed = [(r["op"], r["n"], r["batch"]) for r in rows if r["topk_ratio"] > 1.10]
    assert summ["topk_within_10pct"] == 47 and missed == [("gemm", 48, 256)], missed
    assert summ["table_within_10pct"] == 39
    # what it gains over the table's next-larger-order rule: a better geometric
    # mean and a better worst case, at three measurements per shape
    assert summ["topk_geomean_ratio"] < summ["table_geomean_ratio"]
    assert summ["topk_max_ratio"] < summ["table_max_ratio"]
    assert summ["topk_within_10pct"] >= summ["table_within_10pct"]
