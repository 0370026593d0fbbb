"""Learned placement cost model.

The paper chooses a placement per (op, n, batch) by measuring every candidate
and storing the winner in a static table (Sec. III-A); a shape the table does
not hold takes the entry of the next larger tabulated order.  This module
adds a small regression model trained on the same measurements that proposes
placements for shapes nobody measured: it predicts the log run time of every
feasible placement, proposes the k fastest, and a short measured search over
those k (or over all feasible placements, the fallback) makes the final
choice.

Model: a 3-layer perceptron d -> 64 -> 64 -> 1 with ReLU, FP32, run by the
hand-written kernels behind glass_mlp_forward / glass_mlp_backward /
glass_mlp_adam.  Features (d = 15): one-hot op over the eight table ops, ln n
(ln 4 for SE(3)), ln batch, one-hot scope (thread, wave, workgroup,
sub-wave), log2 pack; each column standardised with the training set's mean and standard
deviation (columns with zero spread are left centred).  Target: ln of the
median microseconds per launch.  Loss: mean squared error over the whole
training set every step (full batch); Adam with lr 3e-3 for 5000 steps
(picked by leave-one-order-out cross-validation on the training sweep
before the held-out cells were measured), beta (0.9, 0.999), eps 1e-8;
He-normal initial weights from a fixed seed.

  python -m paper_2609_28179_amd.costmodel cv       [--sweep FILE] [--configs STEPS:LR,...]
  python -m paper_2609_28179_amd.costmodel train    [--sweep FILE] [--out PREFIX]
  python -m paper_2609_28179_amd.costmodel evaluate [--heldout FILE] [--model PREFIX] [--out JSON]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys

import numpy as np

from . import inputs, timing

PKG = os.path.dirname(os.path.abspath(__file__))
TUNING = os.path.join(PKG, "tuning")
DEFAULT_SWEEP = os.path.join(TUNING, "sweep_gfx950.jsonl")
DEFAULT_HELDOUT = os.path.join(TUNING, "heldout_gfx950.jsonl")
DEFAULT_MODEL = os.path.join(TUNING, "costmodel_gfx950")
DEFAULT_EVAL = os.path.join(TUNING, "costmodel_eval_gfx950.json")

FEATURE_OPS = ("gemm", "gemv", "potrf", "potrs", "posv", "trsv", "se3_compose", "se3_inverse")
D = 15
HIDDEN = 64
TOP_K = 3
STEPS = 5000
LR = 3e-3   # chosen by leave-one-order-out cross-validation on the training sweep
SEED = 0


def features(op: str, n: int, batch: int, scope: int, pack: int) -> np.ndarray:
    f = np.zeros(D)
    f[FEATURE_OPS.index(op)] = 1.0
    f[8] = np.log(4 if op.startswith("se3") else n)
    f[9] = np.log(batch)
    f[10 + scope] = 1.0
    f[14] = np.log2(pack)
    return f


def load_records(path):
    recs = []
    for line in open(path):
        line = line.strip()
        if line:
            r = json.loads(line)
            if r.get("kind") != "meta":
                recs.append(r)
    return recs


def dataset(recs):
    X = np.array([features(r["op"], r["n"], r["batch"], r["scope"], r["pack"]) for r in recs])
    t = np.log(np.array([r["median_us"] for r in recs]))
    return X, t


def _sha256(path):
    h = hashlib.sha256()
    with open(path, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


class CostModel:
    """Trained weights (flat FP32) plus the feature standardisation."""

    def __init__(self, params: np.ndarray, mu: np.ndarray, sd: np.ndarray, meta: dict | None = None):
        self.params = np.ascontiguousarray(params, dtype=np.float32)
        self.mu = np.asarray(mu, dtype=np.float64)
        self.sd = np.asarray(sd, dtype=np.float64)
        self.meta = meta or {}

    # --------------------------------------------------------------- inputs
    def standardise(self, X):
        return ((np.asarray(X, dtype=np.float64) - self.mu) / self.sd).astype(np.float32)

    # ------------------------------------------------------------- training
    @classmethod
    def train(cls, recs, steps=STEPS, lr=LR, seed=SEED, device="cuda:0", log_every=500, log=print):
        import torch
        from . import glass

        X, t = dataset(recs)
        mu = X.mean(0)
        sd = X.std(0)
        sd[sd == 0] = 1.0
        Z = torch.from_numpy(((X - mu) / sd).astype(np.float32)).to(device)
        T = torch.from_numpy(t.astype(np.float32)).to(device)
        N = Z.shape[0]
        P = glass.glass_mlp_num_params(D)
        p = torch.from_numpy(inputs.mlp_init(D, seed).astype(np.float32)).to(device)
        m = torch.zeros(P, dtype=torch.float32, device=device)
        v = torch.zeros_like(m)
        g = torch.empty_like(m)
        H1 = torch.empty((N, HIDDEN), dtype=torch.float32, device=device)
        H2 = torch.empty_like(H1)
        y = torch.empty(N, dtype=torch.float32, device=device)
        wsb = glass.glass_mlp_backward_workspace_size(N, D)
        ws = torch.empty((wsb + 3) // 4, dtype=torch.float32, device=device)
        history = []
        for step in range(1, steps + 1):
            _ok(glass.glass_mlp_forward(N, D, Z, p, H1, H2, y), "mlp_forward")
            if step == 1 or step % log_every == 0:
                mse = float(np.mean((y.cpu().numpy().astype(np.float64) - t) ** 2))
                history.append([step, mse])
                if log:
                    log(f"step {step}: mse {mse:.5f}")
            _ok(glass.glass_mlp_backward(N, D, Z, p, H1, H2, y, T, g, ws, wsb), "mlp_backward")
            _ok(glass.glass_mlp_adam(P, p, g, m, v, step, lr), "mlp_adam")
        _ok(glass.glass_mlp_forward(N, D, Z, p, H1, H2, y), "mlp_forward")
        mse = float(np.mean((y.cpu().numpy().astype(np.float64) - t) ** 2))
        history.append([steps + 1, mse])
        meta = {"d": D, "hidden": HIDDEN, "steps": steps, "lr": lr, "seed": seed, "samples": N,
                "final_mse": mse, "history": history,
                "features": "one-hot op (8), ln n, ln batch, one-hot scope (4), log2 pack; standardised",
                "target": "ln median us per launch"}
        return cls(p.cpu().numpy(), mu, sd, meta)

    # ------------------------------------------------------------ inference
    def predict_log_us(self, rows, device="cuda:0"):
        """Predicted ln(us) for rows of (op, n, batch, scope, pack), by the GPU forward kernel."""
        import torch
        from . import glass

        X = np.array([features(*r) for r in rows])
        Z = torch.from_numpy(self.standardise(X)).to(device)
        p = torch.from_numpy(self.params).to(device)
        y = torch.empty(len(rows), dtype=torch.float32, device=device)
        _ok(glass.glass_mlp_forward(len(rows), D, Z, p, None, None, y), "mlp_forward")
        return y.cpu().numpy()

    def rank(self, glass, op, n, batch, device="cuda:0"):
        """Feasible placements of (op, n, batch), fastest predicted first, with the predictions."""
        pls = timing.feasible_placements(glass, op, n)
        pred = self.predict_log_us([(op, n, batch, s, k) for (s, k) in pls], device)
        order = sorted(range(len(pls)), key=lambda i: (float(pred[i]), pls[i]))
        return [pls[i] for i in order], [float(pred[i]) for i in order]

    def propose(self, glass, op, n, batch, k=TOP_K, device="cuda:0"):
        return self.rank(glass, op, n, batch, device)[0][:k]

    # ------------------------------------------------------------------ I/O
    def save(self, prefix):
        self.params.tofile(prefix + ".f32")
        meta = dict(self.meta, mu=self.mu.tolist(), sd=self.sd.tolist(), n_params=int(self.params.size))
        with open(prefix + ".json", "w") as f:
            json.dump(meta, f, indent=1)

    @classmethod
    def load(cls, prefix=DEFAULT_MODEL):
        with open(prefix + ".json") as f:
            meta = json.load(f)
        params = np.fromfile(prefix + ".f32", dtype=np.float32)
        if params.size != meta["n_params"]:
            raise ValueError(f"{prefix}.f32 holds {params.size} floats, expected {meta['n_params']}")
        return cls(params, np.array(meta.pop("mu")), np.array(meta.pop("sd")), meta)


def _ok(st, what):
    if st != 0:
        from . import glass
        glass._raise(st, what)


def pick(model, glass, torch, op, n, batch, k=TOP_K, device="cuda:0", rounds=10):
    """Measured choice among the model's top-k proposals (all feasible
    placements when there is no model): returns (placement, median us)."""
    pls = model.propose(glass, op, n, batch, k, device) if model is not None else \
        timing.feasible_placements(glass, op, n)
    cell = timing.Cell(torch, op, n, batch, torch.device(device), seed=7)
    samples = timing.time_cell(glass, torch, cell, pls, rounds=rounds)
    meds = {pl: float(np.median(s)) for pl, s in samples.items()}
    best = min(meds, key=lambda pl: (meds[pl], pl))
    return best, meds[best]


# --------------------------------------------------------------- evaluation
def evaluate(model_ranks: dict, table_picks: dict, heldout_recs, k=TOP_K):
    """Score the model's proposals against exhaustive measurements.

    model_ranks[(op, n, batch)] = placements in predicted order;
    table_picks[(op, n, batch)] = the placement the static table dispatches
    (next larger tabulated order).  Returns per-cell rows and a summary."""
    meds = {}
    for r in heldout_recs:
        meds.setdefault((r["op"], r["n"], r["batch"]), {})[(r["scope"], r["pack"])] = r["median_us"]
    rows = []
    for cell in sorted(meds, key=lambda c: (FEATURE_OPS.index(c[0]), c[1], c[2])):
        m = meds[cell]
        best_pl = min(m, key=lambda pl: (m[pl], pl))
        best = m[best_pl]
        ranked = [tuple(pl) for pl in model_ranks[cell]]
        top = ranked[:k]
        top_best = min(m[pl] for pl in top)
        tab = tuple(table_picks[cell])
        rows.append({"op": cell[0], "n": cell[1], "batch": cell[2], "best": list(best_pl), "best_us": best,
                     "model_top": [list(pl) for pl in top], "top1_ratio": m[top[0]] / best,
                     "topk_ratio": top_best / best, "table": list(tab), "table_ratio": m[tab] / best,
                     "n_placements": len(m)})
    r1 = np.array([r["top1_ratio"] for r in rows])
    rk = np.array([r["topk_ratio"] for r in rows])
    rt = np.array([r["table_ratio"] for r in rows])
    gm = lambda v: float(np.exp(np.mean(np.log(v))))
    summary = {"cells": len(rows), "k": k,
               "topk_within_10pct": int(np.sum(rk <= 1.10)), "topk_max_ratio": float(rk.max()),
               "topk_geomean_ratio": gm(rk),
               "top1_within_10pct": int(np.sum(r1 <= 1.10)), "top1_max_ratio": float(r1.max()),
               "top1_geomean_ratio": gm(r1),
               "table_within_10pct": int(np.sum(rt <= 1.10)), "table_max_ratio": float(rt.max()),
               "table_geomean_ratio": gm(rt),
               "gain_top1_vs_table_geomean": gm(rt / r1), "gain_topk_vs_table_geomean": gm(rt / rk)}
    return rows, summary


def cross_validate(recs, configs, log=print):
    """Leave-one-order-out cross-validation on the training sweep only: for
    every tabulated n, train on the other orders and score the held-back
    cells by the best measured time among the model's top-k placements over
    the measured best.  Returns {(steps, lr): (frac within 10 %, geomean, max)}."""
    orders = sorted({r["n"] for r in recs if not r["op"].startswith("se3")})
    out = {}
    for steps, lr in configs:
        ratios = []
        for hold in orders:
            train_recs = [r for r in recs if r["n"] != hold or r["op"].startswith("se3")]
            model = CostModel.train(train_recs, steps=steps, lr=lr, log=None)
            cells = {}
            for r in recs:
                if r["n"] == hold and not r["op"].startswith("se3"):
                    cells.setdefault((r["op"], r["n"], r["batch"]), {})[(r["scope"], r["pack"])] = r["median_us"]
            rows = [(c, pl) for c, meds in cells.items() for pl in meds]
            pred = model.predict_log_us([(c[0], c[1], c[2], pl[0], pl[1]) for c, pl in rows])
            by = {}
            for (c, pl), y in zip(rows, pred):
                by.setdefault(c, []).append((float(y), pl))
            for c, lst in by.items():
                top = [pl for _, pl in sorted(lst)[:TOP_K]]
                meds = cells[c]
                ratios.append(min(meds[pl] for pl in top) / min(meds.values()))
        r = np.array(ratios)
        out[(steps, lr)] = (float(np.mean(r <= 1.10)), float(np.exp(np.mean(np.log(r)))), float(r.max()))
        if log:
            log(f"steps={steps} lr={lr}: top-{TOP_K} within 10 % {out[(steps, lr)][0]:.3f}, geomean "
                f"{out[(steps, lr)][1]:.4f}, max {out[(steps, lr)][2]:.3f} over {len(r)} cells")
    return out


def _cmd_cv(args):
    recs = load_records(args.sweep)
    configs = [(int(c.split(":")[0]), float(c.split(":")[1])) for c in args.configs.split(",")]
    res = cross_validate(recs, configs)
    best = max(res, key=lambda k: (res[k][0], -res[k][1]))
    print(f"chosen: steps={best[0]} lr={best[1]}")
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"sweep_sha256": _sha256(args.sweep), "k": TOP_K,
                       "results": [{"steps": k[0], "lr": k[1], "within_10pct": v[0], "geomean": v[1], "max": v[2]}
                                   for k, v in res.items()],
                       "chosen": {"steps": best[0], "lr": best[1]}}, f, indent=1)


def _cmd_train(args):
    recs = load_records(args.sweep)
    model = CostModel.train(recs, steps=args.steps, lr=args.lr, seed=args.seed)
    model.meta["sweep"] = os.path.basename(args.sweep)
    model.meta["sweep_sha256"] = _sha256(args.sweep)
    model.save(args.out)
    print(f"saved {args.out}.f32/.json (mse {model.meta['final_mse']:.5f} over {model.meta['samples']} samples)")


def _cmd_evaluate(args):
    from . import glass

    model = CostModel.load(args.model)
    recs = load_records(args.heldout)
    cells = sorted({(r["op"], r["n"], r["batch"]) for r in recs})
    ranks, preds, table = {}, {}, {}
    for (op, n, b) in cells:
        ranks[(op, n, b)], preds[(op, n, b)] = model.rank(glass, op, n, b)
        q = glass.glass_query_placement(glass.OPS[op], n, b)
        table[(op, n, b)] = (q.scope, q.pack)
    rows, summary = evaluate(ranks, table, recs)
    for r in rows:
        r["pred_log_us"] = preds[(r["op"], r["n"], r["batch"])]
    summary["model"] = os.path.basename(args.model)
    summary["heldout"] = os.path.basename(args.heldout)
    summary["heldout_sha256"] = _sha256(args.heldout)
    with open(args.out, "w") as f:
        json.dump({"summary": summary, "cells": rows}, f, indent=1)
    for r in rows:
        print(f"{r['op']:6s} n={r['n']:2d} B={r['batch']:5d}: best {r['best']} {r['best_us']:9.2f} us | "
              f"top1 {r['top1_ratio']:.3f} top{summary['k']} {r['topk_ratio']:.3f} | table {r['table']} "
              f"{r['table_ratio']:.3f}")
    print(json.dumps(summary, indent=1))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--sweep", default=DEFAULT_SWEEP)
    t.add_argument("--out", default=DEFAULT_MODEL)
    t.add_argument("--steps", type=int, default=STEPS)
    t.add_argument("--lr", type=float, default=LR)
    t.add_argument("--seed", type=int, default=SEED)
    c = sub.add_parser("cv")
    c.add_argument("--sweep", default=DEFAULT_SWEEP)
    c.add_argument("--configs", default="2000:1e-3,5000:1e-3,10000:1e-3,5000:3e-3")
    c.add_argument("--out", default="")
    e = sub.add_parser("evaluate")
    e.add_argument("--heldout", default=DEFAULT_HELDOUT)
    e.add_argument("--model", default=DEFAULT_MODEL)
    e.add_argument("--out", default=DEFAULT_EVAL)
    args = ap.parse_args(argv)
    {"cv": _cmd_cv, "train": _cmd_train, "evaluate": _cmd_evaluate}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
