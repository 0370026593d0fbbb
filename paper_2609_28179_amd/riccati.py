"""LQR feedback gain K = (R + B^T P B)^{-1} B^T P A, fused and unfused.

Sec. III-B describes the gain as assembled either from the general matrix
and solve primitives or by a fused ``riccati_gain``; Sec. IV-E measures the
two and finds that the winner flips with the batch size, making composition
granularity one more measured placement.  Here:

  fused    one launch of glass_riccati_gain_batched, one problem per
           wavefront, every intermediate in VGPRs / LDS, pack P in
           {1, 2, 4, 8}: for nx >= 9 every product runs on the matrix
           cores in 16 x 16 tiles and S = R + B^T P B is factored as one
           diagonal tile; below, P and B are staged in LDS and the
           products read them as broadcasts;
  fused_subwave  the same launch at sub-wave scope (nx <= 16, nu <= 8):
           four problems per wavefront, one per 16-lane row, every
           cross-lane move a DPP exchange inside the row;
  fused_thread  the same launch at thread scope (nx <= 8, nu <= 4): one
           problem per lane, every operand and intermediate in VGPRs,
           64 P lanes per workgroup;
  unfused  the chain of library calls, each its own launch at the table's
           placement:  PB = P B (GEMM);  S = R (device copy);
           S += B^T PB (GEMM, transposed A);  PA = P A (GEMM);
           K = B^T PA (GEMM, transposed A);  K = S^{-1} K (POSV, nrhs = nx).

  python -m paper_2609_28179_amd.riccati sweep [--out FILE]
  python -m paper_2609_28179_amd.riccati summary [--sweep FILE]

The sweep times both forms over (nx, nu) x batch with HIP graphs of S
launches over rotating buffer sets of >= 1 GiB, in paired shuffled rounds, and
records the medians; ``choose`` reads the records back as the composition
advisor.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import random
import sys

import numpy as np

from . import inputs, timing

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_SWEEP = os.path.join(PKG, "tuning", "riccati_gfx950.jsonl")
SIZES = ((4, 2), (12, 4), (14, 7), (32, 8), (48, 16))
BATCHES = (16, 64, 256, 4096, 65536)
PACKS = (1, 2, 4, 8)


class Workspace:
    """Device buffers of the unfused chain for one (nx, nu, batch)."""

    def __init__(self, torch, nx, nu, batch, device):
        f = torch.float32
        self.PB = torch.empty((batch, nx, nu), dtype=f, device=device)
        self.PA = torch.empty((batch, nx, nx), dtype=f, device=device)
        self.S = torch.empty((batch, nu, nu), dtype=f, device=device)


def _ok(glass, st, what):
    if st != 0:
        glass._raise(st, what)


def fused(glass, A, B, P, R, K, info=None, pack=None, scope="wave"):
    b, nx, nu = B.shape
    force = None if pack is None else (glass.SCOPES[scope], pack)
    _ok(glass, glass.glass_riccati_gain_batched(nx, nu, b, A, B, P, R, K, info, force), "riccati_gain")


def unfused(glass, A, B, P, R, K, ws, info=None):
    b, nx, nu = B.shape
    _ok(glass, glass.glass_gemm_batched(nx, nu, nx, b, 1.0, P, B, 0.0, ws.PB), "gemm P B")
    ws.S.copy_(R)
    _ok(glass, glass.glass_gemm_batched_ex(1, 0, nu, nu, nx, b, 1.0, B, ws.PB, 1.0, ws.S), "gemm B^T PB")
    _ok(glass, glass.glass_gemm_batched(nx, nx, nx, b, 1.0, P, A, 0.0, ws.PA), "gemm P A")
    _ok(glass, glass.glass_gemm_batched_ex(1, 0, nu, nx, nx, b, 1.0, B, ws.PA, 0.0, K), "gemm B^T PA")
    _ok(glass, glass.glass_posv_batched(nu, nx, b, ws.S, K, info), "posv")


def alg_bytes(nx, nu):
    """Minimum bytes per problem: read A, B, P, R, write K."""
    return 4 * (2 * nx * nx + nx * nu + nu * nu + nu * nx)


def flops(nx, nu):
    return 2 * nx * nx * (nx + nu) + 2 * nu * nx * (nx + nu) + nu ** 3 / 3 + 2 * nu * nu * nx


def feasible_packs(glass, nx, nu, scope="wave"):
    return [p for p in PACKS if glass.glass_riccati_placement_feasible(nx, nu, glass.SCOPES[scope], p) == 1]


FUSED_SCOPE = {"fused": "wave", "fused_subwave": "subwave", "fused_thread": "thread"}


def time_forms(glass, torch, nx, nu, batch, rounds=20, warmup=3, rng=None, device="cuda:0"):
    """Median microseconds per call of every fused pack and of the unfused chain."""
    rng = rng or random.Random(0)
    dev = torch.device(device)
    g = inputs.torch_generator(dev, 7000 + nx * 100 + nu)
    base = inputs.riccati_torch(g, batch, nx, nu, dev)
    set_bytes = alg_bytes(nx, nu) * batch + 4 * batch * (nx * nu + nx * nx + nu * nu)
    nsets = int(min(64, max(2, math.ceil(timing.GIB / set_bytes))))
    sets = [base] + [{k: v.clone() for k, v in base.items()} for _ in range(nsets - 1)]
    for s in sets:
        s["K"] = torch.empty((batch, nu, nx), dtype=torch.float32, device=dev)
        s["ws"] = Workspace(torch, nx, nu, batch, dev)
    forms = [(f, p) for f, sc in FUSED_SCOPE.items() for p in feasible_packs(glass, nx, nu, sc)] + [("unfused", 0)]

    def run(form, s):
        if form[0] in FUSED_SCOPE:
            fused(glass, s["A"], s["B"], s["P"], s["R"], s["K"], None, form[1], FUSED_SCOPE[form[0]])
        else:
            unfused(glass, s["A"], s["B"], s["P"], s["R"], s["K"], s["ws"])

    graphs = {}
    for form in forms:
        run(form, sets[0])
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            for s in sets:
                run(form, s)
        graphs[form] = gr
    torch.cuda.synchronize()
    samples = {f: [] for f in forms}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    order = list(forms)
    for r in range(warmup + rounds):
        rng.shuffle(order)
        for f in order:
            e0.record()
            graphs[f].replay()
            e1.record()
            e1.synchronize()
            if r >= warmup:
                samples[f].append(e0.elapsed_time(e1) * 1e3 / nsets)
    del graphs
    return {f: float(np.median(v)) for f, v in samples.items()}, nsets


def sweep(args):
    import torch
    from . import glass
    rng = random.Random(args.seed)
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        for (nx, nu) in SIZES:
            for b in BATCHES:
                meds, nsets = time_forms(glass, torch, nx, nu, b, rounds=args.rounds, rng=rng)
                for (form, pack), us in sorted(meds.items()):
                    rec = {"nx": nx, "nu": nu, "batch": b, "form": form, "pack": pack, "median_us": us,
                           "nsets": nsets, "gbps": alg_bytes(nx, nu) * b / (us * 1e-6) / 1e9}
                    f.write(json.dumps(rec) + "\n")
                f.flush()
                fu = min(us for (fm, _), us in meds.items() if fm in FUSED_SCOPE)
                un = meds[("unfused", 0)]
                print(f"nx={nx} nu={nu} batch={b}: fused {fu:.2f} us, unfused {un:.2f} us "
                      f"({'fused' if fu <= un else 'unfused'} {max(fu, un) / min(fu, un):.2f}x)", flush=True)
                torch.cuda.empty_cache()


def load(path=DEFAULT_SWEEP):
    return [json.loads(l) for l in open(path) if l.strip()]


def choose(nx, nu, batch, recs=None):
    """Composition advisor: ("fused", pack), ("fused_subwave", pack), ("fused_thread", pack) or ("unfused", 0) from the
    measured records, at the nearest measured (nx, nu) (by order, then input
    count) and the nearest measured batch in log2 distance."""
    recs = recs if recs is not None else load()
    sizes = sorted({(r["nx"], r["nu"]) for r in recs})
    size = min(sizes, key=lambda s: (abs(s[0] - nx) + abs(s[1] - nu), s))
    bs = sorted({r["batch"] for r in recs if (r["nx"], r["nu"]) == size})
    bk = min(bs, key=lambda b: (abs(math.log2(b) - math.log2(max(batch, 1))), b))
    cell = [r for r in recs if (r["nx"], r["nu"]) == size and r["batch"] == bk]
    best = min(cell, key=lambda r: (r["median_us"], r["form"], r["pack"]))
    return best["form"], best["pack"]


def summary(args):
    recs = load(args.sweep)
    lines = ["| nx | nu | batch | fused best | fused us | unfused us | winner | ratio | fused alg GB/s |",
             "|---|---|---|---|---|---|---|---|---|"]
    for (nx, nu) in sorted({(r["nx"], r["nu"]) for r in recs}):
        for b in sorted({r["batch"] for r in recs if (r["nx"], r["nu"]) == (nx, nu)}):
            cell = [r for r in recs if (r["nx"], r["nu"], r["batch"]) == (nx, nu, b)]
            fu = min((r for r in cell if r["form"] in FUSED_SCOPE), key=lambda r: r["median_us"])
            un = [r for r in cell if r["form"] == "unfused"][0]
            win = "fused" if fu["median_us"] <= un["median_us"] else "unfused"
            ratio = max(fu["median_us"], un["median_us"]) / min(fu["median_us"], un["median_us"])
            lines.append(f"| {nx} | {nu} | {b} | {FUSED_SCOPE[fu['form']]} P={fu['pack']} | {fu['median_us']:.2f} | "
                         f"{un['median_us']:.2f} | "
                         f"{win} | {ratio:.2f}x | {fu['gbps']:.0f} |")
    text = "\n".join(lines) + "\n"
    if args.out:
        open(args.out, "w").write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--out", default=DEFAULT_SWEEP)
    s.add_argument("--rounds", type=int, default=20)
    s.add_argument("--seed", type=int, default=0)
    m = sub.add_parser("summary")
    m.add_argument("--sweep", default=DEFAULT_SWEEP)
    m.add_argument("--out", default="")
    a = ap.parse_args(argv)
    {"sweep": sweep, "summary": summary}[a.cmd](a)


if __name__ == "__main__":
    sys.exit(main())
