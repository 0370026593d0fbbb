"""Offline placement sweep and static-table emission (Sec. III-A: measure once
on the target GPU, store the choice in an architecture-specific table;
Sec. IV-A: paired randomized rounds, fresh inputs for destructive ops, raw
samples kept, a 5 % dispatch margin).

  python -m paper_2609_28179_amd.autotune sweep [--rounds 20] [--out FILE] [--cells table|heldout]
  python -m paper_2609_28179_amd.autotune emit  [--sweep FILE] [--out INC]
  python -m paper_2609_28179_amd.autotune summary [--sweep FILE]
  python -m paper_2609_28179_amd.autotune ragged [--out FILE]   (per-class ragged placement)
  python -m paper_2609_28179_amd.autotune emit-ragged [--sweep FILE] [--out INC]

The sweep covers the 300 cells {GEMM, GEMV, POTRF, POTRS, POSV, TRSV} x
n in {3,4,6,7,12,16,32,64} x batch in {1,16,256,1024,4096,65536} plus SE(3)
compose / inverse x batch, each at every feasible (scope, pack).  It appends
one JSON record per (cell, placement) and resumes by skipping cells already
complete, and only on the kernel sources it started on (the meta line
records their hash; emit stamps that hash and the sweep file's own into the
table's provenance).  The winner of a cell is the placement with the smallest median;
exact ties go to thread < wave < workgroup, then to the smaller pack.  The
placements within 5 % of the winner form the cell's margin set.
"""
from __future__ import annotations

import argparse
import datetime
import hashlib
import json
import os
import random
import sys

import numpy as np

from . import timing

PKG = os.path.dirname(os.path.abspath(__file__))
DEFAULT_SWEEP = os.path.join(PKG, "tuning", "sweep_gfx950.jsonl")
DEFAULT_INC = os.path.join(PKG, "csrc", "glass_table_gfx950.inc")
OP_ORDER = ("gemm", "gemv", "potrf", "potrs", "posv", "trsv", "se3_compose", "se3_inverse")
MARGIN = 1.05
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E spec peak


# Sources whose kernels a table measures: the batched ops' kernels, their
# device headers and the launch geometry (the host dispatch and the other
# parts' kernels do not change what a sweep times).
TABLE_SOURCES = ("glass_internal.hpp", "device_common.hpp", "chol.hip", "chol_device.hpp", "chol_blk.hip",
                 "chol_blk.hpp", "subwave.hip", "subwave_blas.hip", "gemm.hip", "gemv.hip", "se3.hip")
RAGGED_SOURCES = ("glass_internal.hpp", "device_common.hpp", "chol_device.hpp", "chol_blk.hpp", "ragged.hip")


def _code_only(text: str) -> str:
    """C/C++ source without its comments and with runs of whitespace folded,
    so that a hash over it changes with the code and not with the prose.
    String and character literals are kept whole (a // inside one is not a
    comment)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(kind: str = "table") -> str:
    """First 16 hex digits of a SHA-256 over the code of the sources a table
    is measured on (TABLE_SOURCES or RAGGED_SOURCES under csrc/, in that
    order, comments removed).  A sweep records it when it starts; emit stamps
    it into the table and refuses a sweep taken on other code."""
    h = hashlib.sha256()
    for f in TABLE_SOURCES if kind == "table" else RAGGED_SOURCES:
        h.update(f.encode() + b"\0")
        h.update(_code_only(open(os.path.join(PKG, "csrc", f)).read()).encode())
    return h.hexdigest()[:16]


def file_hash(path) -> str:
    """First 16 hex digits of the SHA-256 of a file's bytes."""
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def load(path):
    meta, recs = None, []
    if not os.path.exists(path):
        return meta, recs
    for line in open(path):
        line = line.strip()
        if not line:
            continue
        r = json.loads(line)
        if r.get("kind") == "meta":
            meta = r
        else:
            recs.append(r)
    return meta, recs


def sweep(args):
    import torch
    from . import glass

    dev = torch.device("cuda:0")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    meta, recs = load(args.out)
    src = source_hash()
    if meta is not None and meta.get("src") != src:
        raise SystemExit(f"{args.out} was started on sources {meta.get('src')}, these are {src}: "
                         "a sweep must measure one version of the kernels (start a new file)")
    done = {(r["op"], r["n"], r["batch"]) for r in recs}
    cells = timing.heldout_cells() if args.cells == "heldout" else timing.table_cells()
    if args.ops:
        cells = [c for c in cells if c[0] in args.ops.split(",")]
    if args.ns:
        cells = [c for c in cells if c[1] in [int(x) for x in args.ns.split(",")]]
    if args.max_batch:
        cells = [c for c in cells if c[2] <= args.max_batch]
    with open(args.out, "a") as f:
        if meta is None:
            p = torch.cuda.get_device_properties(0)
            meta = {"kind": "meta", "gpu": p.name, "arch": p.gcnArchName, "cus": p.multi_processor_count,
                    "torch": torch.__version__, "hip": torch.version.hip, "src": src,
                    "date": datetime.datetime.utcnow().isoformat(timespec="seconds"),
                    "floor_us": timing.floor_us(torch, dev), "copy_gbps": timing.copy_bandwidth(torch, dev),
                    "rounds": args.rounds, "rounds_below_65536": args.rounds_small,
                    "protocol": "graph of S launches per sample, S sets >= 1 GiB"}
            f.write(json.dumps(meta) + "\n")
            f.flush()
            print(f"floor {meta['floor_us']:.2f} us, copy {meta['copy_gbps']:.0f} GB/s", flush=True)
        rng = random.Random(args.seed)
        for ci, (op, n, batch) in enumerate(cells):
            if (op, n, batch) in done:
                continue
            pls = timing.feasible_placements(glass, op, n)
            cell = timing.Cell(torch, op, n, batch, dev, seed=1000 + ci)
            rounds = args.rounds if batch >= 65536 else args.rounds_small
            samples = timing.time_cell(glass, torch, cell, pls, rounds=rounds, warmup=args.warmup, rng=rng)
            ab = timing.alg_bytes(op, n) * batch
            best = None
            for (scope, pack), s in samples.items():
                med = float(np.median(s))
                rec = {"op": op, "n": n, "batch": batch, "scope": scope, "pack": pack, "nsets": cell.nsets,
                       "set_bytes": cell.set_bytes, "alg_bytes": ab, "median_us": med,
                       "p25_us": float(np.percentile(s, 25)), "p75_us": float(np.percentile(s, 75)),
                       "gbps": ab / (med * 1e-6) / 1e9, "samples_us": [round(v, 4) for v in s]}
                f.write(json.dumps(rec) + "\n")
                if best is None or med < best[0]:
                    best = (med, scope, pack)
            f.flush()
            print(f"[{ci + 1}/{len(cells)}] {op} n={n} batch={batch}: best {glass.SCOPE_NAMES[best[1]]}/P={best[2]} "
                  f"{best[0]:.2f} us ({ab / (best[0] * 1e-6) / 1e9:.0f} GB/s) over {len(pls)} placements",
                  flush=True)
            del cell
            torch.cuda.empty_cache()


def choose(recs):
    """Per cell: (winner (scope, pack), median, margin set, all medians)."""
    by_cell = {}
    for r in recs:
        by_cell.setdefault((r["op"], r["n"], r["batch"]), {})[(r["scope"], r["pack"])] = r["median_us"]
    out = {}
    for cell, meds in by_cell.items():
        order = sorted(meds.items(), key=lambda kv: (kv[1], kv[0][0], kv[0][1]))
        (win, wmed) = order[0]
        margin = sorted(pl for pl, m in meds.items() if m <= wmed * MARGIN)
        out[cell] = {"winner": win, "median_us": wmed, "margin": margin, "medians": meds}
    return out


def emit(args):
    meta, recs = load(args.sweep)
    if meta is None or (meta.get("src") != source_hash() and not args.allow_stale):
        raise SystemExit(f"{args.sweep} was measured on sources {meta and meta.get('src')}, the tree has "
                         f"{source_hash()}: re-sweep (or --allow-stale)")
    ch = choose(recs)
    nk, bk = timing.SWEEP_N, timing.TABLE_B
    lines = []
    missing = 0
    for op in OP_ORDER:
        rows = []
        for n in nk:
            ents = []
            for b in bk:
                key = (op, 4 if op.startswith("se3") else n, b)
                if key in ch:
                    s, p = ch[key]["winner"]
                else:
                    s, p = 1, 1
                    missing += 1
                ents.append("{%d, %d}" % (s, p))
            rows.append("{" + ", ".join(ents) + "}")
        lines.append("    {  // %s\n        " % op + ",\n        ".join(rows) + "}")
    prov = (f"gfx950 / {meta.get('gpu', '?')} / torch {meta.get('torch', '?')} hip {meta.get('hip', '?')} / "
            f"src {meta.get('src', '?')} / sweep {file_hash(args.sweep)} {meta.get('date', '?')} / {len(ch)} cells")
    text = (
        "// glass_table_gfx950.inc -- measured placement table for gfx950, generated by\n"
        "// paper_2609_28179_amd/autotune.py emit from the sweep records in\n"
        "// paper_2609_28179_amd/tuning/sweep_gfx950.jsonl.  Do not edit by hand.\n"
        "// Layout: kPlace[op][n_index][batch_index] = {scope, pack}; scope 0 thread,\n"
        "// 1 wave, 2 workgroup, 3 sub-wave.  The SE(3) rows repeat across n (n does\n"
        "// not apply).\n"
        f"static const char kTableProvenance[] = \"{prov}\";\n"
        f"static const int kTableN[{len(nk)}] = {{{', '.join(map(str, nk))}}};\n"
        f"static const int kTableB[{len(bk)}] = {{{', '.join(map(str, bk))}}};\n"
        f"static const unsigned char kPlace[8][{len(nk)}][{len(bk)}][2] = {{\n" + ",\n".join(lines) + "\n};\n")
    with open(args.out, "w") as f:
        f.write(text)
    print(f"wrote {args.out} ({len(ch)} measured cells, {missing} defaulted)")


def summary(args):
    meta, recs = load(args.sweep)
    ch = choose(recs)
    ratios, gaps, lines = [], [], []
    for (op, n, b), c in sorted(ch.items(), key=lambda kv: (OP_ORDER.index(kv[0][0]), kv[0][1], kv[0][2])):
        meds = c["medians"]
        fixed = meds.get((1, 1))
        worst = max(meds.values())
        ratios.append(fixed / c["median_us"])
        gaps.append(worst / c["median_us"])
        ab = timing.alg_bytes(op, n) * b
        # the attainable time is the larger of the HBM time at the spec peak
        # and the measured launch floor; the cell is bound by that one
        t_hbm = ab / (HBM_PEAK_GBPS * 1e3)
        floor = meta["floor_us"] if meta else 0.0
        bound = "HBM" if t_hbm >= floor else "launch"
        lines.append(f"| {op} | {n} | {b} | {'TWGS'[c['winner'][0]]}{c['winner'][1]} | {c['median_us']:.2f} | "
                     f"{fixed:.2f} | {fixed / c['median_us']:.2f} | {worst / c['median_us']:.1f} | "
                     f"{ab / (c['median_us'] * 1e-6) / 1e9:.0f} | {100 * t_hbm / c['median_us']:.1f} | "
                     f"{100 * max(t_hbm, floor) / c['median_us']:.0f} | {bound} | {len(c['margin'])} |")
    g = lambda v: float(np.exp(np.mean(np.log(v))))
    head = [f"floor {meta['floor_us']:.2f} us/launch, copy {meta['copy_gbps']:.0f} GB/s" if meta else "",
            f"cells {len(ch)}; tuned / fixed-wave(P=1) speedup: geomean {g(ratios):.2f}x, max {max(ratios):.1f}x; "
            f"best/worst placement gap: median {np.median(gaps):.1f}x, max {max(gaps):.1f}x",
            "",
            "Columns: % HBM = algorithmic bytes at the 8 TB/s spec peak over the tuned time; % attainable = "
            "max(that HBM time, launch floor) over the tuned time; bound = whichever of the two is larger.",
            "",
            "| op | n | batch | tuned | tuned us | wave/P1 us | speedup | worst/best | alg GB/s | % HBM | "
            "% attainable | bound | margin set |",
            "|---|---|---|---|---|---|---|---|---|---|---|---|---|"]
    text = "\n".join(head + lines) + "\n"
    if args.out:
        with open(args.out, "w") as f:
            f.write(text)
    print(text)


DEFAULT_RAGGED = os.path.join(PKG, "tuning", "ragged_gfx950.jsonl")
DEFAULT_RAGGED_INC = os.path.join(PKG, "csrc", "glass_ragged_gfx950.inc")
RAGGED_PER_SIZE = 5556   # problems per order: the density of the 50,000-system workload over nine orders


def ragged_options(k):
    """Placements a size class k (orders 8k+1 .. 8k+8) can take."""
    return ["wave"] + (["thread"] if k == 0 else []) + (["subwave"] if k <= 2 else [])


def ragged_class_sizes(k):
    from . import inputs
    sizes = [s for s in inputs.RAGGED_SIZES if (s - 1) // 8 == k]
    return sizes or [8 * k + 8]


def ragged_sweep(args):
    """Per size class: a ragged batch of that class's orders (nrhs 1-8), solved
    under every placement the class can take, in paired shuffled rounds of
    graph replays with the inputs restored between them."""
    import torch
    from . import glass, inputs
    rng = random.Random(args.seed)
    dev = torch.device("cuda:0")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    with open(args.out, "w") as f:
        p = torch.cuda.get_device_properties(0)
        f.write(json.dumps({"kind": "meta", "gpu": p.name, "arch": p.gcnArchName, "src": source_hash("ragged"),
                            "date": datetime.datetime.utcnow().isoformat(timespec="seconds"),
                            "per_size": RAGGED_PER_SIZE, "rounds": args.rounds}) + "\n")
        for k in range(8):
            sizes = ragged_class_sizes(k)
            case = inputs.make_ragged(RAGGED_PER_SIZE * len(sizes), seed=100 + k, sizes=sizes)
            rg = glass.Ragged(case, device=dev)
            A0, B0 = rg.A.clone(), rg.B.clone()
            graphs = {}
            for opt in ragged_options(k):
                scopes = ["wave"] * 8
                scopes[k] = opt
                rg.solve(class_scope=scopes)
                torch.cuda.synchronize()
                rg.A.copy_(A0)
                rg.B.copy_(B0)
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g):
                    rg.solve(class_scope=scopes)
                graphs[opt] = g
            samples = {o: [] for o in graphs}
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            order = list(graphs)
            for r in range(3 + args.rounds):
                rng.shuffle(order)
                for o in order:
                    rg.A.copy_(A0)
                    rg.B.copy_(B0)
                    e0.record()
                    graphs[o].replay()
                    e1.record()
                    e1.synchronize()
                    if r >= 3:
                        samples[o].append(e0.elapsed_time(e1) * 1e3)
            for o, v in samples.items():
                f.write(json.dumps({"class": k, "sizes": sizes, "count": len(case["n"]), "scope": o,
                                    "median_us": float(np.median(v)), "samples_us": [round(x, 3) for x in v]}) + "\n")
            f.flush()
            best = min(samples, key=lambda o: (np.median(samples[o]), ragged_options(k).index(o)))
            print(f"class {k} sizes {sizes}: " + ", ".join(f"{o} {np.median(v):.1f} us" for o, v in samples.items())
                  + f" -> {best}", flush=True)
            del graphs, rg
            torch.cuda.empty_cache()


def emit_ragged(args):
    from . import glass
    meta, recs = load(args.sweep)
    if meta is None or (meta.get("src") != source_hash("ragged") and not args.allow_stale):
        raise SystemExit(f"{args.sweep} was measured on sources {meta and meta.get('src')}, the tree has "
                         f"{source_hash('ragged')}: re-sweep (or --allow-stale)")
    codes = {"thread": glass.SCOPE_THREAD, "wave": glass.SCOPE_WAVE, "subwave": glass.SCOPE_SUBWAVE}
    win = []
    for k in range(8):
        cell = [r for r in recs if r["class"] == k]
        best = min(cell, key=lambda r: (r["median_us"], ragged_options(k).index(r["scope"])))
        win.append(codes[best["scope"]])
    prov = (f"gfx950 / {meta.get('gpu', '?')} / src {meta.get('src', '?')} / ragged sweep {file_hash(args.sweep)} "
            f"{meta.get('date', '?')}")
    text = ("// glass_ragged_gfx950.inc -- measured per-class placement of ragged batches on\n"
            "// gfx950, generated by paper_2609_28179_amd/autotune.py emit-ragged from\n"
            "// paper_2609_28179_amd/tuning/ragged_gfx950.jsonl.  Do not edit by hand.\n"
            "// kRaggedScope[k]: scope of size class k (orders 8k+1 .. 8k+8); 0 thread,\n"
            "// 1 wave, 3 sub-wave.\n"
            f"static const char kRaggedProvenance[] = \"{prov}\";\n"
            f"static const int kRaggedScope[8] = {{{', '.join(map(str, win))}}};\n")
    with open(args.out, "w") as f:
        f.write(text)
    print(f"wrote {args.out}: {win}")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("sweep")
    s.add_argument("--out", default=DEFAULT_SWEEP)
    s.add_argument("--rounds", type=int, default=20, help="paired rounds of the 65,536-problem cells")
    s.add_argument("--rounds-small", type=int, default=40,
                   help="paired rounds of the smaller cells (launch-bound cells time with more spread)")
    s.add_argument("--warmup", type=int, default=3)
    s.add_argument("--seed", type=int, default=0)
    s.add_argument("--ops", default="")
    s.add_argument("--ns", default="", help="comma-separated orders to sweep (default: all)")
    s.add_argument("--max-batch", type=int, default=0)
    s.add_argument("--cells", choices=("table", "heldout"), default="table",
                   help="table: the 250 cells of the dispatch table; heldout: n in {5,9,20,48} x "
                        "batch in {256,65536}, the cost model's evaluation set")
    e = sub.add_parser("emit")
    e.add_argument("--sweep", default=DEFAULT_SWEEP)
    e.add_argument("--out", default=DEFAULT_INC)
    e.add_argument("--allow-stale", action="store_true")
    m = sub.add_parser("summary")
    m.add_argument("--sweep", default=DEFAULT_SWEEP)
    m.add_argument("--out", default="")
    rs = sub.add_parser("ragged")
    rs.add_argument("--out", default=DEFAULT_RAGGED)
    rs.add_argument("--rounds", type=int, default=20)
    rs.add_argument("--seed", type=int, default=0)
    re_ = sub.add_parser("emit-ragged")
    re_.add_argument("--sweep", default=DEFAULT_RAGGED)
    re_.add_argument("--out", default=DEFAULT_RAGGED_INC)
    re_.add_argument("--allow-stale", action="store_true")
    args = ap.parse_args(argv)
    {"sweep": sweep, "emit": emit, "summary": summary, "ragged": ragged_sweep,
     "emit-ragged": emit_ragged}[args.cmd](args)


if __name__ == "__main__":
    sys.exit(main())
