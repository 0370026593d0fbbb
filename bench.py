#!/usr/bin/env python3
"""Benchmark: batched small dense linear algebra under the measured placement
table on one MI355X.

A step is one pass of the whole hot path over the placement-sweep workload:
every cell (op, n, batch) of the grid {GEMM, GEMV, POTRF, POTRS, POSV, TRSV}
x n in {3,4,6,7,12,16,32,64} x batch in {1,16,256,4096,65536} plus SE(3)
compose / inverse x batch (250 calls, 3,495,250 problems), each dispatched
through the C-ABI with the built-in table (the bare call).  Inputs are
synthetic, seeded, drawn on the device and resident in HBM before timing;
every step gets its own copy of the destructive ops' inputs, so each
factorization / solve sees a fresh valid input.  A step is captured as HIP
graphs; the largest kernel of the step is launched between two events so its
duration is measured live inside the timed region (roofline).  The same step
with every call forced to wavefront scope, pack 1 (the fixed placement) is
timed the same way.  The FP64 CPU oracle is timed on a bounded sample of the
same workload on the host cores (cpu_baseline).

Prints one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s & % roofline, batched n=6–64 Cholesky/GEMM; tuned vs fixed placement"
HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(cells, sets, shared, sample_cap, min_seconds, torch):
    """Time the FP64 oracle on up to `sample_cap` problems of every cell,
    repeating the pass over the cells until at least `min_seconds` of oracle
    time have accumulated."""
    import oracle

    host, sampled, total = [], 0, 0
    for (op, n, batch) in cells:
        m = min(batch, sample_cap)
        src = dict(shared[(op, n, batch)])
        src.update(sets[0].get((op, n, batch), {}))
        host.append((op, batch, m, {k: v[:m].detach().cpu().numpy() for k, v in src.items()
                                    if v.dtype == torch.float32}))
        sampled += m
        total += batch
    calls = {"gemm": lambda h: oracle.gemm(h["A"], h["B"]), "gemv": lambda h: oracle.gemv(h["A"], h["x"]),
             "potrf": lambda h: oracle.potrf(h["A"]), "posv": lambda h: oracle.posv(h["A"], h["B"]),
             "potrs": lambda h: oracle.potrs(h["L"], h["B"]), "trsv": lambda h: oracle.trsv(h["L"], h["x"], 0),
             "se3_compose": lambda h: oracle.se3_compose(h["Ta"], h["Tb"]),
             "se3_inverse": lambda h: oracle.se3_inverse(h["Ta"])}
    t_est, spent, passes = 0.0, 0.0, 0
    while passes == 0 or spent < min_seconds:
        for op, batch, m, h in host:
            t0 = time.perf_counter()
            calls[op](h)
            dt = time.perf_counter() - t0
            spent += dt
            t_est += dt * batch / m
        passes += 1
    t_est /= passes
    scope = "every problem of the step" if sampled == total else \
        f"the first min(batch, {sample_cap}) problems of each cell, time scaled to the full batch"
    # the same oracle on one thread, over the first min(batch, 1024) problems
    # of each cell, time scaled to the full batch
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        t_one, spent_one = 0.0, 0.0
        for op, batch, m, h in host:
            m1 = min(m, 1024)
            t0 = time.perf_counter()
            calls[op]({k: v[:m1] for k, v in h.items()})
            dt = time.perf_counter() - t0
            spent_one += dt
            t_one += dt * batch / m1
    finally:
        oracle.set_num_threads(threads)
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": total / t_est, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 C oracle (OpenMP) on {scope} ({len(cells)} cells, {sampled} of {total} problems), "
                      f"{passes} passes, {spent:.1f} s of oracle time; {t_est:.2f} s per full step",
            "single_thread_value": total / t_one,
            "single_thread_sample": f"one thread, first min(batch, 1024) problems of each cell, {spent_one:.1f} s",
            "host_cpu": cpu_model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fixed", action="store_true", help="skip the fixed-placement comparator")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the small-POSV, ragged and adjoint workload timings")
    ap.add_argument("--cpu-sample", type=int, default=65536,
                    help="problems per cell the CPU oracle runs (65536: the whole step)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the oracle pass until this much CPU time has accumulated")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the batched problems are independent and this build "
              "measures one GPU's share; multi-GPU runs are not supported.", file=sys.stderr)
        return 2

    import numpy as np
    import torch
    from paper_2609_28179_amd import glass, timing

    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    cells = timing.sweep_cells()
    destructive = timing.DESTRUCTIVE

    # ---------------------------------------------------------------- inputs
    t0 = time.time()
    shared, sets, pristine = {}, [dict() for _ in range(K)], {}
    for ci, (op, n, batch) in enumerate(cells):
        base = timing.make_set(torch, op, n, batch, dev, seed=50_000 + ci)
        dnames = destructive.get(op, ())
        shared[(op, n, batch)] = {k: v for k, v in base.items() if k not in dnames}
        if dnames:
            pristine[(op, n, batch)] = {k: base[k] for k in dnames}
            for k in range(K):
                sets[k][(op, n, batch)] = {d: base[d].clone() for d in dnames}
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f} s; {len(cells)} cells, "
        f"{sum(b for _, _, b in cells)} problems per step, {torch.cuda.memory_allocated() / 2**30:.1f} GiB")

    def bufs(k, cell):
        d = dict(shared[cell])
        d.update(sets[k].get(cell, {}))
        return d

    def restore():
        for k in range(K):
            for cell, d in sets[k].items():
                for name, t in d.items():
                    t.copy_(pristine[cell][name])

    def call(k, cell, force):
        op, n, batch = cell
        st = timing.launch(glass, op, n, batch, bufs(k, cell), force)
        if st != 0:
            raise RuntimeError(f"{cell}: {glass.status_string(st)}")

    # ------------------------------------------ dominant cell (largest kernel)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * len(cells))]
    for cell in cells:  # first eager pass loads every code object
        call(0, cell, None)
    torch.cuda.synchronize()
    restore()
    for i, cell in enumerate(cells):
        ev[2 * i].record()
        call(0, cell, None)
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    restore()
    durs = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(len(cells))]
    dom_i = int(np.argmax(durs))
    dom = cells[dom_i]
    log(f"dominant cell {dom} ~{durs[dom_i] * 1e3:.1f} us of ~{sum(durs) * 1e3:.0f} us eager")

    def capture(force):
        pre, post = [], []
        for k in range(K):
            g1, g2 = torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph()
            with torch.cuda.graph(g1):
                for cell in cells[:dom_i]:
                    call(k, cell, force)
            with torch.cuda.graph(g2):
                for cell in cells[dom_i + 1:]:
                    call(k, cell, force)
            pre.append(g1)
            post.append(g2)
        return pre, post

    def run(force, label):
        pre, post = capture(force)
        torch.cuda.synchronize()
        for w in range(W):
            k = w % K
            pre[k].replay()
            call(k, dom, force)
            post[k].replay()
        torch.cuda.synchronize()
        restore()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for k in range(K):
            pre[k].replay()
            evs[k][0].record()
            call(k, dom, force)
            evs[k][1].record()
            post[k].replay()
        end.record()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end) / K
        dom_us = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e3
        restore()
        torch.cuda.synchronize()
        log(f"{label}: {ms:.3f} ms/step, dominant kernel {dom_us:.1f} us")
        del pre, post
        return ms, dom_us

    ms, dom_us = run(None, "tuned (table)")
    fixed = None
    if not args.no_fixed:
        fms, fdom = run(glass.Placement(glass.SCOPE_WAVE, 1, 0, 0), "fixed wave/P=1")
        fixed = {"ms_per_step": round(fms, 4), "value": sum(b for _, _, b in cells) / (fms * 1e-3),
                 "tuned_speedup": round(fms / ms, 3)}

    problems = sum(b for _, _, b in cells)
    value = problems / (ms * 1e-3)
    op, n, batch = dom
    dom_bytes = timing.alg_bytes(op, n) * batch
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    pl = glass.glass_query_placement(glass.OPS[op], n, batch)
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        t = json.load(open(tpath))
        from paper_2609_28179_amd.traffic import kernel_source_hash
        if tuple(t.get("cell", ())) == tuple(dom) and t.get("source_hash") == kernel_source_hash(dom[0]):
            traffic = t.get("bytes_per_launch")
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": f"{op} n={n} batch={batch} at {glass.SCOPE_NAMES[pl.scope]}/P={pl.pack}",
                "alg_bytes_per_launch": dom_bytes, "avg_launch_us": round(dom_us, 2)}

    extras = None
    if not args.no_extras:
        from paper_2609_28179_amd import workloads
        t0 = time.time()
        extras = {"posv_small": workloads.posv_small(glass, torch),
                  "ragged": workloads.ragged(glass, torch),
                  "adjoint": workloads.adjoint(glass, torch),
                  "riccati_gain": workloads.riccati_gain(glass, torch),
                  "batch1_latency": workloads.batch1_latency(glass, torch)}
        log(f"workloads ({time.time() - t0:.1f} s): " + json.dumps(extras))

    cpu = None
    if not args.no_cpu:
        t0 = time.time()
        cpu = cpu_baseline(cells, sets, shared, args.cpu_sample, args.cpu_seconds, torch)
        log(f"cpu baseline {cpu['value']:.3e} solves/s with {cpu['cores']} threads ({time.time() - t0:.1f} s)")

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "solves/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "placement-sweep grid: {gemm,gemv,potrf,potrs,posv,trsv} x n{3,4,6,7,12,16,32,64} "
                               "x batch{1,16,256,4096,65536} + se3 compose/inverse x batch; 250 calls, "
                               f"{problems} problems per step, FP32, uniform[-1,1] / SPD M M^T + nI / "
                               "Cholesky-factor triangles / random rigid transforms",
                   "placement": "built-in gfx950 table", "table": glass.glass_table_provenance()},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fixed_placement": fixed,
        "workloads": extras,
    }
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
