"""Timings of the workloads beside the placement-sweep step: the plain small
POSV, the ragged batch against per-size launches, the Cholesky-solve
adjoint, the LQR gain, and single-problem latency.  Each returns a small
dict for the benchmark's JSON line.

All timings but the single-problem latency are device-side: HIP graphs
replayed between two events, inputs resident in HBM, destructive inputs
restored from a pristine copy outside the events.
"""
from __future__ import annotations

import numpy as np

from . import inputs, timing


def _median_us(samples):
    return float(np.median(samples))


def posv_small(glass, torch, n=6, batch=1024, rounds=20):
    """POSV n x n, one right-hand side, `batch` systems: microseconds per
    launch at the fixed wavefront placement (one system per 64-lane
    workgroup) and at the table's placement."""
    dev = torch.device("cuda:0")
    table = glass.glass_query_placement(glass.OP_POSV, n, batch)
    pls = [(glass.SCOPE_WAVE, 1)]
    if (table.scope, table.pack) != pls[0]:
        pls.append((table.scope, table.pack))
    cell = timing.Cell(torch, "posv", n, batch, dev, seed=0)
    s = timing.time_cell(glass, torch, cell, pls, rounds=rounds)
    fixed = _median_us(s[pls[0]])
    tuned = _median_us(s[(table.scope, table.pack)])
    return {"workload": f"posv n={n} nrhs=1 batch={batch}",
            "fixed_wave_p1_us": round(fixed, 3), "fixed_solves_per_s": round(batch / (fixed * 1e-6), 1),
            "table": f"{glass.SCOPE_NAMES[table.scope]}/P={table.pack}", "table_us": round(tuned, 3),
            "table_solves_per_s": round(batch / (tuned * 1e-6), 1),
            "alg_bytes": timing.alg_bytes("posv", n) * batch, "sets": cell.nsets}


def ragged(glass, torch, count=50000, seed=2, rounds=20, sets=2):
    """The ragged POSV batch (n over {6,...,64}, 1-8 right-hand sides) solved
    by the one-sequence ragged pipeline versus two comparators on pre-grouped
    contiguous copies (the grouping itself is not timed, which favours them):
    one batched POSV launch per (n, nrhs) group, and one launch per order with
    every system's right-hand sides padded with zero columns to the largest
    count (8), the per-size launches of a batch that is not split by nrhs.
    Each variant is captured once per input set and the `sets` copies are
    replayed back to back between two events (time per set reported), so
    consecutive solves read different buffers."""
    dev = torch.device("cuda:0")
    case = inputs.make_ragged(count, seed=seed)
    n, r = case["n"], case["nrhs"]
    rmax = int(r.max())

    def gather(idx, gn, gr, pad_to=None):
        A = np.concatenate([case["A"][case["offA"][i]:case["offA"][i] + gn * gn] for i in idx])
        cols = pad_to or gr
        B = np.zeros((len(idx), gn, cols), np.float32)
        for row, i in enumerate(idx):
            ri = int(r[i])
            B[row, :, :ri] = case["B"][case["offB"][i]:case["offB"][i] + gn * ri].reshape(gn, ri)
        return A.reshape(len(idx), gn, gn), B

    group_keys = sorted(set(zip(n.tolist(), r.tolist())))
    host_groups = [(gn, gr) + gather(np.nonzero((n == gn) & (r == gr))[0], gn, gr) for gn, gr in group_keys]
    host_sizes = [(gn, rmax) + gather(np.nonzero(n == gn)[0], gn, rmax, pad_to=rmax) for gn in sorted(set(n.tolist()))]

    def device_batches(host):
        out = []
        for gn, gr, A, B in host:
            At, Bt = torch.from_numpy(A).to(dev), torch.from_numpy(B).to(dev)
            out.append({"n": gn, "r": gr, "batch": A.shape[0], "A": At, "B": Bt,
                        "info": torch.zeros(A.shape[0], dtype=torch.int32, device=dev)})
        return out

    variants = {
        "ragged": [glass.Ragged(case, device=dev) for _ in range(sets)],
        "per_group": [device_batches(host_groups) for _ in range(sets)],
        "per_size": [device_batches(host_sizes) for _ in range(sets)],
    }
    pristine = {"ragged": (variants["ragged"][0].A.clone(), variants["ragged"][0].B.clone()),
                "per_group": [(g["A"].clone(), g["B"].clone()) for g in variants["per_group"][0]],
                "per_size": [(g["A"].clone(), g["B"].clone()) for g in variants["per_size"][0]]}

    def run(name, k):
        if name == "ragged":
            variants[name][k].solve()
            return
        for g in variants[name][k]:
            st = glass.glass_posv_batched(g["n"], g["r"], g["batch"], g["A"], g["B"], g["info"], None)
            if st != 0:
                raise RuntimeError(f"posv n={g['n']} nrhs={g['r']}: {glass.status_string(st)}")

    def restore():
        for k in range(sets):
            rg = variants["ragged"][k]
            rg.A.copy_(pristine["ragged"][0])
            rg.B.copy_(pristine["ragged"][1])
            for name in ("per_group", "per_size"):
                for g, (A0, B0) in zip(variants[name][k], pristine[name]):
                    g["A"].copy_(A0)
                    g["B"].copy_(B0)

    for name in variants:
        for k in range(sets):
            run(name, k)
    torch.cuda.synchronize()
    restore()
    graphs = {}
    for name in variants:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for k in range(sets):
                run(name, k)
        graphs[name] = g
    torch.cuda.synchronize()
    samples = {k: [] for k in graphs}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    order = list(graphs)
    for it in range(3 + rounds):
        order = order[1:] + order[:1]
        for name in order:
            restore()
            e0.record()
            graphs[name].replay()
            e1.record()
            e1.synchronize()
            if it >= 3:
                samples[name].append(e0.elapsed_time(e1) * 1e3 / sets)
    restore()
    torch.cuda.synchronize()
    alg = int(sum(timing.alg_bytes("posv", int(a), int(b)) for a, b in zip(n, r)))
    tr, tg, ts = (_median_us(samples[k]) for k in ("ragged", "per_group", "per_size"))
    out = {"workload": f"ragged posv: {count} systems, n uniform over {sorted(set(n.tolist()))}, nrhs 1-{rmax}",
           "ragged_us": round(tr, 2), "per_group_us": round(tg, 2), "groups": len(group_keys),
           "per_size_us": round(ts, 2), "sizes": len(host_sizes), "per_size_nrhs": rmax,
           "ragged_speedup": round(tg / tr, 3), "ragged_speedup_vs_per_size": round(ts / tr, 3),
           "alg_bytes": alg, "ragged_gbps": round(alg / (tr * 1e-6) / 1e9, 1),
           "ragged_solves_per_s": round(count / (tr * 1e-6), 1), "input_sets": sets}
    del variants, graphs
    torch.cuda.empty_cache()
    return out


def adjoint(glass, torch, n=12, batch=16384, nrhs=1, rounds=20):
    """Backward of the batched Cholesky solve at n=12, 16,384 systems:
    microseconds per adjoint launch over rotating buffer sets >= 1 GiB."""
    dev = torch.device("cuda:0")
    gen = inputs.torch_generator(dev, 3)
    L = inputs.lower_factor_torch(gen, batch, n, dev)
    X = inputs.uniform_torch(gen, (batch, n, nrhs), dev)
    G = inputs.uniform_torch(gen, (batch, n, nrhs), dev)
    per_set = 4 * (L.numel() + 3 * X.numel() + L.numel())
    sets = max(2, min(64, -(-timing.GIB // per_set)))
    bufs = [{"L": L.clone(), "X": X.clone(), "G": G.clone(), "dB": torch.empty_like(X), "dA": torch.empty_like(L)}
            for _ in range(sets)]
    table = glass.glass_query_placement(glass.OP_POSV_ADJOINT, n, batch)

    def launch(b):
        st = glass.glass_posv_adjoint_batched(n, nrhs, batch, b["L"], b["X"], b["G"], b["dB"], b["dA"], None)
        if st != 0:
            raise RuntimeError(f"adjoint: {glass.status_string(st)}")

    launch(bufs[0])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for b in bufs:
            launch(b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    samples = []
    for it in range(3 + rounds):
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        if it >= 3:
            samples.append(e0.elapsed_time(e1) * 1e3 / sets)
    us = _median_us(samples)
    alg = 4 * (n * (n + 1) // 2 + 3 * n * nrhs + n * n) * batch
    return {"workload": f"posv adjoint n={n} nrhs={nrhs} batch={batch}",
            "placement": f"{glass.SCOPE_NAMES[table.scope]}/P={table.pack}", "us": round(us, 3),
            "alg_bytes": alg, "gbps": round(alg / (us * 1e-6) / 1e9, 1), "sets": sets}


def riccati_gain(glass, torch, cells=((12, 4, 64), (32, 8, 65536)), rounds=20):
    """LQR gain fused (best feasible scope and pack) against the unfused chain."""
    from . import riccati
    out = []
    for nx, nu, batch in cells:
        meds, nsets = riccati.time_forms(glass, torch, nx, nu, batch, rounds=rounds)
        fu = min(((us, pk, f) for (f, pk), us in meds.items() if f in riccati.FUSED_SCOPE))
        un = meds[("unfused", 0)]
        out.append({"workload": f"riccati_gain nx={nx} nu={nu} batch={batch}", "fused_us": round(fu[0], 2),
                    "fused_scope": riccati.FUSED_SCOPE[fu[2]], "fused_pack": fu[1], "unfused_us": round(un, 2),
                    "fused_speedup": round(un / fu[0], 3),
                    "fused_gbps": round(riccati.alg_bytes(nx, nu) * batch / (fu[0] * 1e-6) / 1e9, 1)})
    return out


def batch1_latency(glass, torch, cells=(("posv", 6), ("posv", 32), ("posv", 64), ("gemm", 64), ("trsv", 64),
                                        ("se3_compose", 4)), reps=200):
    """One problem per call at the table's placement, each call synchronized
    on its own: the host round trip (enqueue to completion, what a control
    loop that waits on every solve sees) and the device time of the launch
    between two events, medians over `reps` calls.  The sweep's batch-1
    cells time back-to-back launches instead, so they hide the round trip."""
    import time
    dev = torch.device("cuda:0")
    out = {}
    for op, n in cells:
        bufs = timing.make_set(torch, op, n, 1, dev, seed=11)
        pristine = {k: bufs[k].clone() for k in timing.DESTRUCTIVE.get(op, ())}
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        host, devt = [], []
        for i in range(reps + 10):
            for k, v in pristine.items():
                bufs[k].copy_(v)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev0.record()
            st = timing.launch(glass, op, n, 1, bufs, None)
            ev1.record()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if st != 0:
                raise RuntimeError(f"{op} n={n}: status {st}")
            if i >= 10:
                host.append((t1 - t0) * 1e6)
                devt.append(ev0.elapsed_time(ev1) * 1e3)
        p = glass.glass_query_placement(glass.OPS[op], n, 1)
        out[f"{op} n={n}"] = {"table": f"{glass.SCOPE_NAMES[p.scope]}/P={p.pack}",
                              "host_round_trip_us": round(_median_us(host), 2),
                              "device_us": round(_median_us(devt), 2)}
    return out
