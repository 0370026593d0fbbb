"""Device-side timing of one (op, n, batch) cell under a placement.

Protocol (after Sec. IV-A): launches of one placement run back to back with
a single synchronisation, here as one HIP graph of S launches replayed
between two events, so the time per launch is the kernel's own and not the
host's enqueue rate; every launch of a destructive op (POTRF, POTRS, POSV,
TRSV) sees a fresh valid input because all S buffer sets are restored from a
pristine copy between replays, outside the events; S rotating buffer sets
totalling >= 1 GiB keep inputs out of the 256 MB last-level cache; placement
order is shuffled in every round; every raw sample is kept.

Algorithmic bytes per problem (the contract's minimum reads + writes, FP32):
  GEMM 4(2n^2 + n^2), GEMV 4(n^2 + 2n), POTRF 4(n(n+1)/2 + n^2),
  POTRS 4(n(n+1)/2 + 2 n r), POSV 4(n(n+1)/2 + n r + n^2 + n r),
  TRSV 4(n(n+1)/2 + 2n), SE(3) compose 160, SE(3) inverse 112.
Flops per problem: GEMM 2n^3, GEMV 2n^2, POTRF n^3/3, POTRS 2 n^2 r,
POSV n^3/3 + 2 n^2 r, TRSV n^2, SE(3) compose 63, inverse 15.
"""
from __future__ import annotations

import math
import random

import numpy as np

from . import inputs

DESTRUCTIVE = {"potrf": ("A",), "potrs": ("B",), "posv": ("A", "B"), "trsv": ("x",)}
SWEEP_OPS = ("gemm", "gemv", "potrf", "potrs", "posv", "trsv")
SE3_OPS = ("se3_compose", "se3_inverse")
SWEEP_N = (3, 4, 6, 7, 12, 16, 32, 64)
SWEEP_B = (1, 16, 256, 4096, 65536)          # the benchmark grid's batches
TABLE_B = (1, 16, 256, 1024, 4096, 65536)    # the dispatch table's batch keys (adds the 1024-system POSV)
PACKS = (1, 2, 4, 8)
HELDOUT_N = (5, 9, 20, 48)          # orders the table does not hold (cost-model evaluation)
HELDOUT_B = (256, 65536)
GIB = 1 << 30


def alg_bytes(op: str, n: int, nrhs: int = 1) -> int:
    tri = n * (n + 1) // 2
    return 4 * {
        "gemm": 3 * n * n,
        "gemv": n * n + 2 * n,
        "potrf": tri + n * n,
        "potrs": tri + 2 * n * nrhs,
        "posv": tri + n * nrhs + n * n + n * nrhs,
        "trsv": tri + 2 * n,
        "se3_compose": 40,
        "se3_inverse": 28,
    }[op]


def flops(op: str, n: int, nrhs: int = 1) -> float:
    return {
        "gemm": 2.0 * n ** 3,
        "gemv": 2.0 * n * n,
        "potrf": n ** 3 / 3.0,
        "potrs": 2.0 * n * n * nrhs,
        "posv": n ** 3 / 3.0 + 2.0 * n * n * nrhs,
        "trsv": float(n * n),
        "se3_compose": 63.0,
        "se3_inverse": 15.0,
    }[op]


def sweep_cells(batches=SWEEP_B):
    """The benchmark grid (250 cells); with batches=TABLE_B the dispatch
    table's grid (300 cells)."""
    cells = [(op, n, b) for op in SWEEP_OPS for n in SWEEP_N for b in batches]
    cells += [(op, 4, b) for op in SE3_OPS for b in batches]
    return cells


def table_cells():
    return sweep_cells(TABLE_B)


def heldout_cells():
    return [(op, n, b) for op in SWEEP_OPS for n in HELDOUT_N for b in HELDOUT_B]


def feasible_placements(glass, op: str, n: int, nrhs: int = 1):
    out = []
    for scope in (glass.SCOPE_THREAD, glass.SCOPE_WAVE, glass.SCOPE_WORKGROUP, glass.SCOPE_SUBWAVE):
        for p in PACKS:
            if glass.glass_placement_feasible(glass.OPS[op], n, nrhs, scope, p) == 1:
                out.append((scope, p))
    return out


# ------------------------------------------------------------------ buffers
def make_set(torch, op: str, n: int, batch: int, device, seed: int, nrhs: int = 1) -> dict:
    """One buffer set of a cell, drawn on the device with the shared recipes."""
    g = inputs.torch_generator(device, seed)
    f32 = torch.float32
    if op == "gemm":
        return {"A": inputs.uniform_torch(g, (batch, n, n), device), "B": inputs.uniform_torch(g, (batch, n, n), device),
                "C": torch.zeros((batch, n, n), dtype=f32, device=device)}
    if op == "gemv":
        return {"A": inputs.uniform_torch(g, (batch, n, n), device), "x": inputs.uniform_torch(g, (batch, n), device),
                "y": torch.zeros((batch, n), dtype=f32, device=device)}
    if op == "potrf":
        return {"A": inputs.spd_torch(g, batch, n, device),
                "info": torch.zeros((batch,), dtype=torch.int32, device=device)}
    if op == "posv":
        return {"A": inputs.spd_torch(g, batch, n, device), "B": inputs.uniform_torch(g, (batch, n, nrhs), device),
                "info": torch.zeros((batch,), dtype=torch.int32, device=device)}
    if op == "potrs":
        return {"L": inputs.lower_factor_torch(g, batch, n, device),
                "B": inputs.uniform_torch(g, (batch, n, nrhs), device)}
    if op == "trsv":
        return {"L": inputs.lower_factor_torch(g, batch, n, device), "x": inputs.uniform_torch(g, (batch, n), device)}
    if op == "se3_compose":
        return {"Ta": inputs.se3_torch(g, batch, device), "Tb": inputs.se3_torch(g, batch, device),
                "T": torch.zeros((batch, 4, 4), dtype=f32, device=device)}
    if op == "se3_inverse":
        return {"Ta": inputs.se3_torch(g, batch, device), "T": torch.zeros((batch, 4, 4), dtype=f32, device=device)}
    raise ValueError(op)


def set_bytes(bufs: dict) -> int:
    return sum(t.numel() * t.element_size() for t in bufs.values())


def launch(glass, op: str, n: int, batch: int, bufs: dict, force, nrhs: int = 1) -> int:
    """One call of the op on a buffer set through the C-ABI (torch's current stream)."""
    if op == "gemm":
        return glass.glass_gemm_batched(n, n, n, batch, 1.0, bufs["A"], bufs["B"], 0.0, bufs["C"], force)
    if op == "gemv":
        return glass.glass_gemv_batched(n, n, batch, 1.0, bufs["A"], bufs["x"], 0.0, bufs["y"], force)
    if op == "potrf":
        return glass.glass_potrf_batched(n, batch, bufs["A"], bufs["info"], force)
    if op == "posv":
        return glass.glass_posv_batched(n, nrhs, batch, bufs["A"], bufs["B"], bufs["info"], force)
    if op == "potrs":
        return glass.glass_potrs_batched(n, nrhs, batch, bufs["L"], bufs["B"], force)
    if op == "trsv":
        return glass.glass_trsv_batched(n, batch, 0, bufs["L"], bufs["x"], force)
    if op == "se3_compose":
        return glass.glass_se3_batched(glass.OP_SE3_COMPOSE, batch, bufs["Ta"], bufs["Tb"], bufs["T"], force)
    if op == "se3_inverse":
        return glass.glass_se3_batched(glass.OP_SE3_INVERSE, batch, bufs["Ta"], None, bufs["T"], force)
    raise ValueError(op)


class Cell:
    """S rotating buffer sets of one cell plus a pristine copy of its destructive inputs."""

    def __init__(self, torch, op, n, batch, device, seed, min_total=GIB, max_sets=64, nrhs=1):
        self.torch, self.op, self.n, self.batch, self.nrhs = torch, op, n, batch, nrhs
        base = make_set(torch, op, n, batch, device, seed, nrhs)
        sb = set_bytes(base)
        self.nsets = int(min(max_sets, max(2, math.ceil(min_total / sb))))
        self.sets = [base] + [{k: v.clone() for k, v in base.items()} for _ in range(self.nsets - 1)]
        self.pristine = {k: base[k].clone() for k in DESTRUCTIVE.get(op, ())}
        self.set_bytes = sb

    def restore(self):
        for s in self.sets:
            for k, v in self.pristine.items():
                s[k].copy_(v)

    def launch(self, glass, i, force):
        return launch(glass, self.op, self.n, self.batch, self.sets[i], force, self.nrhs)


def time_cell(glass, torch, cell: Cell, placements, rounds: int = 20, warmup: int = 3, rng=None):
    """Median-ready raw samples (microseconds per launch) for each placement."""
    rng = rng or random.Random(0)
    graphs = {}
    for pl in placements:
        st = cell.launch(glass, 0, pl)  # eager first launch: loads the code object, checks status
        if st != 0:
            raise RuntimeError(f"{cell.op} n={cell.n} batch={cell.batch} {pl}: status {st}")
        torch.cuda.synchronize()
        cell.restore()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for i in range(cell.nsets):
                cell.launch(glass, i, pl)
        graphs[pl] = g
    torch.cuda.synchronize()
    samples = {pl: [] for pl in placements}
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    order = list(placements)
    for r in range(warmup + rounds):
        rng.shuffle(order)
        for pl in order:
            cell.restore()
            ev0.record()
            graphs[pl].replay()
            ev1.record()
            ev1.synchronize()
            if r >= warmup:
                samples[pl].append(ev0.elapsed_time(ev1) * 1e3 / cell.nsets)
    cell.restore()
    del graphs
    return samples


def floor_us(torch, device, reps: int = 64, rounds: int = 10) -> float:
    """Back-to-back time of a near-empty kernel (one-element fill) in a graph."""
    x = torch.zeros(1, device=device)
    x.fill_(1.0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            x.fill_(1.0)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    out = []
    for _ in range(rounds):
        ev0.record()
        g.replay()
        ev1.record()
        ev1.synchronize()
        out.append(ev0.elapsed_time(ev1) * 1e3 / reps)
    return float(np.median(out))


def copy_bandwidth(torch, device, nbytes: int = GIB, reps: int = 10) -> float:
    """Achievable HBM bandwidth (GB/s, read + write counted) of a device copy."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=device).uniform_()
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    out = []
    for _ in range(reps):
        ev0.record()
        dst.copy_(src)
        ev1.record()
        ev1.synchronize()
        out.append(2 * nbytes / (ev0.elapsed_time(ev1) * 1e-3) / 1e9)
    return float(np.median(out))


STREAM_KINDS = {"read": 0, "write": 1, "copy": 2, "read2_write1": 3}


def stream_ceilings(glass, torch, device, nbytes: int = 2 * GIB, reps: int = 10, blocks=(16384, 32768, 65536, 0)):
    """Attainable bandwidth (GB/s, bytes read + written) of the library's plain
    streaming kernels: read only, write only, copy, and two reads per write
    (c = a + b), each over `nbytes`-byte buffers, the best median over a few
    grid sizes of 1024-lane workgroups (0: one 16-byte element per lane).
    Returns {kind: {"gbps": .., "blocks": ..}}."""
    n = nbytes // 4
    blocks = tuple(b if b else -(-(n // 4) // 1024) for b in blocks)
    a = torch.empty(n, dtype=torch.float32, device=device).fill_(1.0)
    b = torch.empty_like(a).fill_(1.0)
    c = torch.empty_like(a)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    moved = {"read": nbytes, "write": nbytes, "copy": 2 * nbytes, "read2_write1": 3 * nbytes}
    out = {}
    for kind, code in STREAM_KINDS.items():
        best = None
        for nb in blocks:
            st = glass.glass_stream_probe(code, a, b, c, n // 4, nb)
            if st != 0:
                raise RuntimeError(f"stream probe {kind}: status {st}")
            torch.cuda.synchronize()
            samples = []
            for _ in range(reps):
                ev0.record()
                glass.glass_stream_probe(code, a, b, c, n // 4, nb)
                ev1.record()
                ev1.synchronize()
                samples.append(moved[kind] / (ev0.elapsed_time(ev1) * 1e-3) / 1e9)
            med = float(np.median(samples))
            if best is None or med > best[0]:
                best = (med, nb)
        out[kind] = {"gbps": round(best[0], 1), "blocks": best[1]}
    del a, b, c
    torch.cuda.empty_cache()
    return out


def _main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="measured streaming ceilings of this GPU")
    ap.add_argument("cmd", choices=("ceilings",))
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    import torch
    from . import glass
    dev = torch.device("cuda:0")
    res = stream_ceilings(glass, torch, dev)
    p = torch.cuda.get_device_properties(0)
    lines = [f"Streaming ceilings of {p.gcnArchName} ({p.multi_processor_count} CUs), 2 GiB buffers, "
             f"median of 10 launches, best of grids {{16384, 32768, 65536, one element per lane}} x 1024 lanes",
             "",
             "command: python -m paper_2609_28179_amd.timing ceilings", ""]
    for kind, v in res.items():
        lines.append(f"{kind:13s} {v['gbps']:8.1f} GB/s  ({100 * v['gbps'] / 8000:.1f} % of 8 TB/s; "
                     f"{v['blocks']} workgroups)")
    text = "\n".join(lines) + "\n"
    print(text)
    print(json.dumps(res), file=sys.stderr)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)


if __name__ == "__main__":
    _main()
