"""HBM traffic of one benchmark cell from rocprofv3 counters.

  run:        launch one cell's kernel under the built-in placement R times,
              then a plain 1 GiB device-to-device copy R times (the
              calibration kernel of known size).  Meant to run under
              `rocprofv3 --pmc FETCH_SIZE` and, separately, `--pmc WRITE_SIZE`.
  summarize:  read the two counter-collection CSVs, scale each counter by
              what it reads for the copy (known bytes / counter bytes) and
              write bytes per launch to profiles/traffic.json plus a short
              text summary.

  python -m paper_2609_28179_amd.traffic run --op gemm --n 64 --batch 65536
  python -m paper_2609_28179_amd.traffic summarize --fetch DIR --write DIR --op gemm --n 64 --batch 65536

The counters are read per dispatch in KiB.  A counter well above the cell's
algorithmic bytes means re-reads that the kernel could avoid.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
COPY_BYTES = 1 << 30


# Sources a cell's kernel is built from: the op's own files plus the shared
# device helpers, the geometry rule and the placement table that picks it.
_COMMON_SOURCES = ("device_common.hpp", "glass_internal.hpp", "api.cpp", "glass_table_gfx950.inc")
_CHOL_SOURCES = ("chol.hip", "chol_device.hpp", "chol_blk.hip", "chol_blk.hpp", "subwave.hip")
_OP_SOURCES = {"gemm": ("gemm.hip",), "gemv": ("gemv.hip",), "potrf": _CHOL_SOURCES, "potrs": _CHOL_SOURCES,
               "posv": _CHOL_SOURCES, "trsv": _CHOL_SOURCES, "se3_compose": ("se3.hip",),
               "se3_inverse": ("se3.hip",)}


def kernel_source_hash(op: str) -> str:
    """Hash of the sources op's kernels are built from; a traffic record is
    valid for this hash only (a change elsewhere in csrc/ leaves it valid)."""
    h = hashlib.sha256()
    csrc = os.path.join(PKG, "csrc")
    for f in sorted(_COMMON_SOURCES + _OP_SOURCES[op]):
        h.update(f.encode())
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _run(a):
    import torch
    from . import glass, timing

    dev = torch.device("cuda:0")
    bufs = timing.make_set(torch, a.op, a.n, a.batch, dev, seed=77)
    pristine = {k: bufs[k].clone() for k in timing.DESTRUCTIVE.get(a.op, ())}
    torch.cuda.synchronize()
    for r in range(a.reps):
        for k, v in pristine.items():
            bufs[k].copy_(v)
        st = timing.launch(glass, a.op, a.n, a.batch, bufs, None)
        if st != 0:
            raise RuntimeError(f"{a.op} n={a.n} batch={a.batch}: {glass.status_string(st)}")
        torch.cuda.synchronize()
        print(f"launch {r + 1}/{a.reps} done", flush=True)
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for r in range(a.reps):
        dst.copy_(src)
        torch.cuda.synchronize()
    print(f"copy of {COPY_BYTES} bytes x {a.reps} done", flush=True)


def _rows(d):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not f:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    return list(csv.DictReader(open(f[0])))


def _per_dispatch(rows, counter, match):
    vals = {}
    for r in rows:
        if r["Counter_Name"] == counter and match(r["Kernel_Name"]):
            vals.setdefault(r.get("Dispatch_Id", r.get("Correlation_Id")), []).append(float(r["Counter_Value"]))
    return [sum(v) for v in vals.values()]


def _summarize(a):
    from . import timing

    is_glass = lambda name: "glass::" in name
    is_copy = lambda name: "copyBuffer" in name
    fr, wr = _rows(a.fetch), _rows(a.write)
    f_k = _per_dispatch(fr, "FETCH_SIZE", is_glass)
    w_k = _per_dispatch(wr, "WRITE_SIZE", is_glass)
    f_c = _per_dispatch(fr, "FETCH_SIZE", is_copy)
    w_c = _per_dispatch(wr, "WRITE_SIZE", is_copy)
    if not (f_k and w_k and f_c and w_c):
        raise RuntimeError("missing dispatches in the counter CSVs")
    # the 1 GiB calibration copies are the largest copy dispatches (the run
    # also restores destructive inputs with smaller copies between launches)
    f_c = [v for v in f_c if v >= 0.9 * max(f_c)]
    w_c = [v for v in w_c if v >= 0.9 * max(w_c)]
    sf = COPY_BYTES / (statistics.median(f_c) * 1024)
    sw = COPY_BYTES / (statistics.median(w_c) * 1024)
    fetch = statistics.median(f_k) * 1024 * sf
    write = statistics.median(w_k) * 1024 * sw
    alg = timing.alg_bytes(a.op, a.n) * a.batch
    rec = {"cell": [a.op, a.n, a.batch], "source_hash": kernel_source_hash(a.op),
           "fetch_kib_per_launch": statistics.median(f_k), "write_kib_per_launch": statistics.median(w_k),
           "copy_bytes": COPY_BYTES, "copy_fetch_kib": statistics.median(f_c), "copy_write_kib": statistics.median(w_c),
           "scale_fetch": sf, "scale_write": sw, "fetch_bytes": fetch, "write_bytes": write,
           "bytes_per_launch": round(fetch + write), "alg_bytes_per_launch": alg,
           "traffic_over_alg": (fetch + write) / alg, "commands": a.cmd}
    os.makedirs(os.path.dirname(a.out), exist_ok=True)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    lines = [f"HBM traffic of {a.op} n={a.n} batch={a.batch} (built-in placement), rocprofv3 counters", ""]
    lines += ["commands:"] + [f"  {c}" for c in a.cmd] + [""]
    lines += [f"calibration: 1 GiB device copy reads FETCH_SIZE {rec['copy_fetch_kib']:.0f} KiB, "
              f"WRITE_SIZE {rec['copy_write_kib']:.0f} KiB -> scale {sf:.4f} / {sw:.4f}",
              f"kernel per launch: FETCH_SIZE {rec['fetch_kib_per_launch']:.0f} KiB, WRITE_SIZE "
              f"{rec['write_kib_per_launch']:.0f} KiB ({len(f_k)} / {len(w_k)} dispatches)",
              f"scaled: read {fetch / 1e6:.1f} MB + write {write / 1e6:.1f} MB = {(fetch + write) / 1e6:.1f} MB "
              f"per launch; algorithmic {alg / 1e6:.1f} MB; ratio {(fetch + write) / alg:.3f}",
              f"kernel source hash {rec['source_hash']}"]
    text = "\n".join(lines) + "\n"
    if a.txt:
        open(a.txt, "w").write(text)
    print(text)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    r = sub.add_parser("run")
    s = sub.add_parser("summarize")
    for p in (r, s):
        p.add_argument("--op", required=True)
        p.add_argument("--n", type=int, required=True)
        p.add_argument("--batch", type=int, required=True)
    r.add_argument("--reps", type=int, default=5)
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    s.add_argument("--txt", default="")
    s.add_argument("--cmd", action="append", default=[])
    a = ap.parse_args(argv)
    {"run": _run, "summarize": _summarize}[a.cmd_name](a)


if __name__ == "__main__":
    sys.exit(main())
