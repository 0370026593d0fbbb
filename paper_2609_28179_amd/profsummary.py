"""Summarise a rocprofv3 kernel-trace / stats run as short text for profiles/.

  python -m paper_2609_28179_amd.profsummary DIR --kernel SUBSTR --grid GRID_X \
      [--cmd "..."] [--bench-json FILE] [--out FILE]

DIR holds the CSV files of `rocprofv3 --kernel-trace --stats --output-format
csv -o NAME`.  The summary lists the top kernels by total time (stats file)
and, from the per-dispatch trace, the launches of the kernel whose name
contains SUBSTR and whose Grid_Size_X equals GRID_X (one benchmark cell: the
stats file averages a template instance over every batch size it serves).
"""
from __future__ import annotations

import argparse
import csv
import glob
import json
import os
import statistics


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--grid", type=int, required=True)
    ap.add_argument("--cmd", default="")
    ap.add_argument("--bench-json", default="")
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    stats_f = glob.glob(os.path.join(a.dir, "**", "*kernel_stats.csv"), recursive=True)[0]
    trace_f = glob.glob(os.path.join(a.dir, "**", "*kernel_trace.csv"), recursive=True)[0]
    stats = sorted(csv.DictReader(open(stats_f)), key=lambda r: -float(r["TotalDurationNs"]))
    lines = []
    if a.cmd:
        lines += ["command:", "  " + a.cmd, ""]
    lines.append("top kernels by total time (rocprofv3 --stats):")
    lines.append(f"  {'calls':>6} {'avg_us':>10} {'total_ms':>9} {'%':>6}  name")
    for r in stats[:15]:
        lines.append(f"  {r['Calls']:>6} {float(r['AverageNs']) / 1e3:10.2f} {float(r['TotalDurationNs']) / 1e6:9.3f} "
                     f"{float(r['Percentage']):6.2f}  {r['Name'][:110]}")
    durs, meta = [], None
    for r in csv.DictReader(open(trace_f)):
        if a.kernel in r["Kernel_Name"] and int(r["Grid_Size_X"]) == a.grid:
            durs.append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            meta = r
    lines.append("")
    lines.append(f"dispatches of '{a.kernel}' with Grid_Size_X = {a.grid} (kernel trace):")
    if durs:
        lines.append(f"  kernel   {meta['Kernel_Name'][:110]}")
        lines.append(f"  count {len(durs)}  avg {statistics.mean(durs):.2f} us  median {statistics.median(durs):.2f} us  "
                     f"min {min(durs):.2f} us  max {max(durs):.2f} us")
        lines.append(f"  workgroup {meta['Workgroup_Size_X']}  LDS {meta['LDS_Block_Size']} B  VGPR {meta['VGPR_Count']}  "
                     f"AGPR {meta['Accum_VGPR_Count']}  SGPR {meta['SGPR_Count']}  scratch {meta['Scratch_Size']}")
    else:
        lines.append("  none found")
    if a.bench_json and os.path.exists(a.bench_json):
        b = json.loads(open(a.bench_json).read().strip().splitlines()[-1])
        rf = b.get("roofline", {})
        lines.append("")
        lines.append(f"bench.py (separate run, events over the timed region): {rf.get('kernel')}: "
                     f"avg {rf.get('avg_launch_us')} us, {rf.get('achieved')} GB/s algorithmic = "
                     f"{100 * rf.get('frac', 0):.1f} % of {rf.get('peak')} GB/s; ms/step {b.get('ms_per_step')}")
    text = "\n".join(lines) + "\n"
    if a.out:
        open(a.out, "w").write(text)
    print(text)


if __name__ == "__main__":
    main()
