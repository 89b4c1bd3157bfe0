"""Text summary of a rocprofv3 kernel trace of bench.py (for profiles/).

Groups the dispatches by kernel (template arguments dropped) and grid size in
blocks, the same grouping as the per-launch HIP-event profile that bench.py
reports, and puts the average duration of the bench line's roofline kernel from
both sources side by side.

    python -m paper_2404_02493_amd.profsum --trace DIR --bench BENCH.json \\
        --command "rocprofv3 ... -- python3 bench.py ..." --title "..." --out profiles/FILE.md
"""
from __future__ import annotations

import argparse
import collections
import csv
import json
import os
import re


def base_name(kernel: str) -> str:
    """'void helm::k_fg_orth<float, 7>(unsigned long, ...)' -> 'k_fg_orth'."""
    k = kernel.replace("void ", "")
    k = k.split("(")[0]
    k = k.split("<")[0]
    return k.replace("helm::", "").strip()


def trace_groups(trace_dir: str):
    rows = list(csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv"))))
    agg = collections.defaultdict(lambda: [0, 0.0])
    total = 0.0
    for r in rows:
        blocks = int(r["Grid_Size_X"]) // max(1, int(r["Workgroup_Size_X"]))
        d = float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        key = (base_name(r["Kernel_Name"]), blocks)
        agg[key][0] += 1
        agg[key][1] += d
        total += d
    return agg, total, len(rows)


def bench_key(name: str):
    """'(k_fg_orth<P, J>) [2048 blocks]' or '(k_sstep_gram<T, MM, true>) [1924 blocks, 134.2 MB]'."""
    m = re.match(r"\(?\s*([A-Za-z_0-9]+)[^\[]*\[(\d+) blocks", name)
    return (m.group(1), int(m.group(2))) if m else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True, help="rocprofv3 output directory (run_kernel_trace.csv)")
    ap.add_argument("--bench", required=True, help="the JSON line bench.py printed in the same run")
    ap.add_argument("--command", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--top", type=int, default=30)
    a = ap.parse_args()
    agg, total, nd = trace_groups(a.trace)
    with open(a.bench) as f:
        bench = json.loads(f.read().strip().splitlines()[-1])
    roof = bench.get("roofline") or {}
    lines = [f"# {a.title}", "", "Command (from the repository root, MI355X, ROCm 7.2):", "", "```", a.command, "```", ""]
    lines.append(f"bench.py line of this run: value {bench.get('value')} {bench.get('unit')}, "
                 f"{bench.get('iterations')} iterations, relres {bench.get('relres')}.")
    lines.append("")
    if roof:
        key = bench_key(roof.get("kernel", ""))
        tr = agg.get(key) if key else None
        lines.append(f"Roofline kernel of the bench line: `{roof.get('kernel')}`: HIP-event average "
                     f"{roof.get('avg_launch_us')} us per launch over {roof.get('launches')} launches, "
                     f"{roof.get('achieved')} GB/s algorithmic, {roof.get('frac')} of {roof.get('peak')} GB/s.")
        if tr:
            lines.append(f"rocprofv3 kernel trace, same kernel and grid: {tr[0]} dispatches, average "
                         f"{tr[1] / tr[0] / 1e3:.2f} us.")
        lines.append("")
    lines += [f"Kernel time in the trace: {total / 1e6:.1f} ms over {nd} dispatches (every step of the run, "
              "including the tuned-shape lookup and the profiled step).", "",
              "| kernel | blocks | dispatches | avg us | total ms | % |", "|---|---:|---:|---:|---:|---:|"]
    for (name, blocks), (cnt, d) in sorted(agg.items(), key=lambda kv: -kv[1][1])[: a.top]:
        lines.append(f"| `{name}` | {blocks} | {cnt} | {d / cnt / 1e3:.2f} | {d / 1e6:.2f} | {100 * d / total:.2f} |")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:14]))


if __name__ == "__main__":
    main()
