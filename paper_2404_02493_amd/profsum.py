"""Text summary of a rocprofv3 kernel trace of bench.py (for profiles/).

Groups the dispatches by kernel (template arguments dropped) and grid size in
blocks, the same grouping as the per-launch HIP-event profile that bench.py
reports, and puts the average duration of the bench line's roofline kernel from
both sources side by side.

    python -m paper_2404_02493_amd.profsum --trace DIR --bench BENCH.json \\
        --command "rocprofv3 ... -- python3 bench.py ..." --title "..." --out profiles/FILE.md

Counter runs (rocprofv3 --pmc, run_counter_collection.csv) are summarised per kernel
instantiation and grid (mean per dispatch); with SQ_INSTS_VALU and SQ_WAVES present
the table adds the VALU instructions per wavefront, the time the vector units need to
issue them (one wavefront instruction per compute unit per cycle: 256 units at
2.4 GHz) and that time as a fraction of the kernel's average duration in a kernel
trace of the same command:

    python -m paper_2404_02493_amd.profsum counters --pmc DIR [--pmc DIR ...] \\
        --trace TRACE_DIR --match REGEX --command "..." --title "..." --out profiles/FILE.md
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


CUS, CLOCK_HZ = 256, 2.4e9


def counter_groups(pmc_dir: str):
    """{(kernel with template arguments, grid threads): {counter: [values]}}."""
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in csv.DictReader(open(os.path.join(pmc_dir, "run_counter_collection.csv"))):
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("helm::", "").strip()
        agg[(name, int(r["Grid_Size"]))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return agg


def trace_by_instance(trace_dir: str):
    """{(kernel with template arguments, grid threads in all dimensions): (dispatches, mean ns)}."""
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in csv.DictReader(open(os.path.join(trace_dir, "run_kernel_trace.csv"))):
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("helm::", "").strip()
        grid = int(r["Grid_Size_X"]) * int(r.get("Grid_Size_Y") or 1) * int(r.get("Grid_Size_Z") or 1)
        key = (name, grid)
        agg[key][0] += 1
        agg[key][1] += float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    return {k: (v[0], v[1] / v[0]) for k, v in agg.items()}


def counters_main(argv):
    ap = argparse.ArgumentParser(prog="profsum counters")
    ap.add_argument("--pmc", action="append", required=True, help="rocprofv3 --pmc output directory")
    ap.add_argument("--trace", default=None, help="kernel trace of the same command (durations)")
    ap.add_argument("--match", default=".", help="regular expression on the kernel name")
    ap.add_argument("--command", action="append", required=True)
    ap.add_argument("--title", required=True)
    ap.add_argument("--out", required=True)
    a = ap.parse_args(argv)
    merged = collections.defaultdict(dict)
    for d in a.pmc:
        for key, cs in counter_groups(d).items():
            for c, v in cs.items():
                merged[key][c] = (len(v), sum(v) / len(v))
    dur = trace_by_instance(a.trace) if a.trace else {}
    rx = re.compile(a.match)
    keys = sorted(k for k in merged if rx.search(k[0]))
    names = sorted({c for k in keys for c in merged[k]})
    lines = [f"# {a.title}", "", "Commands (from the repository root, MI355X, ROCm 7.2):", "", "```"]
    lines += a.command + ["```", "", "Mean counter value per dispatch, per kernel instantiation and grid "
                          "(grid in threads)."]
    lines += ["", "| kernel | grid | dispatches | " + " | ".join(names) + " |",
              "|---|---:|---:|" + "---:|" * len(names)]
    for k in keys:
        cnt = max(v[0] for v in merged[k].values())
        vals = " | ".join(f"{merged[k][c][1]:.6g}" if c in merged[k] else "" for c in names)
        lines.append(f"| `{k[0]}` | {k[1]} | {cnt} | {vals} |")
    if any("SQ_INSTS_VALU" in merged[k] and "SQ_WAVES" in merged[k] for k in keys):
        lines += ["", "VALU issue bound: SQ_INSTS_VALU / (256 CUs x 2.4 GHz), one wavefront instruction per "
                  "compute unit per cycle (four SIMDs of 16 lanes, a wave64 instruction every four cycles).", "",
                  "| kernel | grid | VALU instr / wave | VALU issue us | trace avg us | VALU-busy fraction |",
                  "|---|---:|---:|---:|---:|---:|"]
        for k in keys:
            m = merged[k]
            if "SQ_INSTS_VALU" not in m or "SQ_WAVES" not in m:
                continue
            valu, waves = m["SQ_INSTS_VALU"][1], m["SQ_WAVES"][1]
            issue_us = valu / (CUS * CLOCK_HZ) * 1e6
            d = dur.get(k)
            frac = f"{issue_us / (d[1] / 1e3):.3f}" if d else ""
            lines.append(f"| `{k[0]}` | {k[1]} | {valu / max(waves, 1):.0f} | {issue_us:.2f} | "
                         f"{d[1] / 1e3:.2f} | {frac} |" if d else
                         f"| `{k[0]}` | {k[1]} | {valu / max(waves, 1):.0f} | {issue_us:.2f} | | |")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:40]))


def main():
    import sys

    if len(sys.argv) > 1 and sys.argv[1] == "counters":
        counters_main(sys.argv[2:])
        return
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
    if "value" in bench:
        lines.append(f"bench.py line of this run: value {bench.get('value')} {bench.get('unit')}, "
                     f"{bench.get('iterations')} iterations, relres {bench.get('relres')}.")
    else:
        lines.append(f"bench.py record of this run: {json.dumps(bench)}")
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
