"""Measured memory traffic of one kernel from rocprofv3 counter runs.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch, one rocprofv3 --pmc run each; a kernel name
without template arguments matches every instantiation) are
scaled by what the same counters read for a plain copy kernel of known size
(bench.py --copy-probe: 128 MiB read and 128 MiB written per dispatch), then
stored with a hash of the kernel sources.  bench.py reports the stored figure
only while the sources still hash the same.

    python -m paper_2404_02493_amd.traffic --copy-fetch DIR --copy-write DIR \\
        --fetch DIR --write DIR --kernel 'k_sstep_gram<float, 3, true>' --grid 524288 \\
        --profile-key '(k_sstep_gram<T, MM, true>) [2048 blocks]' --out profiles/FILE.json
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["common.hpp", "reduce.hpp", "kernels_wave.hpp", "kernels_adr.hpp", "kernels_krylov.hpp",
           "kernels_sstep.hpp", "kernels_jac0.hpp"]


def find(profiles_dir: str, profile_key: str) -> float | None:
    """Measured bytes per dispatch from any traffic_*.json record in profiles_dir for the
    kernel profiled under profile_key (current sources only), else None."""
    if not os.path.isdir(profiles_dir):
        return None
    for name in sorted(os.listdir(profiles_dir)):
        if name.startswith("traffic_") and name.endswith(".json"):
            v = load(os.path.join(profiles_dir, name), profile_key)
            if v is not None:
                return v
    return None
COPY_BYTES = 4096 * 4096 * 8  # bench.py --copy-probe: complex64 4096^2, read once and written once


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in SOURCES:
        with open(os.path.join(_HERE, "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _per_dispatch(run_dir: str, counter: str, kernel: str, grid: int | None = None) -> tuple[float, int]:
    vals = []
    with open(os.path.join(run_dir, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].split("(")[0].replace("void ", "").replace("helm::", "")
            if name != kernel and name.split("<")[0] != kernel:
                continue
            if grid is not None and int(r["Grid_Size"]) != grid:
                continue
            vals.append(float(r["Counter_Value"]))
    if not vals:
        raise SystemExit(f"no {counter} samples for {kernel} (grid {grid}) in {run_dir}")
    return sum(vals) / len(vals), len(vals)


def summarize(copy_fetch: str, copy_write: str, fetch: str, write: str, kernel: str, grid: int,
              profile_key: str, workload: str, algorithmic_bytes: float | None) -> dict:
    cf, _ = _per_dispatch(copy_fetch, "FETCH_SIZE", "k_copy<float>")
    cw, _ = _per_dispatch(copy_write, "WRITE_SIZE", "k_copy<float>")
    fk, nf = _per_dispatch(fetch, "FETCH_SIZE", kernel, grid)
    wk, nw = _per_dispatch(write, "WRITE_SIZE", kernel, grid)
    fs = COPY_BYTES / 1024.0 / cf
    ws = COPY_BYTES / 1024.0 / cw
    total = (fk * fs + wk * ws) * 1024.0
    out = {"kernel": kernel, "grid_threads": grid, "profile_key": profile_key, "workload": workload,
           "fetch_kib_per_dispatch": fk, "write_kib_per_dispatch": wk, "dispatches": [nf, nw],
           "copy_probe": {"bytes_each_way": COPY_BYTES, "fetch_kib": cf, "write_kib": cw},
           "fetch_scale": fs, "write_scale": ws, "bytes_per_dispatch": total,
           "source_sha256": kernel_source_hash()}
    if algorithmic_bytes:
        out["algorithmic_bytes_per_dispatch"] = algorithmic_bytes
        out["traffic_over_algorithmic"] = total / algorithmic_bytes
    return out


def load(path: str, profile_key: str) -> float | None:
    """Measured bytes per dispatch for the kernel profiled under profile_key, or None if
    there is no record for it or the kernel sources changed since it was taken."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("profile_key") != profile_key or rec.get("source_sha256") != kernel_source_hash():
        return None
    return float(rec["bytes_per_dispatch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--grid", type=int, default=None, help="grid size in work-items (all grids if omitted)")
    ap.add_argument("--profile-key", required=True)
    ap.add_argument("--workload", default="layered4096 FP32+refinement solve")
    ap.add_argument("--algorithmic-bytes", type=float, default=None)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    rec = summarize(a.copy_fetch, a.copy_write, a.fetch, a.write, a.kernel, a.grid, a.profile_key, a.workload,
                    a.algorithmic_bytes)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
