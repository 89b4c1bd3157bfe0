"""Benchmark: time to a 1e-6 relative residual on the 4096 x 4096, k = 2100 layered
medium (8 layers + 20 elliptical inclusions, fast-marching phase, 7 levels), FP32
cycles inside FP64 iterative refinement, with the plain FP64 GPU solve beside it.

One "step" is one full solve from a zero initial guess (all parts of the path:
cycles, Krylov, FP64 residual and refinement), inputs resident in HBM.  Prints
one JSON line.  Extra fields: the FP64 solve, the per-kernel profile from HIP
events (with the algorithmic bytes of each launch), the roofline of the
dominant kernel, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(case, iterations: int, budget_s: float = 30.0):
    """The FP64 CPU oracle on a bounded sample of the same workload: one FGMRES
    iteration (one cycle from a zero iterate, A z and one Arnoldi step) at full
    size, extrapolated to the iteration count of the FP64 GPU solve."""
    import torch

    from oracle.cycle import Problem, cycle
    from oracle.grid import apply_A, cdot, cnorm

    threads = os.cpu_count() or 1
    torch.set_num_threads(threads)
    P = Problem(case.velocity, case.k, case.levels, damping_cells=case.damping_cells, phi=case.phi)
    g = torch.as_tensor(case.g)
    t0 = time.perf_counter()
    v = g / cnorm(g)
    z = cycle(P, v, torch.zeros_like(v))
    w = apply_A(z, P.kappa[1], P.h[1])
    h = cdot(v, w)
    w = w - h * v
    _ = cnorm(w)
    t_iter = time.perf_counter() - t0
    cores = torch.get_num_threads()
    single = single_thread_oracle()
    torch.set_num_threads(threads)
    return {"value": t_iter * iterations, "unit": "s", "cores": cores, "kind": "oracle",
            "sample": f"one FP64 FGMRES iteration (cycle + A z + Arnoldi step) at {case.n}x{case.n}, "
                      f"{t_iter:.2f} s, times {iterations} iterations of the FP64 solve",
            "sample_seconds": t_iter, "cpu_model": cpu_model(), "single_thread": single}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def single_thread_oracle():
    """The oracle on one thread: the whole FP64 FGMRES(20) solve of the 128^2 constant
    medium (k = 80), and one FGMRES iteration of the 512^2 random medium (k = 320)
    times the iteration count of its FP64 GPU solve."""
    import torch

    import helm_inputs as hi
    from oracle.cycle import Problem, cycle
    from oracle.grid import apply_A, cdot, cnorm
    from oracle.solve import fgmres
    from paper_2404_02493_amd import Helmholtz

    torch.set_num_threads(1)
    out = {}
    c1 = hi.make_case("const128", seed=0)
    P = Problem(c1.velocity, c1.k, c1.levels, damping_cells=c1.damping_cells, phi=c1.phi)
    t0 = time.perf_counter()
    _, its, rr, _ = fgmres(P, torch.as_tensor(c1.g), tol=1e-6, maxit=500)
    out["const128"] = {"seconds": round(time.perf_counter() - t0, 3), "iterations": its, "relres": rr}
    c2 = hi.make_case("grf512", seed=0)
    H = Helmholtz(c2.velocity, c2.k, levels=c2.levels, precision="c128", damping_cells=c2.damping_cells)
    H.set_phase(c2.phi)
    gd = torch.as_tensor(c2.g).to("cuda:0")
    _, its2, rr2, _ = H.solve(gd, tol=1e-6, maxit=2000, mode=0)
    H.close()
    P2 = Problem(c2.velocity, c2.k, c2.levels, damping_cells=c2.damping_cells, phi=c2.phi)
    g2 = torch.as_tensor(c2.g)
    t0 = time.perf_counter()
    v = g2 / cnorm(g2)
    z = cycle(P2, v, torch.zeros_like(v))
    w = apply_A(z, P2.kappa[1], P2.h[1])
    w = w - cdot(v, w) * v
    _ = cnorm(w)
    t_it = time.perf_counter() - t0
    out["grf512"] = {"seconds_per_iteration": round(t_it, 3), "gpu_fp64_iterations": its2,
                     "extrapolated_seconds": round(t_it * its2, 1)}
    return out


def bench_adjoint(seed: int = 0, K: int = 10, reps: int = 3):
    """The adjoint of K unrolled FP32 cycles on the 1024^2, k = 640 random medium
    (7 levels, fast-marching phase in float32): wall time of one helm_cycle_backward
    (which re-runs the K cycles with their tapes) against K forward cycles, and of the
    split path (a recording forward pass, then only the reverse)."""
    import numpy as np
    import torch

    import helm_inputs as hi
    from paper_2404_02493_amd import Helmholtz

    case = hi.make_case("grf1024", seed=seed)
    H = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c64", damping_cells=case.damping_cells)
    H.set_phase(case.phi)
    g = torch.as_tensor(case.g).to(H.cdtype).to("cuda:0")

    def forward():
        u = torch.zeros_like(g)
        for _ in range(K):
            H.cycle(g, u)
        return u

    u = forward()
    _, gu = H.loss(g, u, grad=True)
    H.cycle_backward(K, g, gu)  # first call allocates the tape
    ur = torch.empty_like(g)
    H.cycle_record(K, g, ur)  # and the split path's graphs
    H.cycle_reverse(K, g, gu)
    torch.cuda.synchronize()

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    tf, tb, trec, trev = [], [], [], []
    for _ in range(reps):
        tf.append(timed(forward))
        tb.append(timed(lambda: H.cycle_backward(K, g, gu)))
        trec.append(timed(lambda: H.cycle_record(K, g, ur)))
        trev.append(timed(lambda: H.cycle_reverse(K, g, gu)))
    H.close()
    f, b = float(np.median(tf)), float(np.median(tb))
    rec, rev = float(np.median(trec)), float(np.median(trev))
    return {"workload": "grf1024 (n=1024, k=640, L=7), K=10 FP32 cycles from zero", "forward_ms": round(1e3 * f, 3),
            "backward_ms": round(1e3 * b, 3), "backward_over_forward": round(b / f, 2),
            "note": "backward re-runs the K cycles recording one tape per cycle, then reverses them",
            "split": {"record_ms": round(1e3 * rec, 3), "reverse_ms": round(1e3 * rev, 3),
                      "reverse_over_forward": round(rev / f, 2),
                      "step_ms": round(1e3 * (rec + rev), 3), "unsplit_step_ms": round(1e3 * (f + b), 3),
                      "note": "the forward pass records its cycles (helm_cycle_record), the backward "
                              "pass only reverses them (helm_cycle_reverse); step = both"}}


HBM_CLEAN = ("k_jac0_restrict", "k_jac0_prolong_jacobi", "k_fg_arnoldi", "k_fg_orth")


def hbm_rooflines(kernels):
    """Kernels of the 4096^2 solve whose data streams through HBM on every launch (the
    fine-grid level-1 passes and the outer Krylov passes: their inputs are not reused
    within the 256 MB Infinity Cache between launches), each with its algorithmic bytes
    per launch over its average event-timed launch duration, and the counter-measured
    HBM bytes of a profiles/ traffic record over the same duration while the kernel
    sources are those the record was taken with."""
    from paper_2404_02493_amd.traffic import find as find_traffic

    out = []
    for fam in HBM_CLEAN:
        ks = [k for k in kernels if k["name"].startswith(f"({fam}<") or k["name"].startswith(f"{fam} ")
              or k["name"].startswith(f"({fam})")]
        if not ks:
            continue
        launches = sum(k["launches"] for k in ks)
        ms = sum(k["ms"] for k in ks)
        by = sum(k["bytes"] for k in ks)
        gbs = by / (ms * 1e-3) / 1e9
        tb = find_traffic(os.path.join(ROOT, "profiles"), fam)
        avg_s = 1e-3 * ms / launches
        out.append({"kernel": fam, "launches": launches, "avg_launch_us": round(1e6 * avg_s, 2),
                    "bytes_per_launch": by / launches, "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "traffic": round(tb / avg_s / 1e9, 1) if tb else None, "traffic_bytes_per_launch": tb})
    return out


def bench_sharp(seed: int, maxit: int = 1000):
    """The same 4096^2 workload without the smoothing of the medium (sharp layers and
    inclusions as generated): FP32+refinement with a bounded iteration count, so that
    the gap to the unsmoothed medium is a measured number (iterations, final relres)."""
    import torch

    import helm_inputs as hi
    from paper_2404_02493_amd import Helmholtz

    case = hi.make_case("layered4096_sharp", seed=seed)
    H = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c64", damping_cells=case.damping_cells)
    H.set_phase(case.phi)
    g = torch.as_tensor(case.g).to("cuda:0")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, its, rr, hist = H.solve(g, tol=1e-6, maxit=maxit, mode=1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    H.close()
    return {"workload": "layered4096_sharp (no smoothing of the medium)", "damping_cells": case.damping_cells,
            "maxit": maxit, "iterations": its, "relres": rr, "seconds": round(dt, 3), "converged": rr < 1e-6}


def bench_shifted(case, g, tol: float = 1e-7, shift: float = 0.01):
    """The shifted equation (relative imaginary shift 0.01 of kappa, the paper's
    Section 4.3.2 test) on the same 4096^2 medium, FP32+refinement to 1e-7."""
    import torch

    from paper_2404_02493_amd import Helmholtz

    H = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c64", damping_cells=case.damping_cells,
                  shift=shift)
    H.set_phase(case.phi)
    H.solve(g, tol=tol, maxit=400, mode=1)  # warm-up (graph capture)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, its, rr, _ = H.solve(g, tol=tol, maxit=2000, mode=1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    H.close()
    return {"shift": shift, "tol": tol, "iterations": its, "relres": rr, "seconds": round(dt, 4)}


def bench_comparison(case, g, maxit: int = 600):
    """The comparison preconditioners of Section 4.3.1 on the same 4096^2 workload and the
    same kernels, FP32+refinement under a bounded iteration count: CSL (cycle for the
    operator shifted by 0.5 k^2 n^2, no ADR correction) and Wave-Ray (eight plane-wave
    ray corrections instead of the eikonal phase)."""
    import torch

    from paper_2404_02493_amd import Helmholtz

    out = {}
    for name, kw in (("csl", dict(cycle_shift=0.5, adr_steps=0)), ("wave_ray", {})):
        H = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c64",
                      damping_cells=case.damping_cells, **kw)
        if name == "wave_ray":
            H.set_rays(8)
        else:
            H.set_phase(case.phi)
        H.solve(g, tol=1e-6, maxit=5, mode=1)  # graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, rr, _ = H.solve(g, tol=1e-6, maxit=maxit, mode=1)
        torch.cuda.synchronize()
        out[name] = {"iterations": its, "relres": rr, "seconds": round(time.perf_counter() - t0, 3),
                     "converged": rr < 1e-6, "maxit": maxit}
        H.close()
    return out


def bench_eikonal(case, g, maxit: int = 1000):
    """The travel-time phase computed on the device (helm_eikonal: factored eikonal
    equation by fast sweeping, product-rule ADR coefficients) against the host
    fast-marching helper that prepares the headline phase, and the FP32+refinement
    solve with that phase."""
    import numpy as np
    import torch

    import helm_inputs as hi
    from paper_2404_02493_amd import Helmholtz

    src = np.asarray(case.sources, dtype=np.float64)
    t0 = time.perf_counter()
    hi.fmm_phase(case.velocity, src)
    host_s = time.perf_counter() - t0
    H = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c64", damping_cells=case.damping_cells)
    H.eikonal(src, max_rounds=1000, tol=1e-10)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rounds, change = H.eikonal(src, max_rounds=1000, tol=1e-10)
    torch.cuda.synchronize()
    dev_s = time.perf_counter() - t0
    H.solve(g, tol=1e-6, maxit=5, mode=1)  # graph capture
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, its, rr, _ = H.solve(g, tol=1e-6, maxit=maxit, mode=1)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    H.close()
    n = case.n
    return {"sources": int(src.shape[0]), "rounds": rounds, "last_change": change, "seconds": round(dev_s, 4),
            "node_updates_per_s": round(4.0 * rounds * n * n / dev_s, 1),
            "host_fast_marching_seconds": round(host_s, 3),
            "solve_iterations": its, "solve_relres": rr, "solve_seconds": round(solve_s, 3), "maxit": maxit}


def bench_rect(seed: int, maxit: int = 3000):
    """A non-square domain (Section 4.3.2): the layered medium on 4096 columns x 1024 rows
    at the headline spacing and frequency, FP32+refinement to 1e-6 with tuned launch
    shapes, in both orientations (the tall one is the transposed problem: same medium,
    phase and source turned by 90 degrees)."""
    import numpy as np
    import torch

    import helm_inputs as hi
    from paper_2404_02493_amd import Helmholtz

    case = hi.make_case("layered4096x1024", seed=seed)
    out = {"workload": "layered4096x1024 (4096 columns x 1024 rows, k = 2100, h = 1/4096)",
           "damping_cells": case.damping_cells, "levels": case.levels}
    for name, tr in (("wide", False), ("tall", True)):
        vel, phi, g_np = case.velocity, case.phi, case.g
        if tr:
            vel, phi, g_np = vel.T.copy(), phi.T.copy(), g_np.T.copy()
        H = Helmholtz(vel, case.k, levels=case.levels, precision="c64", damping_cells=case.damping_cells)
        H.set_phase(phi)
        H.tune(cache=os.path.join(ROOT, "paper_2404_02493_amd", "tuning.json"))
        g = torch.as_tensor(g_np).to("cuda:0")
        H.solve(g, tol=1e-6, maxit=5, mode=1)  # graph capture
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, its, rr, _ = H.solve(g, tol=1e-6, maxit=maxit, mode=1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        H.close()
        out[name] = {"shape": list(vel.shape), "iterations": its, "relres": rr, "seconds": round(dt, 4),
                     "ms_per_iteration": round(1e3 * dt / max(its, 1), 3),
                     "node_iterations_per_s": round(float(np.prod(vel.shape)) * its / dt, 1)}
    return out


def copy_rate(reps: int = 10) -> dict:
    """Rate of a plain device copy of 2 GiB (complex64, far above the 256 MB last-level
    cache), read plus written bytes per second: what a streaming kernel reaches on this
    HBM, beside the published peak the rooflines use."""
    import torch

    n = 1 << 28
    x = torch.ones(n, dtype=torch.complex64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    nbytes = 2 * n * x.element_size()
    del x, y
    return {"GBs": round(nbytes / s / 1e9, 1), "bytes_per_copy": nbytes, "us_per_copy": round(1e6 * s, 1),
            "note": "torch device copy of 2 GiB complex64; read plus written bytes"}


def copy_probe(reps: int = 5):
    """A plain device copy of 4096^2 complex64 values (128 MiB read + 128 MiB written per
    dispatch), the known-size reference for the FETCH_SIZE / WRITE_SIZE counters."""
    import numpy as np
    import torch

    from paper_2404_02493_amd import Helmholtz

    n = 4096
    H = Helmholtz(np.ones((n, n)), 100.0, levels=3, precision="c64", adr_steps=0)
    x = torch.ones((n, n), dtype=torch.complex64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(reps):
        H.debug_op(12, 1, x, None, y)
    torch.cuda.synchronize()
    log(f"copy probe: {reps} dispatches of {n * n * 8 / 2**20:.0f} MiB read + written")
    H.close()


def batch_measure(seed: int, lanes: int, tol: float, maxit: int, steps: int = 1, warmup: int = 1,
                  one_lane: bool = False, tune: bool = True):
    """Mixed batch: 64 problems with n drawn from {256, 512, 1024}, k = 0.625 n, own random
    medium, 1-4 sources with a multi-source fast-marching phase; every problem solved to
    tol with FP32 cycles inside FP64 refinement.  Per size: one problem
    solved alone with per-launch timing gives its algorithmic bytes over its kernel time, with
    the untuned default launch shapes (those the batch runs with) and with the tuner's choice
    for that size."""
    import numpy as np
    import torch

    import helm_inputs as hi
    from paper_2404_02493_amd import HelmholtzBatch

    t = time.perf_counter()
    cases = hi.make_batch(seed)
    log(f"batch inputs ready in {time.perf_counter() - t:.1f} s")
    probs = [dict(velocity=c.velocity, k=c.k, levels=c.levels, damping_cells=c.damping_cells, phi=c.phi)
             for c in cases]
    gs = [torch.as_tensor(c.g).to("cuda:0") for c in cases]
    sizes = sorted({c.n for c in cases})
    res = {}
    tuned, per_size = {}, {}
    for nl in ([lanes, 1] if one_lane else [lanes]):
        t = time.perf_counter()
        B = HelmholtzBatch(probs, precision="c64", lanes=nl)
        torch.cuda.synchronize()
        log(f"lanes={nl}: setup of {len(cases)} contexts in {time.perf_counter() - t:.1f} s")
        if not per_size:
            # one problem of each size alone: untuned default shapes, then the tuner's choice
            for n in sizes:
                p = next(q for q, c in enumerate(cases) if c.n == n)
                P = B.problem(p)
                per_size[str(n)] = {"problems": sum(1 for c in cases if c.n == n)}
                for label in (("default", "tuned") if tune else ("default",)):
                    if label == "tuned":
                        tn = P.tune()
                        tuned[n] = {"sstep_rows": tn["sstep_rows"], "fgmres_blocks": tn["fgmres_blocks"]}
                    P.solve(gs[p], tol=tol, maxit=maxit, mode=1)
                    P.profile_begin()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, its1, _, _ = P.solve(gs[p], tol=tol, maxit=maxit, mode=1)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    prof = P.profile_end()
                    ms = sum(k["ms"] for k in prof["kernels"])
                    by = sum(k["bytes"] for k in prof["kernels"])
                    per_size[str(n)][label] = {
                        "iterations": its1, "seconds_profiled": round(dt, 4), "kernel_ms": round(ms, 3),
                        "algorithmic_GBs_in_kernels": round(by / (ms * 1e-3) / 1e9, 1),
                        "kernel_busy_frac": round(ms * 1e-3 / dt, 3)}
                P.set_tuning({"sstep_rows": {}, "fgmres_blocks": 0})
        for w in range(warmup):
            B.solve(gs, tol=tol, maxit=maxit, mode=1)
        torch.cuda.synchronize()
        times = []
        for s_ in range(steps):
            t0 = time.perf_counter()
            us, its, rr, st = B.solve(gs, tol=tol, maxit=maxit, mode=1)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            log(f"lanes={nl} step {s_}: {times[-1]:.3f} s, iterations {int(its.sum())}, "
                f"max relres {rr.max():.2e}, statuses {sorted(set(st.tolist()))}")
        res[nl] = (float(np.mean(times)), its, rr, st)
        classes = B.classes()
        B.close()
    tb, its, rr, st = res[lanes]
    out = {"problems_per_s": round(len(cases) / tb, 3), "seconds": round(tb, 3), "problems": len(cases),
           "fine_points": sum(c.n * c.n for c in cases), "lanes": lanes,
           "sizes": {str(n): sum(1 for c in cases if c.n == n) for n in sizes},
           "all_converged": bool(np.all(st == 0)), "total_iterations": int(its.sum()),
           "max_relres": float(rr.max()), "per_size": per_size, "tuned": {str(k): v for k, v in tuned.items()},
           "lockstep_classes": int(len(set(classes.tolist()) - {-1})),
           "problems_in_lockstep": int(np.sum(classes >= 0))}
    if one_lane:
        t1 = res[1][0]
        out["one_lane"] = {"seconds": round(t1, 3), "problems_per_s": round(len(cases) / t1, 3),
                           "speedup_of_lanes": round(t1 / tb, 2)}
    return out


def bench_batch(args):
    """--workload batch64: the mixed batch as the main line (value = problems per second)."""
    r = batch_measure(args.seed, args.lanes, args.tol, args.maxit, args.steps, args.warmup, one_lane=True)
    out = {
        "metric": "problems/s, 64-problem mixed batch (n in {256,512,1024}, k=0.625n), FP32+refine to 1e-6",
        "value": r["problems_per_s"], "unit": "problems/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * r["seconds"], 2), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch64", "problems": r["problems"], "fine_points": r["fine_points"],
                   "lanes": args.lanes, "sizes": r["sizes"], "seed": args.seed, "tol": args.tol},
        "batch": r,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="layered4096")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--maxit", type=int, default=3000)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--lanes", type=int, default=4)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the side measurements (sharp medium, shifted equation, batch)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="time only the adjoint of 10 unrolled cycles at 1024^2 and print its record")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain copy kernel of known size (reference for memory counters)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2404_02493_amd", "tuning.json"),
                    help="JSON cache of measured launch shapes ('none' = built-in defaults)")
    ap.add_argument("--tuning", default=None,
                    help="launch shapes to apply to the FP32-cycle context instead of measuring or "
                         "reading a cache (the JSON of helm_set_tuning), e.g. for runs under a profiler")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the solver has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch64":
        bench_batch(args)
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": bench_adjoint()}), flush=True)
        return

    import numpy as np
    import torch

    import helm_inputs as hi
    from paper_2404_02493_amd import Helmholtz

    dev = "cuda:0"
    log(f"generating workload {args.workload} seed {args.seed}")
    t = time.perf_counter()
    case = hi.make_case(args.workload, seed=args.seed)
    log(f"inputs ready in {time.perf_counter() - t:.1f} s (n={case.n}, k={case.k}, L={case.levels})")
    g = torch.as_tensor(case.g).to(dev)

    log("setup FP32-cycle context")
    H32 = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c64", damping_cells=case.damping_cells)
    H32.set_phase(case.phi)
    tuning = None
    if args.tuning is not None:
        H32.set_tuning(args.tuning)
        tuning = H32.get_tuning()
        log(f"tuning given: sstep_rows {tuning['sstep_rows']}, fgmres_blocks {tuning['fgmres_blocks']}")
    elif args.tune_cache != "none":
        t = time.perf_counter()
        tuning = H32.tune(cache=args.tune_cache)
        log(f"tuning ({time.perf_counter() - t:.1f} s): sstep_rows {tuning['sstep_rows']}, "
            f"fgmres_blocks {tuning['fgmres_blocks']}")

    def run32():
        u = torch.zeros_like(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, its, rr, _ = H32.solve(g, u, tol=args.tol, maxit=args.maxit, mode=1)
        torch.cuda.synchronize()
        return u, its, rr, time.perf_counter() - t0

    for w in range(args.warmup):
        _, its, rr, dt = run32()
        log(f"warmup {w}: FP32+refinement {its} iterations, relres {rr:.2e}, {dt:.3f} s")
    times, iters = [], []
    torch.cuda.synchronize()
    for s in range(args.steps):
        u32, its, rr32, dt = run32()
        times.append(dt)
        iters.append(its)
        log(f"step {s}: FP32+refinement {its} iterations, relres {rr32:.2e}, {dt:.3f} s")
    t32 = float(np.mean(times))

    prof32 = None
    if not args.no_profile:
        H32.profile_begin()
        _, its_p, _, dtp = run32()
        prof32 = H32.profile_end()
        log(f"profiled FP32 step: {dtp:.3f} s")

    fp64 = None
    prof64 = None
    if not args.no_fp64:
        log("setup FP64 context")
        H64 = Helmholtz(case.velocity, case.k, levels=case.levels, precision="c128",
                        damping_cells=case.damping_cells)
        H64.set_phase(case.phi)
        if args.tune_cache != "none":
            H64.tune(cache=args.tune_cache)
        u64 = torch.zeros_like(g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u64, its64, rr64, _ = H64.solve(g, u64, tol=args.tol, maxit=args.maxit, mode=0)
        torch.cuda.synchronize()
        t64 = time.perf_counter() - t0
        diff = (torch.linalg.norm(u32 - u64) / torch.linalg.norm(u64)).item()
        log(f"FP64 solve: {its64} iterations, relres {rr64:.2e}, {t64:.3f} s; |u32-u64|/|u64| = {diff:.2e}")
        fp64 = {"seconds": t64, "iterations": its64, "relres": rr64, "rel_diff_fp32_vs_fp64": diff}
        if not args.no_profile:
            H64.profile_begin()
            u64b = torch.zeros_like(g)
            H64.solve(g, u64b, tol=args.tol, maxit=args.maxit, mode=0)
            prof64 = H64.profile_end()
        H64.close()

    roofline = None
    summary = {}
    if prof32:
        ks = prof32["kernels"]
        tot_ms = sum(k["ms"] for k in ks)
        tot_bytes = sum(k["bytes"] for k in ks)
        top = ks[0]
        achieved = top["bytes"] / (top["ms"] * 1e-3) / 1e9
        from paper_2404_02493_amd.traffic import find as find_traffic

        # measured HBM bytes per launch (FETCH_SIZE + WRITE_SIZE counter runs, scaled by a
        # plain copy of known size), as a rate over the same average launch time
        tbytes = find_traffic(os.path.join(ROOT, "profiles"), top["name"])
        avg_s = 1e-3 * top["ms"] / top["launches"]
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": round(tbytes / avg_s / 1e9, 1) if tbytes else None,
                    "kernel": top["name"], "launches": top["launches"],
                    "avg_launch_us": round(1e6 * avg_s, 2),
                    "bytes_per_launch": top["bytes"] / top["launches"],
                    "traffic_bytes_per_launch": tbytes}
        summary = {"kernel_ms_total": round(tot_ms, 3), "algorithmic_GB": round(tot_bytes / 1e9, 3),
                   "effective_GBs_in_kernels": round(tot_bytes / (tot_ms * 1e-3) / 1e9, 1),
                   "top_kernels": [{"name": k["name"], "launches": k["launches"], "ms": round(k["ms"], 3),
                                    "GBs": round(k["bytes"] / max(k["ms"], 1e-9) / 1e6, 1)} for k in ks[:8]]}

    roofline_hbm = hbm_rooflines(prof32["kernels"]) if prof32 else None
    copy_ref = copy_rate()
    log(f"plain copy: {copy_ref['GBs']} GB/s")

    shifted = sharp = batch = comparison = eikonal = rect = None
    if not args.no_extras:
        log("shifted equation (relative shift 0.01) to 1e-7")
        shifted = bench_shifted(case, g)
        log(f"shifted: {shifted}")
        log("mixed batch of 64 problems")
        batch = batch_measure(args.seed, args.lanes, args.tol, args.maxit)
        log(f"batch: {batch['problems_per_s']} problems/s, per size {batch['per_size']}")
        log("comparison preconditioners (CSL, Wave-Ray), at most 600 iterations")
        comparison = bench_comparison(case, g)
        log(f"comparison: {comparison}")
        log("unsmoothed layered medium, at most 1000 iterations")
        sharp = bench_sharp(args.seed)
        log(f"sharp: {sharp}")
        log("travel-time phase on the device (factored eikonal) and its solve")
        eikonal = bench_eikonal(case, g)
        log(f"eikonal: {eikonal}")
        log("non-square domain 4096 x 1024, both orientations")
        rect = bench_rect(args.seed)
        log(f"rect: {rect}")

    adjoint = None
    if not args.no_adjoint:
        log("timing the adjoint of 10 unrolled cycles at 1024^2")
        adjoint = bench_adjoint()
        log(f"adjoint: {adjoint}")

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on one FP64 FGMRES iteration")
        cpu = cpu_baseline(case, fp64["iterations"] if fp64 else int(np.mean(iters)))
        log(f"CPU oracle sample {cpu['sample_seconds']:.1f} s on {cpu['cores']} threads")

    out = {
        "metric": "time to 1e-6 rel. residual + HBM GB/s, 4096^2 k~2100, FP32+refine vs FP64",
        "value": round(t32, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * t32, 2),
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": case.n, "k": case.k, "levels": case.levels,
                   "seed": args.seed, "medium": case.meta["medium"],
                   "medium_detail": "8 layers + 20 elliptical inclusions (+-30%), c in [1.5, 4.5]"
                                    + (f", Gaussian-smoothed with sigma {case.meta['smooth']}"
                                       if case.meta.get("smooth") else ", not smoothed"),
                   "smooth": case.meta.get("smooth", 0.0), "damping_cells": case.damping_cells,
                   "phase": "first-order fast marching",
                   "solver": "FP64 iterative refinement around FP32 FGMRES(20), FP32 Wave-ADR cycles (coarsest FP64)",
                   "adr_steps": 8, "tol": args.tol},
        "iterations": int(np.mean(iters)),
        "relres": rr32,
        "fp64": fp64,
        "roofline": roofline,
        "roofline_hbm": roofline_hbm,
        "hbm_copy": copy_ref,
        "cpu_baseline": cpu,
        "shifted": shifted,
        "sharp": sharp,
        "batch64": batch,
        "comparison": comparison,
        "eikonal_phase": eikonal,
        "non_square": rect,
        "profile_fp32": summary,
        "adjoint": adjoint,
        "tuning": {k: v for k, v in tuning.items() if k != "timings_ms"} if tuning else None,
    }
    if prof64:
        ks = prof64["kernels"]
        out["profile_fp64"] = {"kernel_ms_total": round(sum(k["ms"] for k in ks), 3),
                               "top_kernels": [{"name": k["name"], "launches": k["launches"], "ms": round(k["ms"], 3),
                                                "GBs": round(k["bytes"] / max(k["ms"], 1e-9) / 1e6, 1)}
                                               for k in ks[:5]]}
    print(json.dumps(out), flush=True)
    H32.close()


if __name__ == "__main__":
    main()
