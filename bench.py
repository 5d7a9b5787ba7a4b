"""Benchmark of the OBK-RCM sweep on one MI355X.

Default workload: the 1024x1024 5-point stencil (1,048,576 rows, 5,238,784
nonzeros) under a random symmetric permutation, delta = 0.1, FP64.  The plan
(RCM, norms, cosines, grouping, relayout) is built once and timed on its own;
a timed step is one full sweep over every group.  The iterate stays in HBM
for the whole timed region.

Prints one JSON line (see the keys below).  ``--gpus`` above 1 is refused:
this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, published


def sweep_bytes(n: int, m: int, nnz: int, touched: int | None = None, sv: int = 8, sx: int = 8) -> int:
    """Algorithmic bytes of one sweep: A read once (value + int32 column),
    int32 row offsets, f and 1/||a||^2 per row, x read and written once."""
    return nnz * (sv + 4) + m * (4 + sv + sv) + 2 * n * sx


def cpu_baseline_sweeps(system, delta: float, budget_s: float = 12.0) -> dict:
    """The FP64 oracle timed on the host: plan once, then sweeps until the time
    budget is used (single thread)."""
    import oracle
    t0 = time.perf_counter()
    pl = oracle.plan_system(system, delta)
    plan_s = time.perf_counter() - t0
    x = np.zeros(system.n)
    done, t1 = 0, time.perf_counter()
    while True:
        x = oracle.sweep(pl, x, 1)
        done += 1
        el = time.perf_counter() - t1
        if el >= budget_s or done >= 2000:
            break
    return {"value": done / el, "unit": "sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} FP64 sweeps of the full workload after a {plan_s:.1f} s oracle plan "
                      f"({el:.1f} s of sweeps, one thread)"}


def bench_stencil(args) -> dict:
    import torch
    import synth
    import paper_2401_00672_amd as obk

    grid = args.grid
    s = synth.c2(grid=grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = obk.plan_system(s, args.delta)
    plan_s = time.perf_counter() - t0
    st = P.stats()
    g, ng = P.groups()
    m = int((g >= 0).sum())
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    if args.warmup > 0:
        P.sweep_device(x, args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    P.sweep_device(x, args.steps)          # the K timed sweeps, replayed from captured graphs
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    B = sweep_bytes(s.n, m, s.nnz)
    achieved = B / (ms * 1e-3) / 1e9
    res = {
        "metric": "sweeps/s + GB/s vs HBM peak",
        "value": 1000.0 / ms,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"stencil-{grid}x{grid}-symperm-rcm-delta{args.delta}-fp64-sweep",
                   "n": s.n, "nnz": s.nnz, "groups": ng, "bandwidth_after_rcm": st["bandwidth"],
                   "algorithmic_bytes_per_sweep": B},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole sweep (all launches of one sweep)"},
        "nnz_per_s": s.nnz * 1000.0 / ms,
        "plan_seconds": plan_s,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_sweeps(s, args.delta, args.cpu_budget)
    P.free()
    return res


def copy_calibration(mib: int = 256, reps: int = 5) -> dict:
    """A plain device copy of known size, for scaling the HBM byte counters
    (FETCH_SIZE / WRITE_SIZE) that a profiler reports per dispatch."""
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    return {"calibration": "copy", "bytes_read_per_copy": n * 8, "bytes_written_per_copy": n * 8,
            "kib_per_copy": n * 8 / 1024, "reps": reps}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--delta", type=float, default=0.1)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a 256 MiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        print(json.dumps(copy_calibration()), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design note, not a measured path.", file=sys.stderr)
        return 2
    res = bench_stencil(args)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
