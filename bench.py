"""Benchmark of the OBK-RCM sweep on one MI355X.

Default workload: the 1024x1024 5-point stencil (1,048,576 rows, 5,238,784
nonzeros) under a random symmetric permutation, delta = 0.1, FP64.  The plan
(RCM, norms, cosines, grouping, relayout) is built once and timed on its own;
a timed step is one full sweep over every group.  The iterate stays in HBM
for the whole timed region.

Prints one JSON line (see the keys below).  ``--gpus`` above 1 is refused:
the library runs one GPU per process, and this benchmark measures one.
"""
from __future__ import annotations

import argparse
import hashlib
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


REAL_SWEEP_SOURCES = ("obk_sweep_tiles.h", "obk_tile.h")
BANDED_SOURCES = ("obk_slab.hip",)
COMPLEX_SWEEP_SOURCES = ("obk_complex.hip", "obk_sweep_tiles.h", "obk_tile.h")


def _kernel_source_sha(files=REAL_SWEEP_SOURCES) -> str:
    """Hash of the sweep kernel sources: counter figures recorded for an older
    kernel are not reported."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2401_00672_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_traffic(kernel: str, workload: str, files=REAL_SWEEP_SOURCES, key: str = "hbm_bytes_per_launch"):
    """HBM bytes per launch (or per sweep, key "hbm_bytes_per_sweep") of
    `kernel` from the committed rocprofv3 counter summary (FETCH_SIZE and
    WRITE_SIZE, calibrated against a plain copy), or None when no summary
    matches the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != _kernel_source_sha(files) or kv.get("kernel") != kernel:
        return None
    try:
        return float(kv[key])
    except (KeyError, ValueError):
        return None


def cpu_baseline_sweeps(system, delta: float, budget_s: float = 12.0) -> dict:
    """The FP64 oracle timed on the host: plan once (its conflict pass on all
    threads), then sweeps until the time budget is used -- the plain sweep on
    one thread, and the threaded sweep (rows of a group, then touched
    columns, on every OpenMP thread; the same iterate) on all threads."""
    import oracle
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    pl = oracle.plan_system(system, delta)
    plan_s = time.perf_counter() - t0
    x = np.zeros(system.n)
    done, t1 = 0, time.perf_counter()
    while True:
        x = oracle.sweep(pl, x, 1)
        done += 1
        el = time.perf_counter() - t1
        if el >= budget_s / 2 or done >= 2000:
            break
    one = done / el
    ts = oracle.ThreadedSweep(pl)
    xm = np.zeros(system.n)
    ts.sweep(xm, 1)
    dm, t2 = 0, time.perf_counter()
    while True:
        ts.sweep(xm, 1)
        dm += 1
        em = time.perf_counter() - t2
        if em >= budget_s / 2 or dm >= 20000:
            break
    ts.close()
    return {"value": dm / em, "unit": "sweeps/s", "cores": threads, "kind": "oracle",
            "one_thread": {"value": one, "unit": "sweeps/s", "cores": 1},
            "sample": f"full workload after a {plan_s:.1f} s oracle plan: {dm} FP64 sweeps on {threads} threads "
                      f"({em:.1f} s), {done} on one thread ({el:.1f} s)"}


def bench_stencil(args) -> dict:
    import torch
    import synth
    import paper_2401_00672_amd as obk

    grid = args.grid
    s = synth.c2(grid=grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = obk.plan_system(s, args.delta, sweep_kernel=args.sweep_kernel)
    plan_s = time.perf_counter() - t0
    st = P.stats()
    eng = P.engine()
    g, ng = P.groups()
    m = int((g >= 0).sum())
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    if args.warmup > 0:
        P.sweep_device(x, args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # a few untimed sweeps keep the device busy while the host submits the
    # timed call, so that the events bracket the K sweeps and not the host's
    # submission latency
    P.sweep_device(x, 8)
    e0.record(stream)
    P.sweep_device(x, args.steps)          # the K timed sweeps (one persistent launch, or captured graphs)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    B = sweep_bytes(s.n, m, s.nnz)
    sweep_gbs = B / (ms * 1e-3) / 1e9
    # the sweep's kernels, timed per launch with HIP events on the launch
    # stream (eager sweeps); the roofline unit is one sweep: the
    # algorithmic bytes of sweep_bytes() over the summed kernel time of one
    # sweep
    prof = P.sweep_profile(x, args.profile_sweeps)
    sweep_kernel_s = sum(k["seconds"] for k in prof) / args.profile_sweeps
    launches_per_sweep = sum(k["launches"] for k in prof) / args.profile_sweeps
    achieved = B / sweep_kernel_s / 1e9
    if eng["engine"] == "banded":
        # one launch runs every sweep of a call: the summary is per sweep
        traffic = kernel_traffic("k_slab_sweeps", "stencil_banded", BANDED_SOURCES, "hbm_bytes_per_sweep")
    else:
        traffic = kernel_traffic("+".join(k["name"] for k in prof), "stencil")
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
                   "algorithmic_bytes_per_sweep": B, "engine": eng},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "+".join(k["name"] for k in prof), "unit_of_work": "one sweep",
                     "algorithmic_bytes_per_sweep": B, "kernel_us_per_sweep": sweep_kernel_s * 1e6,
                     "launches_per_sweep": launches_per_sweep, "sweeps_profiled": args.profile_sweeps,
                     "traffic_unit": "bytes/sweep" if eng["engine"] == "banded" else "bytes/launch"},
        "sweep_effective": {"formula_bytes_per_sweep": B, "achieved_gbs": sweep_gbs,
                            "frac": sweep_gbs / HBM_PEAK_GBS},
        # per kernel, with the implementation's own bytes per launch (A is read
        # in both phases, x once per group), not the algorithmic bytes
        "kernels": [{"name": k["name"], "launches": k["launches"], "avg_us": k["seconds"] / k["launches"] * 1e6,
                     "implementation_bytes_per_launch": k["bytes"] / k["launches"],
                     "implementation_gbs": k["bytes"] / k["seconds"] / 1e9} for k in prof],
        "nnz_per_s": s.nnz * 1000.0 / ms,
        "plan_seconds": plan_s,
    }
    P.free()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_sweeps(s, args.delta, args.cpu_budget)
    if args.compact_batch > 0:
        # the batched FP32 + refinement form at a stated compact size, so that
        # every run of the default line also reports solves/s to 1e-10
        res["batched_compact"] = run_batched(args.compact_batch, args.delta, args.inner, args.check_every, 4)
    return res


def cpu_baseline_block(system, k: int, thr: float, budget_s: float = 12.0) -> dict:
    """The oracle's block form timed on the host: plan once, then block
    projections (dense pseudo-inverse of each block) in sweep order until the
    time budget is used; sweeps/s = projections/s / k."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    except Exception:
        cores = 1
    t0 = time.perf_counter()
    bp = oracle.block_plan(system.n, system.row_ptr, system.col, system.val, system.f, k, thr)
    plan_s = time.perf_counter() - t0
    order = [t for pr in bp.pairs for t in pr] + list(bp.nclass)
    x = np.zeros(system.n)
    done, t1 = 0, time.perf_counter()
    while True:
        x = oracle.block_project(bp, order[done % k], x)
        done += 1
        el = time.perf_counter() - t1
        if el >= budget_s or done >= 20 * k:
            break
    return {"value": done / k / el, "unit": "sweeps/s", "cores": cores, "kind": "oracle",
            "sample": f"{done} block projections ({done / k:.2f} sweeps) of the full workload after a "
                      f"{plan_s:.1f} s oracle plan ({el:.1f} s; numpy pinv on {cores} BLAS threads)"}


def bench_block(args) -> dict:
    """Block form of Algorithm 4 on a banded system of the paper's size class:
    a 5-point stencil under a random symmetric permutation, k uniform blocks
    after RCM, thr = 0.02 (the paper's global threshold).  A timed step is one
    sweep (every Oclass pair, then Nclass), each block projected exactly:
    from its banded Cholesky factor of A_t A_t^T (--block-solver direct, the
    default) or by in-kernel conjugate gradients (--block-solver cg); all
    sweeps of the timed region run in one launch."""
    import torch
    import synth
    import paper_2401_00672_amd as obk
    grid, k, thr = args.block_grid, args.block_k, args.block_thr
    s = synth.c2(grid=grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = obk.plan_system(s, thr, block_k=k, block_wgs=args.block_wgs, block_solver=args.block_solver)
    plan_s = time.perf_counter() - t0
    info = P.blocks()
    x = torch.zeros(s.n, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    if args.warmup > 0:
        P.sweep_device(x, args.warmup)
    torch.cuda.synchronize()
    it0 = int(P.blocks()["cg_iters"].sum())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    P.sweep_device(x, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    iters = (int(P.blocks()["cg_iters"].sum()) - it0) / args.steps
    prof = P.sweep_profile(x, args.profile_sweeps)[0]
    achieved = prof["bytes"] / prof["seconds"] / 1e9
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
        "config": {"workload": f"block-form-stencil-{grid}x{grid}-symperm-rcm-k{k}-thr{thr}-fp64-sweep",
                   "n": s.n, "nnz": s.nnz, "k": k, "pairs": len(info["pairs"]), "nclass": len(info["nclass"]),
                   "workgroups": args.block_wgs or "auto", "solver": args.block_solver,
                   "direct_blocks": int(info["direct"].sum()),
                   "factor_bandwidth_max": int(info["factor_bandwidth"].max()),
                   "cg_iterations_per_sweep": iters},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": prof["name"],
                     "avg_launch_us": prof["seconds"] / prof["launches"] * 1e6,
                     "algorithmic_bytes_per_launch": prof["bytes"] / prof["launches"],
                     "sweeps_per_launch": args.profile_sweeps, "traffic_unit": "bytes/launch"},
        "us_per_cg_iteration": ms * 1e3 / iters if iters > 0 else None,
        "plan_seconds": plan_s,
    }
    zn, nn = P.block_zn_nn()
    P.free()
    # block-count criteria of Section 3.6 over the paper's range k < 20
    t1 = time.perf_counter()
    best, scores = obk.select_block_k(s, thr, list(range(2, 20)))
    res["k_selection"] = {"candidates": "2..19", "chosen": best, "seconds": time.perf_counter() - t1,
                          "benched_k_zn": zn, "benched_k_nn": nn}
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_block(s, k, thr, args.cpu_budget)
    return res


def cpu_baseline_complex(system, delta: float, budget_s: float = 12.0) -> dict:
    """The oracle's complex path timed on the host: plan once, then complex
    sweeps until the time budget is used (single thread)."""
    import oracle
    t0 = time.perf_counter()
    pl = oracle.plan_system_complex(system, delta)
    plan_s = time.perf_counter() - t0
    x = np.zeros(system.n, dtype=np.complex128)
    done, t1 = 0, time.perf_counter()
    while True:
        x = oracle.sweep_complex(pl, x, 1)
        done += 1
        el = time.perf_counter() - t1
        if el >= budget_s or done >= 2000:
            break
    return {"value": done / el, "unit": "sweeps/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} complex FP64 sweeps of the full workload after a {plan_s:.1f} s oracle plan "
                      f"({el:.1f} s of sweeps, one thread)"}


def bench_complex(args) -> dict:
    """Complex counterpart of the default line (the paper's kim1 case): the
    1024x1024 stencil pattern with complex values under a random symmetric
    permutation, delta = 0.1, complex FP64 sweeps."""
    import torch
    import synth
    import paper_2401_00672_amd as obk
    grid = args.grid
    s = synth.c2z(grid=grid)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = obk.plan_system(s, args.delta)
    plan_s = time.perf_counter() - t0
    st = P.stats()
    g, ng = P.groups()
    m = int((g >= 0).sum())
    x = torch.zeros(s.n, dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    if args.warmup > 0:
        P.sweep_device(x, args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    P.sweep_device(x, args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    B = sweep_bytes(s.n, m, s.nnz, sv=16, sx=16)
    prof = P.sweep_profile(x, args.profile_sweeps)
    dom = max(prof, key=lambda k: k["seconds"])
    dom_avg_s = dom["seconds"] / dom["launches"]
    dom_bytes = dom["bytes"] / dom["launches"]
    achieved = dom_bytes / dom_avg_s / 1e9
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
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": f"complex-stencil-{grid}x{grid}-symperm-rcm-delta{args.delta}-fp64-sweep",
                   "n": s.n, "nnz": s.nnz, "groups": ng, "bandwidth_after_rcm": st["bandwidth"],
                   "algorithmic_bytes_per_sweep": B},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": kernel_traffic(dom["name"], "complex_stencil", COMPLEX_SWEEP_SOURCES),
                     "kernel": dom["name"], "avg_launch_us": dom_avg_s * 1e6, "algorithmic_bytes_per_launch": dom_bytes,
                     "launches_profiled": dom["launches"], "traffic_unit": "bytes/launch"},
        "sweep_effective": {"formula_bytes_per_sweep": B, "achieved_gbs": B / (ms * 1e-3) / 1e9,
                            "frac": B / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "kernels": [{"name": k["name"], "launches": k["launches"], "avg_us": k["seconds"] / k["launches"] * 1e6,
                     "gbs": k["bytes"] / k["seconds"] / 1e9} for k in prof],
        "plan_seconds": plan_s,
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline_complex(s, args.delta, args.cpu_budget)
    P.free()
    return res


def _log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def _oracle_errors(systems, xs, delta: float, inner: int, tol: float = 1e-10) -> list:
    """Relative error of batched FP32 + FP64-refinement results against the
    oracle's FP64 run of the same refinement schedule (O11), per system."""
    import oracle
    out = []
    for s, x in zip(systems, xs):
        pl = oracle.plan_system(s, delta)
        xt, _, _ = oracle.refine(pl, inner, 200, tol)
        x64 = oracle.unpermute(pl.p, xt)
        out.append(float(np.linalg.norm(x - x64) / np.linalg.norm(x64)))
    return out


def run_batched(count: int, delta: float, inner: int, check_every: int, oracle_systems: int) -> dict:
    """`count` systems of the batched family (n log-uniform in [1e3, 2e5],
    4..16 nnz/row, the first `count` of its 512 sizes), row-dominant
    companion: all solved to relative residual 1e-10 by batched FP32 sweeps +
    FP64 refinement (autotuned launch schedule) against a loop of plain FP64
    solves, one system at a time, on the same plans.  Errors are stated
    against the oracle's FP64 refinement for the `oracle_systems` smallest."""
    import torch
    import synth
    import paper_2401_00672_amd as obk
    sizes = synth.c4_sizes(512)[:count]
    plans, keep = [], {}
    order = [int(i) for i in np.argsort(sizes)[:oracle_systems]]
    t0 = time.perf_counter()
    for i, n in enumerate(sizes):
        sy = synth.c4_system(i, n=int(n), companion=True)
        plans.append(obk.plan_system(sy, delta, precision=obk.FP32_IR, inner_sweeps=inner))
        if i in order:
            keep[i] = sy
        if i % 64 == 0:
            _log(f"[c4] planned {i + 1}/{len(sizes)} ({time.perf_counter() - t0:.1f} s)")
    plan_s = time.perf_counter() - t0
    nnz = sum(p.nnz for p in plans)
    tuned, step_s = obk.batch_tune(plans)
    _log(f"[c4] tuned {tuned}: {step_s * 1e3:.2f} ms per refinement step")
    obk.solve_batch(plans, tol=1e-10, maxit=3, opts=tuned)          # warm-up
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    xs, infos = obk.solve_batch(plans, tol=1e-10, maxit=100, opts=tuned)
    t_batch = time.perf_counter() - t1
    ok = sum(1 for i in infos if i.status == "converged")
    steps = max(i.outer_steps for i in infos)
    for p in plans:
        p.set_opts(precision=obk.FP64, check_every=check_every)
    plans[0].solve(maxit=check_every, tol=1e-10)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    base_ok = 0
    for p in plans:
        _, inf = p.solve(maxit=5000, tol=1e-10)
        base_ok += inf.status == "converged"
    t_base = time.perf_counter() - t2
    for p in plans:
        p.free()
    errs = _oracle_errors([keep[i] for i in order], [xs[i] for i in order], delta, inner)
    return {
        "solves_per_s": count / t_batch, "seconds_batched": t_batch, "refinement_steps": steps,
        "converged": ok, "systems": count, "rows": int(sizes.sum()), "nnz": int(nnz), "tuned": tuned,
        "baseline_plain_fp64_loop": {"solves_per_s": count / t_base, "seconds": t_base, "converged": base_ok,
                                     "check_every": check_every},
        "speedup_vs_plain_fp64_loop": t_base / t_batch,
        "error_vs_fp64_oracle": {"systems": [int(sizes[i]) for i in order], "max": max(errs),
                                 "median": float(np.median(errs))},
        "plan_seconds_total": plan_s,
    }


def _make_request(job):
    """Worker: one request system of the serving (c5) or batched (c4) family."""
    import synth
    kind, i, n = job
    return synth.c5_system(i, n=n) if kind == "c5" else synth.c4_system(i, n=n, companion=True)


def make_requests(kind: str, sizes, workers: int) -> list:
    """The systems of `sizes`, generated in order by `workers` processes
    (spawned: none of them touches the GPU)."""
    import multiprocessing as mp
    jobs = [(kind, i, int(n)) for i, n in enumerate(sizes)]
    if workers <= 1 or len(jobs) < 64:
        return [_make_request(j) for j in jobs]
    out = []
    with mp.get_context("spawn").Pool(workers) as pool:
        for s in pool.imap(_make_request, jobs, chunksize=8):
            out.append(s)
            if len(out) % 512 == 0:
                _log(f"[{kind}] generated {len(out)}/{len(jobs)} requests")
    return out


def _oracle_request(job):
    """Worker: the oracle's FP64 plan + solve to `tol` of one request, on one
    thread; returns (seconds, status)."""
    import oracle
    kind, i, n, delta, tol, check_every = job
    oracle.set_threads(1)
    s = _make_request((kind, i, n))
    t0 = time.perf_counter()
    pl = oracle.plan_system(s, delta)
    _, info = oracle.solve_tol(pl, tol, 200000, check_every)
    return time.perf_counter() - t0, info.status


def cpu_baseline_requests(kind: str, sizes, delta: float, check_every: int, budget_s: float, workers: int) -> dict:
    """The oracle solving independent requests in parallel, one request per
    core (FP64 plan + plain FP64 sweeps to relative residual 1e-10, residual
    checked every `check_every` sweeps): the requests are taken in order in
    rounds of `workers` until `budget_s` has passed; solves/s over the rounds
    run."""
    import multiprocessing as mp
    done, statuses = 0, []
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_make_request, [(kind, 0, 500)] * workers)           # start the workers
        t0 = time.perf_counter()
        i = 0
        while i < len(sizes) and time.perf_counter() - t0 < budget_s:
            jobs = [(kind, j, int(sizes[j]), delta, 1e-10, check_every) for j in range(i, min(i + workers, len(sizes)))]
            for sec, st in pool.map(_oracle_request, jobs, chunksize=1):
                statuses.append(st)
            done += len(jobs)
            i += len(jobs)
    wall = time.perf_counter() - t0
    return {"value": done / wall, "unit": "solves/s", "cores": workers, "kind": "oracle",
            "sample": f"the first {done} requests of the workload (n {int(min(sizes[:done]))}..{int(max(sizes[:done]))}), "
                      f"{workers} at a time, one per process on one thread: FP64 oracle plan + sweeps to 1e-10 "
                      f"({sum(1 for x in statuses if x == 'converged')} converged) in {wall:.1f} s"}


def bench_batched(args) -> dict:
    """The batched configuration at its stated size (512 systems)."""
    import synth
    r = run_batched(args.systems, args.delta, args.inner, args.check_every, 8)
    cpu = None
    if not args.no_cpu_baseline:
        _log("[c4] CPU baseline: the oracle on independent systems, one per core")
        cpu = cpu_baseline_requests("c4", synth.c4_sizes(512)[:args.systems], args.delta, args.check_every,
                                    args.cpu_budget, min(16, os.cpu_count() or 1))
    return {
        "metric": "solves/s to rel. residual 1e-10",
        "value": r["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1, "steps": r["refinement_steps"], "warmup": 1,
        "ms_per_step": r["seconds_batched"] * 1e3 / max(r["refinement_steps"], 1),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 sweeps + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"batched-{r['systems']}-systems-n-loguniform-1e3-2e5-4to16nnz-companion-fp32ir",
                   "systems": r["systems"], "rows": r["rows"], "nnz": r["nnz"], "inner_sweeps": args.inner,
                   "tuned": r["tuned"]},
        **{k: r[k] for k in ("converged", "seconds_batched", "baseline_plain_fp64_loop",
                             "speedup_vs_plain_fp64_loop", "error_vs_fp64_oracle", "plan_seconds_total")},
        "cpu_baseline": cpu,
    }


def bench_serving(args) -> dict:
    """Continuous batching of single-system requests: n log-uniform in
    [500, 5e5], 4..16 nnz/row (companion family, to relative residual 1e-10),
    Poisson arrivals.  A first run with every request arriving at t = 0 gives
    the capacity; the reported run uses arrivals at 0.7 x that capacity.  The
    baseline serves the same requests one at a time, first in first out, with
    a plain FP64 plan + solve each (service times measured; queueing computed
    on the same arrival times)."""
    import torch
    import synth
    import paper_2401_00672_amd as obk
    from paper_2401_00672_amd.serve import LibobkBackend, Request, Server, latency_summary

    count = args.requests
    sizes = synth.c5_sizes(8192)[:count]
    t0 = time.perf_counter()
    systems = make_requests("c5", sizes, min(16, os.cpu_count() or 1))
    _log(f"[c5] generated {count} requests in {time.perf_counter() - t0:.1f} s "
         f"(mean n {sizes.mean():.0f}, total nnz {sum(s.nnz for s in systems)})")
    budget = int(args.budget_gib * (1 << 30))
    be = LibobkBackend(delta=args.delta, inner_sweeps=args.inner, planners=args.planners,
                       rcm_engine=args.rcm_engine)
    warm = Server(be, budget, tol=1e-10, planners=args.planners)
    warm.run([Request(0, 0.0, systems[0])])
    torch.cuda.synchronize()

    def serve(arrivals):
        reqs = [Request(i, float(arrivals[i]), systems[i]) for i in range(count)]
        srv = Server(be, budget, tol=1e-10, max_steps=args.max_steps, planners=args.planners,
                     progress=lambda k, n: _log(f"[c5] served {k}/{n}"), progress_every=512,
                     reuse_batch=not args.c5_new_batch_objects)
        ts = time.perf_counter()
        res = srv.run(reqs)
        span = time.perf_counter() - ts
        return res, srv.stats, span

    sat, sat_stats, sat_span = serve(np.zeros(count))
    capacity = count / sat_span
    _log(f"[c5] saturation: {capacity:.1f} solves/s, {sat_stats}")
    rate = 0.7 * capacity
    arrivals = synth.c5_arrivals(count, rate)
    res, stats, span = serve(arrivals)
    makespan = max(r.finished for r in res)
    lat = latency_summary(res)
    conv = sum(r.status == "converged" for r in res)
    worst = 0.0
    for i in range(0, count, max(1, count // 16)):
        s = systems[i]
        worst = max(worst, float(np.linalg.norm(s.f - s.scipy() @ res[i].x) / np.linalg.norm(s.f)))
    _log(f"[c5] poisson {rate:.1f}/s: {count / makespan:.1f} solves/s, latency {lat}, {stats}")
    # baseline: FIFO, one request at a time, plain FP64 plan + solve
    service = []
    base_conv = 0
    for i, s in enumerate(systems):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        with obk.plan_system(s, args.delta, check_every=args.check_every) as P:
            _, inf = P.solve(maxit=20000, tol=1e-10)
        service.append(time.perf_counter() - tb)
        base_conv += inf.status == "converged"
        if (i + 1) % 512 == 0:
            _log(f"[c5] FIFO baseline {i + 1}/{count}")
    free_at, base_lat = 0.0, []
    for a, sv in zip(arrivals, service):
        start = max(a, free_at)
        free_at = start + sv
        base_lat.append(free_at - a)
    base_lat = np.array(base_lat)
    cpu = None
    if not args.no_cpu_baseline:
        _log("[c5] CPU baseline: the oracle on independent requests, one per core")
        cpu = cpu_baseline_requests("c5", sizes, args.delta, args.check_every, args.cpu_budget,
                                    min(16, os.cpu_count() or 1))
    return {
        "metric": "solves/s and p50/p99 latency to rel. residual 1e-10 (continuous batching)",
        "value": count / makespan,
        "unit": "solves/s",
        "n_gpus": 1, "steps": stats["steps"], "warmup": 1, "ms_per_step": stats["step_seconds"] * 1e3 / max(1, stats["steps"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 sweeps + f64 refinement",
        "data": "synthetic",
        "config": {"workload": f"serving-{count}-requests-n-loguniform-500-5e5-4to16nnz-companion-poisson",
                   "requests": count, "arrival_rate_per_s": rate, "budget_bytes": budget,
                   "planners": args.planners, "inner_sweeps": args.inner, "rcm_engine": args.rcm_engine,
                   "membership": "new batch object per change" if args.c5_new_batch_objects
                   else "one batch object reset in place"},
        "latency_s": lat,
        "converged": conv,
        "worst_sampled_relres": worst,
        "saturation": {"solves_per_s": capacity, "latency_s": latency_summary(sat), "stats": sat_stats},
        "server_stats": stats,
        "baseline_fifo_plain_fp64": {"solves_per_s": count / float(free_at), "converged": base_conv,
                                     "p50_s": float(np.percentile(base_lat, 50)),
                                     "p99_s": float(np.percentile(base_lat, 99)),
                                     "mean_service_s": float(np.mean(service))},
        "cpu_baseline": cpu,
    }


def bench_c3(args) -> dict:
    """2,000,000 rows, 12 nnz/row.  Literal family: FP32 inner-sweep throughput
    (sweeps/s, GB/s) and the residual reached after a sweep cap.  Companion
    family: FP32 sweeps + FP64 refinement to 1e-10 with the error against the
    oracle's FP64 run of the same refinement schedule (and against the plain
    FP64 GPU solve, timed as the baseline)."""
    import torch
    import synth
    import paper_2401_00672_amd as obk
    n = args.n3
    s = synth.c3(n=n)
    t0 = time.perf_counter()
    P = obk.plan_system(s, args.delta, precision=obk.FP32_IR, inner_sweeps=args.inner)
    plan_s = time.perf_counter() - t0
    st = P.stats()
    P.solve(maxit=1, tol=0.0)               # warm-up: captures the sweep graphs
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    x, info = P.solve(maxit=args.ir_steps, tol=0.0)
    torch.cuda.synchronize()
    t_lit = time.perf_counter() - t1
    sweeps = info.sweeps
    B32 = sweep_bytes(s.n, s.n, s.nnz, sv=4, sx=4)
    P.free()
    lit = {
        "metric": "sweeps/s + GB/s vs HBM peak (FP32 inner sweeps); time to rel. residual 1e-10",
        "value": sweeps / t_lit, "unit": "sweeps/s", "n_gpus": 1, "steps": sweeps, "warmup": 0,
        "ms_per_step": t_lit * 1e3 / max(sweeps, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 sweeps + f64 refinement", "data": "synthetic",
        "config": {"workload": f"scattered-n{n}-12nnz-fp32ir", "n": n, "nnz": s.nnz, "groups": st["groups"]},
        "gb_per_s_fp32_sweep_incl_refinement": B32 * sweeps / t_lit / 1e9,
        "literal_relres_after": {"refinement_steps": info.outer_steps, "sweeps": sweeps, "relres": info.relres},
        "plan_seconds": plan_s,
    }
    if args.c3_sweeps_only:
        return lit
    sc = synth.c3(n=n, companion=True)
    Pc = obk.plan_system(sc, args.delta, precision=obk.FP32_IR, inner_sweeps=args.inner)
    Pc.solve(maxit=1, tol=0.0)              # warm-up: captures the sweep graphs
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    xc, ic = Pc.solve(maxit=100, tol=1e-10)
    torch.cuda.synchronize()
    t_comp = time.perf_counter() - t2
    Pc.set_opts(precision=obk.FP64, check_every=args.check_every)
    Pc.solve(maxit=args.check_every, tol=0.0)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    x64, i64 = Pc.solve(maxit=5000, tol=1e-10)
    t_64 = time.perf_counter() - t3
    Pc.free()
    err_gpu64 = float(np.linalg.norm(xc - x64) / np.linalg.norm(x64))
    err_star = float(np.linalg.norm(xc - sc.x_star) / np.linalg.norm(sc.x_star))
    _log("[c3] oracle FP64 refinement of the companion (same schedule)")
    err = _oracle_errors([sc], [xc], args.delta, args.inner)[0]
    return {
        "metric": "sweeps/s + GB/s vs HBM peak (FP32 inner sweeps); time to rel. residual 1e-10",
        "value": sweeps / t_lit, "unit": "sweeps/s", "n_gpus": 1, "steps": sweeps, "warmup": 0,
        "ms_per_step": t_lit * 1e3 / max(sweeps, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 sweeps + f64 refinement", "data": "synthetic",
        "config": {"workload": f"scattered-n{n}-12nnz-fp32ir", "n": n, "nnz": s.nnz, "groups": st["groups"]},
        "gb_per_s_fp32_sweep_incl_refinement": B32 * sweeps / t_lit / 1e9,
        "literal_relres_after": {"refinement_steps": info.outer_steps, "sweeps": sweeps, "relres": info.relres},
        "companion_to_1e10": {"seconds": t_comp, "refinement_steps": ic.outer_steps, "relres": ic.relres,
                              "status": ic.status, "error_vs_fp64_oracle": err,
                              "error_vs_gpu_fp64_solve": err_gpu64, "error_vs_xstar": err_star,
                              "fp64_seconds": t_64, "fp64_sweeps": i64.sweeps},
        "plan_seconds": plan_s,
    }


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


def arg_parser() -> argparse.ArgumentParser:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--grid", type=int, default=1024)
    ap.add_argument("--delta", type=float, default=0.1)
    ap.add_argument("--sweep-kernel", default="auto", choices=["auto", "phases", "banded"],
                    help="c2: which kernels run the sweeps")
    ap.add_argument("--profile-sweeps", type=int, default=20,
                    help="eager sweeps timed per launch for the dominant-kernel roofline")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--config", default="c2", choices=["c2", "c3", "c4", "c5", "block", "complex"],
                    help="c2: 1024^2 stencil sweeps (default line); c3: 2M-row FP32+IR; c4: 512 batched systems; "
                         "c5: continuous-batching server; block: block form of Algorithm 4; "
                         "complex: complex counterpart of c2")
    ap.add_argument("--block-grid", type=int, default=128, help="block: stencil grid side")
    ap.add_argument("--block-k", type=int, default=16, help="block: number of blocks")
    ap.add_argument("--block-thr", type=float, default=0.02, help="block: centroid cosine threshold")
    ap.add_argument("--block-wgs", type=int, default=0, help="block: workgroups of the projection launch (0: auto)")
    ap.add_argument("--block-solver", default="direct", choices=["direct", "cg"],
                    help="block: projections from banded Cholesky factors, or by conjugate gradients")
    ap.add_argument("--systems", type=int, default=512)
    ap.add_argument("--compact-batch", type=int, default=64,
                    help="c2: systems of the compact batched sub-run reported beside the sweep line (0: none)")
    ap.add_argument("--inner", type=int, default=8)
    ap.add_argument("--check-every", type=int, default=5)
    ap.add_argument("--n3", type=int, default=2_000_000)
    ap.add_argument("--ir-steps", type=int, default=20)
    ap.add_argument("--c3-sweeps-only", action="store_true",
                    help="c3: the FP32 sweep throughput only (no companion solve, for profiling)")
    ap.add_argument("--requests", type=int, default=512, help="c5: requests in the sample")
    ap.add_argument("--budget-gib", type=float, default=8.0, help="c5: device-memory admission budget")
    ap.add_argument("--planners", type=int, default=4, help="c5: planner threads")
    ap.add_argument("--rcm-engine", default="auto", choices=["auto", "device", "host"],
                    help="c5: how each request's plan forms its RCM order")
    ap.add_argument("--max-steps", type=int, default=200, help="c5: refinement steps before a request gives up")
    ap.add_argument("--c5-new-batch-objects", action="store_true",
                    help="c5: build a new batch object at every change of membership instead of resetting one")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a 256 MiB device copy (counter calibration) and exit")
    return ap


def main() -> int:
    args = arg_parser().parse_args()
    if args.copy_calibration:
        print(json.dumps(copy_calibration()), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "layout is a design note, not a measured path.", file=sys.stderr)
        return 2
    if args.config == "c4":
        res = bench_batched(args)
    elif args.config == "c3":
        res = bench_c3(args)
    elif args.config == "c5":
        res = bench_serving(args)
    elif args.config == "block":
        res = bench_block(args)
    elif args.config == "complex":
        res = bench_complex(args)
    else:
        res = bench_stencil(args)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
