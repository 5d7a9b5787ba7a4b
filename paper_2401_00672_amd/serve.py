"""Continuous-batching solve server over the batched sweep engine.

Requests (one sparse system ``A x = f`` each) arrive over time.  The server
keeps every admitted system's plan and iterate resident in HBM and advances
all of them together, one batched step per loop turn (``obk_batch_step``: an
FP64 residual, then the inner FP32 sweeps of every unfinished system in one
persistent launch, then the FP64 update):

* **admission** -- first in, first out, against a device-memory budget: a
  request is admitted when its footprint fits beside the admitted ones (an
  estimate until its plan exists, then the plan's exact ``obk_plan_bytes``);
  a request larger than the whole budget is rejected;
* **planning** -- on planner threads, each with its own HIP stream, so plans
  for new arrivals are built while the batch steps;
* **joining** -- planned requests join at the next step boundary: the batch
  object is re-formed over the new member set in place (``obk_batch_reset``:
  its device storage and captured step graph are kept while they are large
  enough; members keep their iterates, which live in their plans) and only
  the newcomers are started from x0 = 0;
* **retiring** -- a member whose relative residual reached ``tol`` (or that hit
  ``max_steps``) leaves at the step boundary; its solution is copied to the
  host.  Its slot in the batch object is disabled (``obk_batch_enable``);
  its plan stays allocated while the batch object refers to it and is freed
  when the batch is next re-formed -- when requests join, when disabled
  slots outnumber the live ones, or when the head of the queue waits for
  memory that retired plans hold;
* **failure and cancellation** -- a request whose plan fails (a malformed
  system, memory) gets a ``failed`` result and returns its budget; ``cancel``
  (from any thread) withdraws a request that is waiting, planning or being
  solved, with a ``cancelled`` result, and leaves the others' work as it is.

Latency is measured from a request's arrival to its solution being on the
host.  The backend is pluggable so that the scheduling logic can be tested on
the CPU with a stand-in backend; the default backend is libobk on the GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import queue
import threading
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the server clock starts
    system: object          # row_ptr, col, val, f (host arrays), n, nnz


@dataclasses.dataclass
class Result:
    rid: int
    x: np.ndarray | None
    arrival: float
    admitted: float
    finished: float
    steps: int
    relres: float
    status: str             # "converged" | "maxit" | "rejected" | "failed" | "cancelled"
    error: str = ""

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def footprint_estimate(n: int, nnz: int) -> int:
    """Device bytes of an FP32-refinement plan before it exists: the
    group-major CSR and per-group CSC in FP64 and FP32 plus per-row vectors
    (an upper estimate of obk_plan_bytes for 4..16 entries per row)."""
    return 48 * int(nnz) + 112 * int(n) + (1 << 20)


class LibobkBackend:
    """Plans and batched steps through libobk (FP32 sweeps + FP64 refinement)."""

    # Plans are built on planner threads beside the batched solves.  Either
    # RCM engine gives the same order; with plan temporaries reused inside the
    # library, the automatic choice (device levels, host loop for narrow
    # ones) served 281 against 241 solves/s at saturation with four planners
    # on the first 2,048 requests, so it is the default.
    def __init__(self, delta: float = 0.1, inner_sweeps: int = 8, batch_opts=None, planners: int = 2,
                 rcm_engine: str = "auto"):
        import torch

        import paper_2401_00672_amd as obk
        self.obk = obk
        self.delta = delta
        self.rcm_engine = rcm_engine
        self.inner = inner_sweeps
        self.batch_opts = batch_opts
        self._slots = queue.Queue()
        for _ in range(planners):
            self._slots.put(torch.cuda.Stream())
        self.stream = torch.cuda.Stream()

    def plan(self, system):
        st = self._slots.get()
        try:
            return self.obk.plan_system(system, self.delta, precision=self.obk.FP32_IR,
                                        inner_sweeps=self.inner, rcm_engine=self.rcm_engine,
                                        stream=st.cuda_stream)
        finally:
            self._slots.put(st)

    def plan_bytes(self, plan) -> int:
        return plan.device_bytes()

    def make_batch(self, plans):
        return self.obk.Batch(plans, self.batch_opts)

    def reset_batch(self, batch, plans) -> None:
        batch.reset(plans, stream=self.stream.cuda_stream)

    def enable(self, batch, enabled) -> None:
        batch.enable(np.asarray(enabled, dtype=np.int32), stream=self.stream.cuda_stream)

    def start(self, batch, i: int) -> None:
        batch.start(i, stream=self.stream.cuda_stream)

    def step(self, batch, tol: float):
        return batch.step(tol, stream=self.stream.cuda_stream)

    def result(self, batch, i: int) -> np.ndarray:
        return batch.result(i, stream=self.stream.cuda_stream)

    def free_batch(self, batch) -> None:
        batch.free()

    def free_plan(self, plan) -> None:
        # its last use (a step, a result copy) was on the server's stream:
        # the release waits for that stream only, not for the planners' work
        # on the device, and the library keeps the memory for later plans
        plan.free(stream=self.stream.cuda_stream)


@dataclasses.dataclass
class _Member:
    req: Request
    plan: object
    nbytes: int
    admitted: float
    steps: int = 0
    live: bool = True       # False once retired (its slot in the batch is disabled)


class Server:
    """Continuous batching with FIFO admission under an HBM budget."""

    def __init__(self, backend, budget_bytes: int, tol: float = 1e-10, max_steps: int = 200,
                 planners: int = 2, clock=time.perf_counter, idle_wait: float = 0.002, progress=None,
                 progress_every: int = 0, reuse_batch: bool = True):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.tol = float(tol)
        self.max_steps = int(max_steps)
        self.planners = int(planners)
        self.clock = clock
        self.idle_wait = idle_wait
        self.progress = progress                 # called with (finished, total) every progress_every results
        self.progress_every = int(progress_every)
        # True: one batch object re-formed in place when members join
        # (obk_batch_reset); False: a new batch object each time
        self.reuse_batch = bool(reuse_batch)
        # rebuilds / rebuild_seconds: re-formations of the batch over a new
        # member list (in place, or a new object with reuse_batch=False);
        # free_seconds: plan releases; plan_seconds: summed over planner threads
        self.stats = {"steps": 0, "rebuilds": 0, "peak_bytes": 0, "peak_members": 0, "step_seconds": 0.0,
                      "rebuild_seconds": 0.0, "free_seconds": 0.0, "plan_seconds": 0.0, "failed": 0, "cancelled": 0}
        self._cancel_lock = threading.Lock()
        self._cancel: set[int] = set()

    def cancel(self, rid: int) -> None:
        """Withdraw request `rid` (thread-safe): it is dropped at the next loop
        turn with a ``cancelled`` result, whatever stage it is in."""
        with self._cancel_lock:
            self._cancel.add(int(rid))

    def _plan(self, system):
        # on a planner thread: the time it spends is summed in plan_seconds
        t = time.perf_counter()
        try:
            return self.backend.plan(system)
        finally:
            with self._cancel_lock:
                self.stats["plan_seconds"] += time.perf_counter() - t

    def _cancelled(self) -> set[int]:
        with self._cancel_lock:
            return set(self._cancel)

    def run(self, requests) -> list[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque(reqs)
        t0 = self.clock()
        now = lambda: self.clock() - t0          # noqa: E731
        results: dict[int, Result] = {}
        members: list[_Member] = []              # the batch's slots, in batch order
        joining: list[_Member] = []
        planning: dict[cf.Future, tuple[Request, int, float]] = {}
        used = 0
        batch = None
        pool = cf.ThreadPoolExecutor(max_workers=max(1, self.planners))

        def finish(r: Request, admitted: float, status: str, x=None, steps=0, relres=float("nan"), err=""):
            results[r.rid] = Result(r.rid, x, r.arrival, admitted, now(), steps, relres, status, err)
            if status in ("failed", "cancelled"):
                self.stats[status] += 1
            if self.progress and self.progress_every > 0 and len(results) % self.progress_every == 0:
                self.progress(len(results), len(reqs))

        try:
            while len(results) < len(reqs):
                t = now()
                gone = self._cancelled()
                # 0. cancellations: waiting requests leave the queue at once
                if gone and any(r.rid in gone for r in pending):
                    for r in [r for r in pending if r.rid in gone]:
                        finish(r, t, "cancelled")
                    pending = collections.deque(r for r in pending if r.rid not in gone)
                # 1. admission: FIFO, the head blocks when it does not fit
                blocked = False
                while pending and pending[0].arrival <= t:
                    r = pending[0]
                    est = footprint_estimate(r.system.n, r.system.nnz)
                    if est > self.budget:
                        pending.popleft()
                        finish(r, t, "rejected")
                        continue
                    if used + est > self.budget:
                        blocked = True
                        break
                    pending.popleft()
                    used += est
                    planning[pool.submit(self._plan, r.system)] = (r, est, t)
                # 2. planned requests join at this step boundary (a failed or
                # cancelled one returns its budget)
                for fut in [f for f in planning if f.done()]:
                    r, est, ta = planning.pop(fut)
                    try:
                        plan = fut.result()
                    except Exception as e:               # noqa: BLE001 -- reported per request
                        used -= est
                        finish(r, ta, "failed", err=str(e))
                        continue
                    if r.rid in gone:
                        self.backend.free_plan(plan)
                        used -= est
                        finish(r, ta, "cancelled")
                        continue
                    nb = self.backend.plan_bytes(plan)
                    used += nb - est
                    joining.append(_Member(r, plan, nb, ta))
                self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used)
                # cancelled members retire like finished ones, without a result
                if gone and any(m.live and m.req.rid in gone for m in members):
                    for m in members:
                        if m.live and m.req.rid in gone:
                            m.live = False
                            finish(m.req, m.admitted, "cancelled", steps=m.steps)
                    self.backend.enable(batch, [1 if m.live else 0 for m in members])
                live = [m for m in members if m.live]
                retired_held = len(members) - len(live)
                if joining or (retired_held and (len(live) < retired_held or blocked)):
                    # re-form the batch over the live members and the
                    # newcomers; the retired members' plans are freed once no
                    # batch refers to them
                    tb = self.clock()
                    retired_members = [m for m in members if not m.live]
                    first_new = len(live)
                    members = live + joining
                    joining = []
                    plans = [m.plan for m in members]
                    if batch is not None and self.reuse_batch:
                        self.backend.reset_batch(batch, plans)
                    else:
                        if batch is not None:
                            self.backend.free_batch(batch)
                            batch = None
                        if members:
                            batch = self.backend.make_batch(plans)
                    for i in range(first_new, len(members)):
                        self.backend.start(batch, i)
                    self.stats["rebuilds"] += 1 if members else 0
                    tf = self.clock()
                    self.stats["rebuild_seconds"] += tf - tb
                    for m in retired_members:
                        self.backend.free_plan(m.plan)
                        used -= m.nbytes
                    self.stats["free_seconds"] += self.clock() - tf
                live_count = sum(1 for m in members if m.live)
                self.stats["peak_members"] = max(self.stats["peak_members"], live_count)
                # 3. one batched step, then retire the finished members
                if live_count:
                    ts = self.clock()
                    relres, active = self.backend.step(batch, self.tol)
                    self.stats["step_seconds"] += self.clock() - ts
                    self.stats["steps"] += 1
                    retired = False
                    for i, m in enumerate(members):
                        if not m.live:
                            continue
                        if active[i]:
                            m.steps += 1
                        if active[i] and m.steps < self.max_steps:
                            continue
                        x = self.backend.result(batch, i)
                        status = "converged" if relres[i] <= self.tol and not active[i] else "maxit"
                        finish(m.req, m.admitted, status, x, m.steps, float(relres[i]))
                        m.live = False
                        retired = True
                    if retired and any(m.live for m in members):
                        self.backend.enable(batch, [1 if m.live else 0 for m in members])
                    continue
                # 4. idle: wait for a plan or the next arrival
                wait = self.idle_wait
                if pending:
                    wait = min(wait, max(0.0, pending[0].arrival - now()))
                if planning:
                    cf.wait(list(planning), timeout=wait, return_when=cf.FIRST_COMPLETED)
                elif wait > 0:
                    time.sleep(wait)
        finally:
            pool.shutdown(wait=True)
            if batch is not None:
                self.backend.free_batch(batch)
            # plans still held (retired members of the last batch, or all of
            # them when the loop ends early on an error elsewhere)
            for m in members + joining:
                self.backend.free_plan(m.plan)
            for fut in planning:
                try:
                    self.backend.free_plan(fut.result())
                except Exception:                        # noqa: BLE001 -- its error was the request's
                    pass
        return [results[r.rid] for r in reqs]


def latency_summary(results) -> dict:
    lat = np.array([r.latency for r in results if r.status != "rejected"])
    if lat.size == 0:
        return {"p50_s": None, "p99_s": None, "mean_s": None}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}
