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
  object is rebuilt over the new member set (members keep their iterates,
  which live in their plans) and only the newcomers are started from x0 = 0;
* **retiring** -- a member whose relative residual reached ``tol`` (or that hit
  ``max_steps``) leaves at the step boundary; its solution is copied to the
  host and its plan freed.

Latency is measured from a request's arrival to its solution being on the
host.  The backend is pluggable so that the scheduling logic can be tested on
the CPU with a stand-in backend; the default backend is libobk on the GPU.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import queue
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
    status: str             # "converged" | "maxit" | "rejected"

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

    # Plans are built on planner threads beside the batched solves.  The host
    # BFS then runs on otherwise idle cores, while the device RCM's per-level
    # launches and synchronisations compete with the solve stream (saturation
    # measured at 109 solves/s with the host loop against 97-100 with the
    # automatic choice), so the server forms RCM orders on the host.
    def __init__(self, delta: float = 0.1, inner_sweeps: int = 8, batch_opts=None, planners: int = 2,
                 rcm_engine: str = "host"):
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

    def start(self, batch, i: int) -> None:
        batch.start(i, stream=self.stream.cuda_stream)

    def step(self, batch, tol: float):
        return batch.step(tol, stream=self.stream.cuda_stream)

    def result(self, batch, i: int) -> np.ndarray:
        return batch.result(i, stream=self.stream.cuda_stream)

    def free_batch(self, batch) -> None:
        batch.free()

    def free_plan(self, plan) -> None:
        plan.free()


@dataclasses.dataclass
class _Member:
    req: Request
    plan: object
    nbytes: int
    admitted: float
    steps: int = 0


class Server:
    """Continuous batching with FIFO admission under an HBM budget."""

    def __init__(self, backend, budget_bytes: int, tol: float = 1e-10, max_steps: int = 200,
                 planners: int = 2, clock=time.perf_counter, idle_wait: float = 0.002):
        self.backend = backend
        self.budget = int(budget_bytes)
        self.tol = float(tol)
        self.max_steps = int(max_steps)
        self.planners = int(planners)
        self.clock = clock
        self.idle_wait = idle_wait
        self.stats = {"steps": 0, "rebuilds": 0, "peak_bytes": 0, "peak_members": 0, "step_seconds": 0.0,
                      "rebuild_seconds": 0.0}

    def run(self, requests) -> list[Result]:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        pending = collections.deque(reqs)
        t0 = self.clock()
        now = lambda: self.clock() - t0          # noqa: E731
        results: dict[int, Result] = {}
        members: list[_Member] = []
        joining: list[_Member] = []
        planning: dict[cf.Future, tuple[Request, int, float]] = {}
        used = 0
        batch = None
        pool = cf.ThreadPoolExecutor(max_workers=max(1, self.planners))
        try:
            while len(results) < len(reqs):
                t = now()
                # 1. admission: FIFO, the head blocks when it does not fit
                while pending and pending[0].arrival <= t:
                    r = pending[0]
                    est = footprint_estimate(r.system.n, r.system.nnz)
                    if est > self.budget:
                        pending.popleft()
                        results[r.rid] = Result(r.rid, None, r.arrival, t, now(), 0, float("nan"), "rejected")
                        continue
                    if used + est > self.budget:
                        break
                    pending.popleft()
                    used += est
                    planning[pool.submit(self.backend.plan, r.system)] = (r, est, t)
                # 2. planned requests join at this step boundary
                for fut in [f for f in planning if f.done()]:
                    r, est, ta = planning.pop(fut)
                    plan = fut.result()
                    nb = self.backend.plan_bytes(plan)
                    used += nb - est
                    joining.append(_Member(r, plan, nb, ta))
                self.stats["peak_bytes"] = max(self.stats["peak_bytes"], used)
                if joining:
                    tb = self.clock()
                    if batch is not None:
                        self.backend.free_batch(batch)
                    first_new = len(members)
                    members.extend(joining)
                    joining = []
                    batch = self.backend.make_batch([m.plan for m in members])
                    for i in range(first_new, len(members)):
                        self.backend.start(batch, i)
                    self.stats["rebuilds"] += 1
                    self.stats["rebuild_seconds"] += self.clock() - tb
                self.stats["peak_members"] = max(self.stats["peak_members"], len(members))
                # 3. one batched step, then retire the finished members
                if members:
                    ts = self.clock()
                    relres, active = self.backend.step(batch, self.tol)
                    self.stats["step_seconds"] += self.clock() - ts
                    self.stats["steps"] += 1
                    keep = []
                    for i, m in enumerate(members):
                        if active[i]:
                            m.steps += 1
                        done = (not active[i]) or m.steps >= self.max_steps
                        if not done:
                            keep.append(m)
                            continue
                        x = self.backend.result(batch, i)
                        status = "converged" if relres[i] <= self.tol and not active[i] else "maxit"
                        results[m.req.rid] = Result(m.req.rid, x, m.req.arrival, m.admitted, now(), m.steps,
                                                    float(relres[i]), status)
                        self.backend.free_plan(m.plan)
                        used -= m.nbytes
                    if len(keep) != len(members):
                        self.backend.free_batch(batch)
                        batch = None
                        members = keep
                        if members:
                            tb = self.clock()
                            batch = self.backend.make_batch([m.plan for m in members])
                            self.stats["rebuilds"] += 1
                            self.stats["rebuild_seconds"] += self.clock() - tb
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
        return [results[r.rid] for r in reqs]


def latency_summary(results) -> dict:
    lat = np.array([r.latency for r in results if r.status != "rejected"])
    if lat.size == 0:
        return {"p50_s": None, "p99_s": None, "mean_s": None}
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean())}
