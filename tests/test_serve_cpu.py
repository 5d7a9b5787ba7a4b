"""Scheduling logic of the continuous-batching server, on the CPU.

A stand-in backend keeps per-plan state the way libobk does (the iterate
lives in the plan; a batch object is only a schedule over plans), so the
tests catch a member restarted by a rebuild, a result read from the wrong
slot, admission over the budget, and lost or duplicated requests.
"""
import dataclasses

import numpy as np
import pytest

from paper_2401_00672_amd.serve import Request, Server, footprint_estimate, latency_summary


@dataclasses.dataclass
class _Sys:
    n: int
    nnz: int
    f: np.ndarray
    need: int            # steps this system needs to converge


class _Plan:
    def __init__(self, s):
        self.s = s
        self.k = None    # steps taken since start; None until started
        self.freed = False


class _Batch:
    def __init__(self, plans):
        self.plans = list(plans)
        self.freed = False


class FakeBackend:
    """relres after k steps = 10**-k; converged when k >= need."""

    def __init__(self, plan_bytes_factor=1.0):
        self.live_plans = set()
        self.factor = plan_bytes_factor

    def plan(self, system):
        p = _Plan(system)
        self.live_plans.add(p)
        return p

    def plan_bytes(self, plan):
        return int(footprint_estimate(plan.s.n, plan.s.nnz) * self.factor)

    def make_batch(self, plans):
        assert all(not p.freed for p in plans)
        return _Batch(plans)

    def start(self, batch, i):
        assert batch.plans[i].k is None, "a member was started twice"
        batch.plans[i].k = 0

    def step(self, batch, tol):
        assert not batch.freed
        rr, act = [], []
        for p in batch.plans:
            assert p.k is not None, "stepped a member that was never started"
            r = 10.0 ** (-min(p.k, p.s.need))
            a = r > tol
            rr.append(r)
            act.append(a)
            if a:
                p.k += 1
        return np.array(rr), np.array(act)

    def result(self, batch, i):
        p = batch.plans[i]
        return p.s.f * p.k          # depends on the member's own step count

    def free_batch(self, batch):
        batch.freed = True

    def free_plan(self, plan):
        assert not plan.freed
        plan.freed = True
        self.live_plans.discard(plan)


def _requests(count, seed=0, rate=200.0, big=None):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for i in range(count):
        n = int(rng.integers(100, 2000))
        nnz = n * int(rng.integers(4, 17))
        if big is not None and i in big:
            n, nnz = 10 ** 7, 10 ** 8
        out.append(Request(i, float(t[i]), _Sys(n, nnz, rng.standard_normal(3), int(rng.integers(1, 12)))))
    return out


def test_every_request_served_once_with_its_own_result():
    reqs = _requests(60)
    be = FakeBackend()
    res = Server(be, budget_bytes=1 << 40, tol=1e-10, planners=3).run(reqs)
    assert [r.rid for r in res] == [q.rid for q in reqs]
    for q, r in zip(reqs, res):
        need = min(q.system.need, 11)
        # converged after exactly `need` advancing steps: relres 10**-need <= 1e-10 needs need >= 10
        if q.system.need >= 10:
            assert r.status == "converged" and r.steps == 10
            assert np.array_equal(r.x, q.system.f * 10)
        else:
            assert r.status == "maxit" or r.steps <= need
        assert r.latency >= 0 and r.finished >= r.admitted >= r.arrival - 1e-9
    assert not be.live_plans


def test_budget_is_never_exceeded_and_fifo_order_of_admission():
    reqs = _requests(50, seed=1, rate=1e6)            # everything arrives at once
    est = [footprint_estimate(q.system.n, q.system.nnz) for q in reqs]
    budget = int(np.sort(est)[-1] * 3)                # about three systems at a time
    be = FakeBackend()
    srv = Server(be, budget_bytes=budget, tol=1e-10, max_steps=5)
    res = srv.run(reqs)
    assert srv.stats["peak_bytes"] <= budget
    adm = [r.admitted for r in res]
    assert all(a <= b + 1e-12 for a, b in zip(adm, adm[1:])), "admission must be FIFO"
    assert all(r.status in ("converged", "maxit") for r in res)
    assert all(r.steps <= 5 for r in res)


def test_oversized_request_is_rejected_others_served():
    reqs = _requests(20, seed=2, big={3, 7})
    res = Server(FakeBackend(), budget_bytes=1 << 30, tol=1e-10).run(reqs)
    st = {r.rid: r.status for r in res}
    assert st[3] == "rejected" and st[7] == "rejected"
    assert all(st[i] != "rejected" for i in st if i not in (3, 7))
    lat = latency_summary(res)
    assert lat["p50_s"] is not None and lat["p99_s"] >= lat["p50_s"]


def test_result_alone_equals_result_in_mix():
    reqs = _requests(30, seed=3)
    mixed = Server(FakeBackend(), budget_bytes=1 << 40, tol=1e-10, planners=2).run(reqs)
    for q, r in zip(reqs[:8], mixed[:8]):
        alone = Server(FakeBackend(), budget_bytes=1 << 40, tol=1e-10).run([Request(q.rid, 0.0, q.system)])[0]
        assert alone.steps == r.steps and np.array_equal(alone.x, r.x)


@pytest.mark.parametrize("factor", [0.5, 1.0])
def test_exact_plan_bytes_replace_estimate(factor):
    reqs = _requests(25, seed=4, rate=1e6)
    budget = int(max(footprint_estimate(q.system.n, q.system.nnz) for q in reqs) * 2)
    srv = Server(FakeBackend(plan_bytes_factor=factor), budget_bytes=budget, tol=1e-10, max_steps=3)
    res = srv.run(reqs)
    assert len(res) == 25 and srv.stats["peak_bytes"] <= budget
