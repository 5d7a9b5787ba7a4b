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
        self.enabled = [True] * len(self.plans)
        self.freed = False


class FakeBackend:
    """relres after k steps = 10**-k; converged when k >= need."""

    def __init__(self, plan_bytes_factor=1.0, fail=()):
        self.live_plans = set()
        self.factor = plan_bytes_factor
        self.fail = set(fail)           # systems (by id) whose plan raises
        self.batches = []
        self.resets = 0

    def plan(self, system):
        if id(system) in self.fail:
            raise RuntimeError("OBK_E_CSR: malformed system")
        p = _Plan(system)
        self.live_plans.add(p)
        return p

    def plan_bytes(self, plan):
        return int(footprint_estimate(plan.s.n, plan.s.nnz) * self.factor)

    def make_batch(self, plans):
        assert all(not p.freed for p in plans)
        b = _Batch(plans)
        self.batches.append(b)
        return b

    def reset_batch(self, batch, plans):
        # like obk_batch_reset: the same object over a new member list, every
        # member enabled, iterates (in the plans) untouched
        assert not batch.freed
        assert all(not p.freed for p in plans)
        batch.plans = list(plans)
        batch.enabled = [True] * len(batch.plans)
        self.resets += 1

    def enable(self, batch, enabled):
        assert not batch.freed
        batch.enabled = [bool(e) for e in enabled]

    def start(self, batch, i):
        assert batch.plans[i].k is None, "a member was started twice"
        batch.plans[i].k = 0

    def step(self, batch, tol):
        assert not batch.freed
        rr, act = [], []
        for p, en in zip(batch.plans, batch.enabled):
            # like the library's step, every member's residual is read: its
            # plan must still exist, enabled or not
            assert not p.freed, "a batch step read a freed plan"
            assert p.k is not None, "stepped a member that was never started"
            r = 10.0 ** (-min(p.k, p.s.need))
            a = en and r > tol
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
        assert not any(plan in b.plans for b in self.batches if not b.freed), "plan freed under a live batch"
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


def test_failed_plan_is_reported_and_budget_returned():
    """A request whose plan raises gets a 'failed' result with the message;
    its budget comes back and every other request is served."""
    reqs = _requests(30, seed=5, rate=1e6)
    bad = {id(reqs[4].system), id(reqs[11].system)}
    budget = int(max(footprint_estimate(q.system.n, q.system.nnz) for q in reqs) * 3)
    be = FakeBackend(fail=bad)
    srv = Server(be, budget_bytes=budget, tol=1e-10, max_steps=12)
    res = srv.run(reqs)
    st = {r.rid: r for r in res}
    assert st[4].status == "failed" and "malformed" in st[4].error and st[11].status == "failed"
    assert all(r.status in ("converged", "maxit") for r in res if r.rid not in (4, 11))
    assert srv.stats["failed"] == 2 and not be.live_plans


def test_cancellation_leaves_the_others_unchanged():
    """Cancelling a request mid-flight (queued, planning or being solved)
    withdraws it with a 'cancelled' result; every other request's result is
    the one it gets without the cancellation."""
    reqs = _requests(24, seed=6, rate=1e6)
    for q in reqs:
        q.system.need = 14                            # long enough to be caught mid-solve
    ref = Server(FakeBackend(), budget_bytes=1 << 40, tol=1e-10, max_steps=20).run(reqs)

    class _Cancelling(FakeBackend):
        def step(self, batch, tol):
            out = super().step(batch, tol)
            self.steps = getattr(self, "steps", 0) + 1
            if self.steps == 3:
                srv.cancel(5)                         # a member being solved
                srv.cancel(23)                        # the last one, still queued or planning
            return out

    be = _Cancelling()
    srv = Server(be, budget_bytes=1 << 40, tol=1e-10, max_steps=20)
    res = srv.run(reqs)
    got = {r.rid: r for r in res}
    assert got[5].status == "cancelled" and got[23].status == "cancelled"
    for a in ref:
        if a.rid in (5, 23):
            continue
        b = got[a.rid]
        assert (b.status, b.steps) == (a.status, a.steps) and np.array_equal(b.x, a.x)
    assert not be.live_plans and srv.stats["cancelled"] == 2


def test_retired_members_are_disabled_not_rebuilt():
    """Retiring a member disables its slot; the batch is rebuilt only when
    members join or retired slots outnumber the live ones."""
    reqs = _requests(40, seed=7, rate=1e6)
    be = FakeBackend()
    srv = Server(be, budget_bytes=1 << 40, tol=1e-10, max_steps=30)
    res = srv.run(reqs)
    assert all(r.status in ("converged", "maxit") for r in res)
    retirements = sum(1 for r in res)
    assert srv.stats["rebuilds"] < retirements


@pytest.mark.parametrize("seed", [3, 11])
def test_in_place_reset_equals_new_batch_objects(seed):
    """Re-forming one batch object in place gives every request the same
    result, step count and status as building a new batch object per change
    of membership, and frees every plan."""
    out = []
    for reuse in (True, False):
        be = FakeBackend()
        srv = Server(be, budget_bytes=6 * footprint_estimate(3000, 15000), tol=1e-10, max_steps=30,
                     reuse_batch=reuse)
        res = srv.run(_requests(60, seed=seed, rate=3000.0))
        assert not be.live_plans
        if reuse:
            assert be.resets >= 1 and len(be.batches) == 1
        else:
            assert be.resets == 0 and len(be.batches) == srv.stats["rebuilds"]
        out.append({r.rid: r for r in res})
    a, b = out
    assert a.keys() == b.keys()
    for k in a:
        assert (a[k].status, a[k].steps) == (b[k].status, b[k].steps)
        assert (a[k].x is None) == (b[k].x is None)
        if a[k].x is not None:
            assert np.array_equal(a[k].x, b[k].x)
