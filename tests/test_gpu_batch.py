"""Batched solves on the GPU: many systems in shared launches.

Each system's result in a batch must equal its result when solved alone,
bit for bit: the batch runs the same tile reductions in the same order, the
same FP64 residual blocking and the same stopping rule; only the placement
of work on workgroups differs.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
import paper_2401_00672_amd as obk

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.init()


SIZES = [1000, 1733, 2500, 4096, 7001, 12000, 20000, 31000]


def _systems(companion=True):
    return [synth.c4_system(i, n=n, companion=companion) for i, n in enumerate(SIZES)]


@pytest.mark.parametrize("opts", [None, {"team_work": 4096, "max_team": 16}, {"wgs_per_cu": 2}],
                         ids=["default", "multi-wg-teams", "two-per-cu"])
def test_batch_fp32_refinement_equals_single(opts):
    systems = _systems()
    _say(f"[batch] fp32-ir opts={opts}")
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8) for s in systems]
    singles = [p.solve(maxit=100, tol=1e-10) for p in plans]
    xs, infos = obk.solve_batch(plans, tol=1e-10, maxit=100, opts=opts)
    for s, (x1, i1), x2, i2 in zip(systems, singles, xs, infos):
        assert i1.status == "converged" and i2.status == "converged", (i1, i2)
        assert i2.relres <= 1e-10
        assert i1.outer_steps == i2.outer_steps
        assert np.array_equal(x1, x2), f"n={s.n}: batch and single differ"
        err = np.linalg.norm(x2 - s.x_star) / np.linalg.norm(s.x_star)
        assert err < 1e-8
    for p in plans:
        p.free()


def test_batch_fp64_equals_single():
    systems = _systems(companion=False)[:5]
    _say("[batch] fp64")
    plans = [obk.plan_system(s, 0.1, check_every=5) for s in systems]
    xs, infos = obk.solve_batch(plans, tol=0.0, maxit=4, opts={"team_work": 8192})
    for s, p, x, inf in zip(systems, plans, xs, infos):
        x1, i1 = p.solve(maxit=20)
        assert inf.sweeps == 20 and inf.status == "maxit"
        assert np.array_equal(x, x1)
        pl = oracle.plan_system(s, 0.1)
        xo = oracle.solve(pl, 20)
        assert np.linalg.norm(x - xo) / np.linalg.norm(xo) <= 1e-10
    for p in plans:
        p.free()


def test_batch_step_enable_and_results():
    """The serving primitives: steps with retirement of converged systems and
    disabling of others; a disabled system keeps its iterate."""
    systems = _systems()[:6]
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR) for s in systems]
    b = obk.Batch(plans)
    b.begin()
    done = np.zeros(len(plans), bool)
    for it in range(60):
        rr, act = b.step(1e-10)
        done |= ~act
        if done.all():
            break
    assert done.all()
    for i, s in enumerate(systems):
        x = b.result(i)
        assert np.linalg.norm(s.f - s.scipy() @ x) / np.linalg.norm(s.f) <= 1.5e-10
    # disable system 0 from the start: it must stay at x0 = 0
    b.begin()
    b.enable([0] + [1] * (len(plans) - 1))
    for _ in range(3):
        rr, act = b.step(1e-10)
        assert not act[0]
    assert np.array_equal(b.result(0), np.zeros(systems[0].n))
    b.free()
    for p in plans:
        p.free()


def test_batch_graph_replays_equal_eager_steps(monkeypatch):
    """A step is replayed from a captured graph; every replay (with the host's
    copies and checks in between) must equal the eagerly launched step."""
    import torch
    systems = _systems()[:5]
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR) for s in systems]

    def run(eager):
        if eager:
            monkeypatch.setenv("OBK_BATCH_EAGER", "1")
        else:
            monkeypatch.delenv("OBK_BATCH_EAGER", raising=False)
        b = obk.Batch(plans)
        b.begin()
        hist = []
        for _ in range(7):
            rr, act = b.step(1e-10)
            hist.append((rr.copy(), act.copy()))
            torch.cuda.synchronize()
        xs = [b.result(i) for i in range(len(plans))]
        b.free()
        return hist, xs

    _say("[batch] graph vs eager steps")
    h_graph, x_graph = run(False)
    h_eager, x_eager = run(True)
    for (r1, a1), (r2, a2) in zip(h_graph, h_eager):
        assert np.array_equal(r1, r2) and np.array_equal(a1, a2)
    for a, b in zip(x_graph, x_eager):
        assert np.array_equal(a, b)
    for p in plans:
        p.free()


def test_batch_tune_and_errors():
    systems = _systems()[:4]
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR) for s in systems]
    best, sec = obk.batch_tune(plans)
    _say(f"[batch] tuned {best} {sec * 1e3:.3f} ms/step")
    assert best["wgs_per_cu"] in (1, 2, 4, 8) and best["tiles_per_wg"] in (1, 2, 4) and sec > 0
    xs, infos = obk.solve_batch(plans, tol=1e-10, maxit=100, opts=best)
    assert all(i.status == "converged" for i in infos)
    p64 = obk.plan_system(systems[0], 0.1)
    with pytest.raises(obk.ObkError) as ei:
        obk.solve_batch([plans[0], p64], tol=1e-10)
    assert ei.value.code == -1
    with pytest.raises(obk.ObkError):
        obk.solve_batch([plans[0], plans[0]], tol=1e-10)
    for p in plans + [p64]:
        p.free()


@pytest.mark.parametrize("eager", [False, True], ids=["graph", "eager"])
def test_batch_reset_members_continue_and_equal_single(monkeypatch, eager):
    """obk_batch_reset: one batch object re-formed over changing member lists.
    Members that stay continue from their iterates, new members start from
    zero, and every system's result equals its solve alone for the number of
    steps that advanced it -- through growth (new storage, new graph), shrinkage
    (storage and graph kept), an empty list, a change of precision and a
    rejected list (the batch keeps its members)."""
    if eager:
        monkeypatch.setenv("OBK_BATCH_EAGER", "1")
    else:
        monkeypatch.delenv("OBK_BATCH_EAGER", raising=False)
    systems = _systems()
    tol = 1e-10
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8) for s in systems]
    steps = [0] * len(plans)
    results = {}
    state = {"members": [0, 1, 2]}
    b = obk.Batch([plans[i] for i in state["members"]])
    b.begin()

    def run(k):
        for _ in range(k):
            rr, act = b.step(tol)
            for slot, i in enumerate(state["members"]):
                steps[i] += int(act[slot])

    def reform(new):
        old = state["members"]
        for slot, i in enumerate(old):
            if i not in new:
                results[i] = b.result(slot)
        _say(f"[batch] reset {old} -> {new}")
        b.reset([plans[i] for i in new])
        for slot, i in enumerate(new):
            if i not in old:
                b.start(slot)
        for i in old:
            if i not in new:
                plans[i].free()          # the batch no longer refers to it
        state["members"] = new

    run(2)
    reform([1, 3, 2, 7])                  # grows
    run(3)
    with pytest.raises(obk.ObkError) as ei:
        b.reset([plans[3], plans[3]])
    assert ei.value.code == -1 and len(b.plans) == 4
    run(1)
    reform([3, 2])                        # shrinks
    run(2)
    reform([])
    reform([4, 5, 6])
    for _ in range(60):
        rr, act = b.step(tol)
        for slot, i in enumerate(state["members"]):
            steps[i] += int(act[slot])
        if not act.any():
            break
    reform([])
    assert sorted(results) == list(range(len(systems)))
    for i, x in sorted(results.items()):
        q = obk.plan_system(systems[i], 0.1, precision=obk.FP32_IR, inner_sweeps=8)
        x1, info = q.solve(maxit=steps[i], tol=tol)
        q.free()
        assert info.outer_steps == steps[i], (i, info.outer_steps, steps[i])
        assert np.array_equal(x1, x), f"system {i} after {steps[i]} steps: reset batch and single differ"
    # the same object over FP64 plans: another kernel, graphs captured again
    p64 = [obk.plan_system(systems[i], 0.1, check_every=5) for i in (0, 4)]
    b.reset(p64)
    b.start(0)
    b.start(1)
    for _ in range(2):
        b.step(0.0)
    for slot, p in enumerate(p64):
        q = obk.plan_system(systems[(0, 4)[slot]], 0.1, check_every=5)
        x1, info = q.solve(maxit=10)
        q.free()
        assert np.array_equal(b.result(slot), x1)
    b.free()
    for p in p64:
        p.free()


def test_free_async_releases_on_its_stream_and_memory_is_reused():
    """obk_free_async: a plan released waiting only for its stream (no
    device-wide wait); plans built afterwards take the kept blocks and solve
    as before, bit for bit."""
    import torch
    systems = _systems()[:3]
    st = torch.cuda.Stream()
    ref = []
    for s in systems:
        p = obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8)
        ref.append(p.solve(maxit=100, tol=1e-10)[0])
        p.free(stream=st.cuda_stream)
        p.free(stream=st.cuda_stream)          # a freed handle: no-op
    _say("[batch] free_async")
    for _ in range(2):
        for s, x0 in zip(systems, ref):
            p = obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8, stream=st.cuda_stream)
            x, info = p.solve(maxit=100, tol=1e-10, stream=st.cuda_stream)
            assert info.status == "converged" and np.array_equal(x, x0)
            p.free(stream=st.cuda_stream)
    assert obk.lib().obk_free_async(None, None) == 0
    st.synchronize()


def test_batch_created_empty_then_reset():
    """A batch object created with no members steps as a no-op and takes its
    members later through obk_batch_reset; their results equal solves alone."""
    systems = _systems()[:2]
    b = obk.Batch([])
    rr, act = b.step(1e-10)
    assert rr.size == 0 and act.size == 0
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8) for s in systems]
    b.reset(plans)
    b.start(0)
    b.start(1)
    steps = [0, 0]
    for _ in range(60):
        rr, act = b.step(1e-10)
        for i in range(2):
            steps[i] += int(act[i])
        if not act.any():
            break
    _say(f"[batch] empty then reset: steps {steps}")
    for i, s in enumerate(systems):
        x = b.result(i)
        q = obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8)
        x1, info = q.solve(maxit=steps[i], tol=1e-10)
        q.free()
        assert info.outer_steps == steps[i] and np.array_equal(x, x1)
    b.free()
    for p in plans:
        p.free()
