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
