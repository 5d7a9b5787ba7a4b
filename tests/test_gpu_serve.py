"""The continuous-batching server on the GPU: requests admitted while others
run must each come out equal to their solve alone (obk_solve with the same
refinement schedule), and every converged result must satisfy the residual
bound on the host."""
import sys

import numpy as np
import pytest

import synth
import paper_2401_00672_amd as obk
from paper_2401_00672_amd.serve import LibobkBackend, Request, Server, footprint_estimate, latency_summary

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.init()


def _requests(count=14, rate=400.0):
    sizes = synth.c5_sizes(count, lo=500, hi=30000)
    t = synth.c5_arrivals(count, rate)
    return [Request(i, float(t[i]), synth.c5_system(i, n=int(sizes[i]))) for i in range(count)]


def test_serving_results_equal_solve_alone():
    reqs = _requests()
    _say(f"[serve] {len(reqs)} requests, n in [{min(q.system.n for q in reqs)}, {max(q.system.n for q in reqs)}]")
    be = LibobkBackend(delta=0.1, inner_sweeps=8, planners=2)
    budget = 4 * max(footprint_estimate(q.system.n, q.system.nnz) for q in reqs)
    srv = Server(be, budget_bytes=budget, tol=1e-10, max_steps=100, planners=2)
    res = srv.run(reqs)
    _say(f"[serve] stats {srv.stats} latency {latency_summary(res)}")
    assert srv.stats["peak_bytes"] <= budget
    assert srv.stats["rebuilds"] >= 2
    for q, r in zip(reqs, res):
        assert r.status == "converged", (q.rid, r.status, r.relres)
        A = q.system.scipy()
        rel = np.linalg.norm(q.system.f - A @ r.x) / np.linalg.norm(q.system.f)
        assert rel <= 1.5e-10, (q.rid, rel)
        with obk.plan_system(q.system, 0.1, precision=obk.FP32_IR, inner_sweeps=8) as P:
            assert P.device_bytes() <= footprint_estimate(q.system.n, q.system.nnz)
            x1, info = P.solve(maxit=100, tol=1e-10)
        assert info.outer_steps == r.steps
        assert np.array_equal(x1, r.x), f"request {q.rid}: served result differs from its solve alone"
