"""Parity at the benchmark sizes.

Scattered 2,000,000-row system (12 nnz/row):
  * the whole oracle plan (its conflict pass runs on all cores): the RCM
    permutation and every row's group are bit-exact;
  * x after 2 FP64 sweeps equals the oracle's element-wise (threaded oracle
    sweep, the same operations as the plain one);
  * FP64 sweeps never increase ||x - x*|| (the group step is non-expansive on
    a consistent system), and FP32 sweeps + FP64 refinement bring the
    row-dominant companion to relative residual 1e-10 (checked on the host),
    with its error against the oracle's FP64 refinement stated.

512 batched systems, in the launch configuration the benchmark times (tuned):
  every system's batched result equals its single solve bit for bit, and the
  smallest, median and largest systems have oracle-exact plans.
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


@pytest.mark.timeout(900)
def test_scattered_2m_full_size():
    """The whole oracle plan (RCM, conflicts on all cores, first fit) of the
    2,000,000-row system against the GPU's: permutation and groups bit-exact;
    the iterate after 2 FP64 sweeps against the oracle's (threaded sweep,
    the same operations) element-wise; FP32 sweeps + FP64 refinement on the
    companion to relative residual 1e-10, with its error against the oracle's
    FP64 run of the same refinement schedule."""
    s = synth.c3()
    n = s.n
    _say(f"[full] scattered n={n} nnz={s.nnz}: oracle plan on {oracle.max_threads()} threads")
    pl = oracle.plan_system(s, 0.1)
    _say(f"[full] scattered: oracle {pl.ngroups} groups, {pl.cidx.size} conflicts")
    with obk.plan_system(s, 0.1) as P:
        assert np.array_equal(P.perm(), pl.p), "RCM permutation differs"
        g, ng = P.groups()
        assert ng == pl.ngroups and np.array_equal(g, pl.group), "group assignment differs"
        assert P.stats()["conflicts"] == pl.cidx.size
        x2, _ = P.solve(maxit=2)
        errs = []
        for k in range(1, 5):
            x, _ = P.solve(maxit=k)
            errs.append(np.linalg.norm(x - s.x_star))
        _say(f"[full] scattered: ||x_k - x*|| = {['%.6e' % e for e in errs]}")
        assert all(b <= a for a, b in zip(errs, errs[1:]))
    ts = oracle.ThreadedSweep(pl)
    xo = oracle.unpermute(pl.p, ts.sweep(np.zeros(n), 2))
    ts.close()
    dev = np.abs(x2 - xo).max()
    _say(f"[full] scattered: 2 sweeps, max |x_gpu - x_oracle| = {dev:.3e} (max |x| {np.abs(xo).max():.3e}), "
         f"bitwise={np.array_equal(x2, xo)}")
    assert dev <= 1e-10 * np.abs(xo).max()
    sc = synth.c3(companion=True)
    with obk.plan_system(sc, 0.1, precision=obk.FP32_IR, inner_sweeps=8) as P:
        x, info = P.solve(maxit=100, tol=1e-10)
    rel = np.linalg.norm(sc.f - sc.scipy() @ x) / np.linalg.norm(sc.f)
    _say(f"[full] scattered companion fp32-ir: {info.status} steps={info.outer_steps} relres={rel:.3e}; "
         f"oracle FP64 refinement")
    assert info.status == "converged" and rel <= 1.5e-10
    plc = oracle.plan_system(sc, 0.1)
    xt64, steps64, rho64 = oracle.refine(plc, 8, 100, 1e-10)
    x64 = oracle.unpermute(plc.p, xt64)
    err = np.linalg.norm(x - x64) / np.linalg.norm(x64)
    _say(f"[full] scattered companion: oracle FP64 refinement {steps64} steps relres {rho64:.3e}; "
         f"error of the FP32+IR result vs the FP64 oracle {err:.3e}")
    assert err <= 1e-8


@pytest.mark.timeout(900)
def test_batched_512_full_size():
    sizes = synth.c4_sizes(512)
    _say(f"[full] batched: 512 systems, sum n = {int(sizes.sum())}")
    systems = [synth.c4_system(i, n=int(nn), companion=True) for i, nn in enumerate(sizes)]
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8) for s in systems]
    try:
        best, sec = obk.batch_tune(plans)
        _say(f"[full] batched: tuned {best} ({sec * 1e3:.2f} ms per step)")
        xs, infos = obk.solve_batch(plans, tol=1e-10, maxit=100, opts=best)
        assert all(i.status == "converged" for i in infos)
        for k, p in enumerate(plans):
            x1, i1 = p.solve(maxit=100, tol=1e-10)
            assert i1.outer_steps == infos[k].outer_steps
            assert np.array_equal(x1, xs[k]), f"system {k}: batch and single differ"
        order = np.argsort(sizes)
        for k in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
            _say(f"[full] batched: oracle plan of system {k} (n={systems[k].n})")
            pl = oracle.plan_system(systems[k], 0.1)
            g, ng = plans[k].groups()
            assert np.array_equal(plans[k].perm(), pl.p)
            assert ng == pl.ngroups and np.array_equal(g, pl.group)
    finally:
        for p in plans:
            p.free()
