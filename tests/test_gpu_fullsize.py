"""Parity at the benchmark sizes, where the whole oracle plan is too slow to run.

Scattered 2,000,000-row system (12 nnz/row):
  * the RCM permutation is bit-exact against the oracle's RCM, run in full;
  * the grouping is checked row by row on a random sample with the oracle's
    own cosine (O6): no sampled row shares a group with a row it conflicts
    with, and a sampled row of group c has, for every c' < c, an earlier
    conflicting row in group c' (which, with the first property, is exactly
    first-fit at that row);
  * FP64 sweeps never increase ||x - x*|| (the group step is non-expansive on
    a consistent system), and FP32 sweeps + FP64 refinement bring the
    row-dominant companion to relative residual 1e-10 (checked on the host).

512 batched systems, in the launch configuration the benchmark times (tuned):
  every system's batched result equals its single solve bit for bit, and the
  smallest, median and largest systems have oracle-exact plans.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

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


def _check_first_fit_sample(n, trp, tci, tv, nu, group, delta, rows):
    A = sp.csr_matrix((tv, tci, trp), shape=(n, n))
    C = A.tocsc()
    for i in rows:
        gi = int(group[i])
        if nu[i] == 0.0:
            assert gi == -1
            continue
        cols = tci[trp[i]:trp[i + 1]]
        cand = np.unique(np.concatenate([C.indices[C.indptr[c]:C.indptr[c + 1]] for c in cols]))
        cand = cand[cand != i]
        conf = [int(j) for j in cand
                if nu[j] != 0.0 and oracle.cosine(i, j, trp, tci, tv, nu) >= delta]
        assert all(int(group[j]) != gi for j in conf), f"row {i} shares group {gi} with a conflicting row"
        earlier = {int(group[j]) for j in conf if j < i}
        assert set(range(gi)) <= earlier, f"row {i}: group {gi} is not the first free one"


@pytest.mark.timeout(900)
def test_scattered_2m_full_size():
    s = synth.c3()
    n = s.n
    _say(f"[full] scattered n={n} nnz={s.nnz}: oracle RCM")
    p_o = oracle.rcm(n, s.row_ptr, s.col)
    trp, tci, tv, tf = oracle.permute(n, s.row_ptr, s.col, s.val, s.f, p_o)
    nu, _ = oracle.norms(n, trp, tv)
    with obk.plan_system(s, 0.1) as P:
        assert np.array_equal(P.perm(), p_o)
        g, ng = P.groups()
        assert ng == int(g.max()) + 1
        rows = np.random.default_rng(7).choice(n, 2000, replace=False)
        _say(f"[full] scattered: {ng} groups, first-fit check on {len(rows)} sampled rows")
        _check_first_fit_sample(n, trp, tci, tv, nu, g, 0.1, rows)
        errs = []
        for k in range(1, 5):
            x, _ = P.solve(maxit=k)
            errs.append(np.linalg.norm(x - s.x_star))
        _say(f"[full] scattered: ||x_k - x*|| = {['%.6e' % e for e in errs]}")
        assert all(b <= a for a, b in zip(errs, errs[1:]))
    sc = synth.c3(companion=True)
    with obk.plan_system(sc, 0.1, precision=obk.FP32_IR, inner_sweeps=8) as P:
        x, info = P.solve(maxit=100, tol=1e-10)
    rel = np.linalg.norm(sc.f - sc.scipy() @ x) / np.linalg.norm(sc.f)
    _say(f"[full] scattered companion fp32-ir: {info.status} steps={info.outer_steps} relres={rel:.3e}")
    assert info.status == "converged" and rel <= 1.5e-10


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
