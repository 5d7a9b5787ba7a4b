"""GPU checks of the plan options of the C ABI (obk_opts): the relaxation
omega against the oracle's relaxed sweep on every engine, the paper's pair
rule (max_group = 2) against the oracle's block form with one-row blocks,
deterministic, and a caller-supplied device allocator."""
import ctypes
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


def _close(x, xo, tol=1e-10):
    return (np.linalg.norm(x - xo) <= tol * np.linalg.norm(xo) and
            np.abs(x - xo).max() <= tol * np.abs(xo).max())


OMEGA_CASES = [
    ("c1-phases", lambda: synth.c1(), 0.1, 40, "phases", 0.7),
    ("c1-one-slab", lambda: synth.c1(), 0.1, 40, "banded", 1.4),
    ("stencil64-banded", lambda: synth.c2(grid=64), 0.1, 30, "banded", 1.3),
    ("stencil64-phases", lambda: synth.c2(grid=64), 0.1, 30, "phases", 0.6),
    ("stencil200-banded", lambda: synth.c2(grid=200), 0.1, 12, "banded", 1.2),
]


@pytest.mark.parametrize("name,maker,delta,K,engine,omega", OMEGA_CASES, ids=[c[0] for c in OMEGA_CASES])
def test_relaxed_sweeps_match_oracle(name, maker, delta, K, engine, omega):
    s = maker()
    _say(f"[options] omega={omega} {name}: n={s.n} engine={engine}")
    pl = oracle.plan_system(s, delta, omega=omega)
    with obk.plan_system(s, delta, omega=omega, sweep_kernel=engine) as P:
        assert P.engine()["engine"] == engine
        x, _ = P.solve(maxit=K)
    xo = oracle.solve(pl, K)
    _say(f"[options] {name}: maxabs {np.abs(x - xo).max():.3e} bitwise {np.array_equal(x, xo)}")
    assert _close(x, xo)


def test_relaxed_complex_sweeps_match_oracle():
    s = synth.c1z(n=1500)
    po = oracle.plan_system_complex(s, 0.1, omega=0.8)
    with obk.plan_system(s, 0.1, omega=0.8) as P:
        x, _ = P.solve(maxit=20)
    xo = oracle.solve_complex(po, 20)
    assert _close(x, xo)


def test_relaxed_refinement_and_batch():
    """FP32 sweeps + FP64 refinement with omega: converges to 1e-10; the
    batched engine equals the single solve bit for bit; the error against
    the oracle's FP64 run of the same relaxed schedule is small."""
    systems = [synth.c4_system(i, n=n, companion=True) for i, n in enumerate((3000, 11000, 1200))]
    plans = [obk.plan_system(s, 0.1, precision=obk.FP32_IR, inner_sweeps=8, omega=1.2) for s in systems]
    try:
        xs, infos = obk.solve_batch(plans, tol=1e-10, maxit=60)
        for k, p in enumerate(plans):
            assert infos[k].status == "converged"
            x1, _ = p.solve(maxit=60, tol=1e-10)
            assert np.array_equal(x1, xs[k])
        pl = oracle.plan_system(systems[0], 0.1, omega=1.2)
        xt, _, rho = oracle.refine(pl, 8, 60, 1e-10)
        x64 = oracle.unpermute(pl.p, xt)
        err = np.linalg.norm(xs[0] - x64) / np.linalg.norm(x64)
        _say(f"[options] relaxed refinement: oracle relres {rho:.2e}, error vs oracle {err:.2e}")
        assert err <= 1e-8
    finally:
        for p in plans:
            p.free()


@pytest.mark.parametrize("maker,thr", [(lambda: synth.c1(n=600), 0.1), (lambda: synth.c2(grid=40), 0.1),
                                       (lambda: synth.from_dense(np.tile(np.arange(1.0, 7.0), (6, 1)) +
                                                                 np.eye(6), f=np.ones(6)), 0.1)])
def test_pair_rule_is_the_block_form_with_one_row_blocks(maker, thr):
    """max_group = 2 (the paper's class rule: pairs of near-orthogonal rows
    projected one after the other, then Nclass row by row) equals the
    oracle's block form with k = n."""
    s = maker()
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, s.n, thr)
    with obk.plan_system(s, thr, max_group=2) as P:
        info = P.blocks()
        assert len(info["pairs"]) == len(bp.pairs) and list(info["nclass"]) == list(bp.nclass)
        x, _ = P.solve(maxit=6)
    xo = oracle.block_solve(bp, 6)
    _say(f"[options] pair rule n={s.n}: {len(bp.pairs)} pairs, {len(bp.nclass)} in Nclass, "
         f"maxabs {np.abs(x - xo).max():.2e}")
    assert _close(x, xo)


def test_deterministic_flag_changes_nothing():
    s = synth.c2(grid=100)
    with obk.plan_system(s, 0.1, deterministic=False) as P:
        a, _ = P.solve(maxit=20)
    with obk.plan_system(s, 0.1, deterministic=True) as P:
        b, _ = P.solve(maxit=20)
    assert np.array_equal(a, b)


class _HipAllocator:
    """Device memory from hipMalloc through ctypes, with a count of what is
    outstanding."""

    def __init__(self):
        self.hip = ctypes.CDLL("libamdhip64.so")
        self.hip.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.hip.hipFree.argtypes = [ctypes.c_void_p]
        self.live, self.calls, self.bytes = {}, 0, 0

    def alloc(self, nbytes):
        p = ctypes.c_void_p()
        if self.hip.hipMalloc(ctypes.byref(p), nbytes) != 0:
            return 0
        self.live[p.value] = nbytes
        self.calls += 1
        self.bytes += nbytes
        return p.value

    def dealloc(self, ptr):
        assert ptr in self.live, "dealloc of a block alloc did not return"
        del self.live[ptr]
        self.hip.hipFree(ctypes.c_void_p(ptr))


@pytest.mark.parametrize("kw", [dict(), dict(precision=1), dict(sweep_kernel="phases")])
def test_caller_allocator(kw):
    """A plan built with the caller's allocator takes every device buffer from
    it, returns every one by obk_free, and computes the same iterate as a
    plan on the runtime's allocator."""
    s = synth.c2(grid=80)
    al = _HipAllocator()
    P = obk.plan_system(s, 0.1, allocator=al, **kw)
    x, info = P.solve(maxit=12, tol=0.0)
    assert al.calls > 0 and al.live
    held = sum(al.live.values())
    P.free()
    assert not al.live, f"{len(al.live)} blocks not returned"
    with obk.plan_system(s, 0.1, **kw) as Q:
        y, _ = Q.solve(maxit=12, tol=0.0)
        own = Q.device_bytes()
    _say(f"[options] caller allocator {kw}: {al.calls} blocks, {al.bytes} bytes in all, {held} held by the plan "
         f"(plan reports {own})")
    assert np.array_equal(x, y)


def _dense_cross(n=3000, k_off=8, seed=4):
    """Nine entries per row (so the plan takes the per-row Gram kernel) plus
    one dense row and one dense column: every row shares the dense column
    with all the others, more candidates than the kernel's LDS table holds
    (its pairwise path)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    A = synth.random_rows(n, k_off, seed).scipy().tolil()
    A[0, :] = rng.standard_normal(n)
    A[:, 0] = rng.standard_normal((n, 1))
    A[0, 0] = n
    A = A.tocsr()
    A.sort_indices()
    return synth.from_scipy(A, rng.standard_normal(n), name="dense-cross")


LAMBDA_CASES = [
    ("c1", lambda: synth.c1(), 0.1, False),
    ("c1-companion", lambda: synth.c1(companion=True), 0.1, False),
    ("stencil64", lambda: synth.c2(grid=64), 0.1, False),
    ("scattered-20000", lambda: synth.c3(n=20000), 0.1, False),
    ("random-rows-delta0.4", lambda: synth.random_rows(3000, 6, 11), 0.4, False),
    ("random-rows-k19-hash-and-pairwise", lambda: synth.random_rows(4000, 19, 5), 0.1, False),
    ("dense-cross-pairwise", lambda: _dense_cross(), 0.1, False),
    ("zero-rows", lambda: synth.from_dense(np.diag([2.0, 0.0, 1.0, 0.0, 3.0])), 0.1, False),
    ("c1z", lambda: synth.c1z(), 0.1, True),
    ("c2z-grid64", lambda: synth.c2z(grid=64), 0.1, True),
    ("stencil-1024-full", lambda: synth.c2(), 0.1, False),
]


@pytest.mark.parametrize("name,maker,delta,cplx", LAMBDA_CASES, ids=[c[0] for c in LAMBDA_CASES])
def test_lambda_bound_matches_oracle(name, maker, delta, cplx):
    """obk_plan_lambda_bound: every group's Gershgorin bound on
    lambda_max(B_g B_g^H) against the oracle's (the same groups: the plans are
    bit-exact), to 1e-12 relative (the cosines are summed in another order)."""
    s = maker()
    po = oracle.plan_system_complex(s, delta) if cplx else oracle.plan_system(s, delta)
    bo, per_o = oracle.lambda_bound(po)
    with obk.plan_system(s, delta) as P:
        b, per = P.lambda_bound()
        g, ng = P.groups()
    _say(f"[lambda] {name}: {ng} groups, bound {b:.15f} (oracle {bo:.15f}), max per-group deviation "
         f"{np.abs(per - per_o).max() if ng else 0.0:.3e}")
    assert ng == po.ngroups and np.array_equal(g, po.group)
    assert per.shape == per_o.shape and np.all(np.abs(per - per_o) <= 1e-12 * per_o)
    assert b == per.max() if ng else b == 0.0


def test_lambda_bound_refused_for_block_form():
    s = synth.c1(n=600)
    with obk.plan_system(s, 0.1, block_k=8) as P:
        with pytest.raises(obk.ObkError, match="OBK_E_ARG"):
            P.lambda_bound()


def test_plan_validator_passes_on_device_plans(monkeypatch):
    """OBK_VALIDATE=1: every plan's group-major layout, column segments and
    tiles are checked on the host against their definition (no two rows of a
    group with |cos| >= delta, every entry owned once) inside obk_plan."""
    monkeypatch.setenv("OBK_VALIDATE", "1")
    cases = [(synth.c1(), 0.1, {}), (synth.c2(grid=64), 0.1, {}), (synth.c3(n=20000), 0.1, {}),
             (synth.c1(n=3000, companion=True), 0.1, dict(precision=obk.FP32_IR)), (synth.c1z(), 0.1, {}),
             (synth.random_rows(2000, 6, 12), 0.4, {})]
    for s, delta, kw in cases:
        with obk.plan_system(s, delta, **kw) as P:
            _say(f"[validate] {s.name}: {P.stats()['groups']} groups, layout valid")


LOG_CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import synth
import paper_2401_00672_amd as obk
s = synth.c1(n=600)
with obk.plan_system(s, 0.1) as P:
    P.solve(maxit=5)
plans = [obk.plan_system(synth.c1(n=n), 0.1, precision=obk.FP32_IR) for n in (500, 700, 900)]
b = obk.Batch(plans[:2])
b.begin()
b.step(1e-10)
b.reset(plans)
b.start(2)
b.step(1e-10)
b.free()
for p in plans:
    p.free()
print("child done", flush=True)
"""


def test_log_levels_name_plans_solves_and_batches():
    """OBK_LOG=3 prints a line per plan, solve, batch formation and batched
    step (the level is read once per process, so this runs in a child)."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, OBK_LOG="3")
    _say("[log] child with OBK_LOG=3")
    r = subprocess.run([sys.executable, "-c", LOG_CHILD.format(root=root)], capture_output=True, text=True,
                       timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-3000:]
    lines = [l for l in r.stderr.splitlines() if l.startswith("[obk]")]
    kinds = [l.split()[1] + (" " + l.split()[2] if l.split()[1] == "batch" else "") for l in lines]
    assert kinds.count("plan") == 4 and kinds.count("solve") == 1, lines
    assert kinds.count("batch create") == 1 and kinds.count("batch reset") == 1, lines
    assert kinds.count("batch step") == 2, lines
    assert not any("error" in l for l in lines), lines
