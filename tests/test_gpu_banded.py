"""GPU parity of the banded sweep engine (one persistent launch, a slab of
the reordered unknowns per workgroup, neighbour exchanges of w) against the
FP64 oracle and against the per-group phase kernels, through the C ABI.

Bar: the iterate after K sweeps equals the oracle's bit for bit (both sum
every row and column in ascending order without contraction); the stated
contract is 1e-10 relative, the bitwise result is asserted because it holds
by construction."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2401_00672_amd as obk
from test_banded_cpu import _banded, _zero_rows_stencil

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


CASES = [
    ("stencil64", lambda: synth.c2(grid=64), 0.1, 25),
    ("stencil200-ragged", lambda: synth.c2(grid=200), 0.1, 9),
    ("stencil333", lambda: synth.c2(grid=333), 0.1, 5),
    ("banded-irregular", _banded, 0.1, 17),
    ("banded-delta0.02", _banded, 0.02, 8),
    ("stencil40-zero-rows", _zero_rows_stencil, 0.1, 11),
    ("c1-one-slab", lambda: synth.c1(), 0.1, 30),
    ("single-group", lambda: synth.c2(grid=30), 1.5, 6),
]


@pytest.mark.parametrize("name,maker,delta,K", CASES, ids=[c[0] for c in CASES])
def test_banded_engine_matches_oracle_and_phase_kernels(name, maker, delta, K):
    s = maker()
    pl = oracle.plan_system(s, delta)
    _say(f"[banded] {name}: n={s.n} nnz={s.nnz} groups={pl.ngroups} K={K}")
    with obk.plan_system(s, delta, sweep_kernel="banded") as P:
        eng = P.engine()
        _say(f"[banded] {name}: engine {eng}")
        assert eng["engine"] == "banded" and eng["slabs"] >= 1
        assert np.array_equal(P.perm(), pl.p)
        x, info = P.solve(maxit=K, tol=0.0)
    with obk.plan_system(s, delta, sweep_kernel="phases") as Q:
        assert Q.engine()["engine"] == "phases"
        xq, _ = Q.solve(maxit=K, tol=0.0)
    xo = oracle.solve(pl, K)
    _say(f"[banded] {name}: maxabs vs oracle {np.abs(x - xo).max():.3e}, vs phases {np.abs(x - xq).max():.3e}")
    assert np.array_equal(x, xo)
    assert np.array_equal(x, xq)
    assert info.sweeps == K


def test_banded_device_sweeps_and_profile():
    """Device-resident sweeps (graph replays of one launch per 8 sweeps plus
    single-sweep launches) and the profiled launch continue the same
    iterate as the oracle's."""
    s = synth.c2(grid=128)
    pl = oracle.plan_system(s, 0.1)
    with obk.plan_system(s, 0.1) as P:
        assert P.engine()["engine"] == "banded"
        x0 = np.random.default_rng(2).standard_normal(s.n)
        xt = torch.tensor(oracle.permute_vec(pl.p, x0), device="cuda")
        P.sweep_device(xt, 19)
        prof = P.sweep_profile(xt, 3)
        torch.cuda.synchronize()
        got = xt.cpu().numpy()
    assert prof[0]["name"] == "k_slab_sweeps" and prof[0]["launches"] == 1 and prof[0]["bytes"] > 0
    want = oracle.sweep(pl, oracle.permute_vec(pl.p, x0), 22)
    assert np.array_equal(got, want)


def test_banded_refused_for_a_scattered_system():
    """sweep_kernel = 2 on a system whose band fills the matrix: OBK_E_ARG;
    the default picks the phase kernels for it."""
    s = synth.c3(n=20000)
    with pytest.raises(obk.ObkError) as e:
        obk.plan_system(s, 0.1, sweep_kernel="banded")
    assert e.value.code == -1
    with obk.plan_system(s, 0.1) as P:
        assert P.engine()["engine"] == "phases"


def test_banded_full_size_stencil():
    """The benchmark system (1024 x 1024 stencil, 1,048,576 rows, symmetric
    random permutation, delta 0.1) runs on the banded engine, and its
    iterate after 3 sweeps from a random start is the oracle's, bit for bit."""
    s = synth.c2()
    _say(f"[banded] full-size stencil n={s.n}")
    pl = oracle.plan_system(s, 0.1)
    x0 = np.random.default_rng(4).standard_normal(s.n)
    with obk.plan_system(s, 0.1) as P:
        eng = P.engine()
        _say(f"[banded] full-size engine {eng}")
        assert eng["engine"] == "banded"
        x, _ = P.solve(x0=x0, maxit=3, tol=0.0)
    want = oracle.solve(pl, 3, x0=x0)
    _say(f"[banded] full-size maxabs {np.abs(x - want).max():.3e}")
    assert np.array_equal(x, want)
