"""Host logic of the banded sweep engine (no device): its plan-time layout
for a given slab count, run by the host emulation of the kernel, must give
the oracle's iterate bit for bit (eq. 3.3, groups in ascending order, every
row of a group from the same iterate).  This checks the slab windows, the
neighbour publications and the ELL rounds without a GPU."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
import paper_2401_00672_amd as obk


def _banded(n=3000, half=40, seed=5):
    """Random banded system: diagonal U(1, 2) + |row sum| and 6 entries per
    row within `half` of the diagonal, N(0, 1) values; rows of 1 to 7
    entries (irregular ELL rounds)."""
    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for i in range(n):
        k = int(rng.integers(0, 7))
        lo, hi = max(0, i - half), min(n, i + half + 1)
        cand = np.setdiff1d(np.arange(lo, hi), [i])
        c = rng.choice(cand, size=min(k, cand.size), replace=False)
        v = rng.standard_normal(c.size)
        rows += [i] * (c.size + 1)
        cols += list(c) + [i]
        vals += list(v) + [rng.uniform(1, 2) + np.abs(v).sum()]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return synth.from_scipy(A, rng.standard_normal(n), name="banded")


def _zero_rows_stencil():
    s = synth.c2(grid=40)
    A = s.scipy().tolil()
    A[17, :] = 0
    A[900, :] = 0
    return synth.from_scipy(A.tocsr(), s.x_star, name="stencil40-zero-rows")


CASES = [
    ("stencil64", lambda: synth.c2(grid=64), 0.1, 7, [1, 2, 4, 8, 16, 31]),
    ("stencil100-ragged", lambda: synth.c2(grid=100), 0.1, 4, [7, 20, 33]),
    ("banded-irregular", _banded, 0.1, 5, [1, 3, 16, 35]),
    ("banded-delta0.02", _banded, 0.02, 3, [5, 20]),
    ("stencil40-zero-rows", _zero_rows_stencil, 0.1, 5, [1, 4, 9]),
    ("c1-scattered-one-slab", lambda: synth.c1(n=300), 0.1, 6, [1]),
    ("single-group", lambda: synth.c2(grid=30), 1.5, 4, [1, 5]),
]


def _check_layout(name, maker, delta, K, slabs):
    """Run the layout for each slab count against the oracle; return which
    kinds of phases (cached in LDS, streamed) the runs used."""
    s = maker()
    pl = oracle.plan_system(s, delta)
    x0 = np.random.default_rng(11).standard_normal(s.n)
    want = oracle.sweep(pl, x0, K)
    kinds = set()
    for S in slabs:
        got, st = obk.banded_emulate_host(pl.rp, pl.ci, pl.v, pl.f, pl.inv, pl.group, pl.ngroups, S, K, x0)
        assert st["slabs"] == S and st["lds_bytes"] <= 159 * 1024
        kinds |= {k for k in ("cached", "streamed") if st[k] > 0}
        assert np.array_equal(got, want), (name, S, np.abs(got - want).max())
    return kinds


@pytest.mark.parametrize("name,maker,delta,K,slabs", CASES, ids=[c[0] for c in CASES])
def test_banded_layout_matches_oracle(name, maker, delta, K, slabs):
    _check_layout(name, maker, delta, K, slabs)


def test_banded_layout_covers_cached_and_streamed_phases():
    """Phases run both from the LDS cache and streamed in these cases."""
    kinds = set()
    for name, maker, delta, K, slabs in CASES[:3]:
        kinds |= _check_layout(name, maker, delta, K, slabs)
    assert kinds == {"cached", "streamed"}


def test_banded_layout_rejections():
    """A slab count whose windows reach past the neighbours, or more groups
    than the engine keeps descriptors for, is refused (OBK_E_ARG)."""
    s = synth.c2(grid=64)                       # band 64: slabs of 64 rows are too narrow
    pl = oracle.plan_system(s, 0.1)
    x0 = np.zeros(s.n)
    with pytest.raises(obk.ObkError) as e:
        obk.banded_emulate_host(pl.rp, pl.ci, pl.v, pl.f, pl.inv, pl.group, pl.ngroups, 64, 1, x0)
    assert e.value.code == -1
    t = synth.from_dense(np.tile(np.arange(1.0, 81.0), (80, 1)), f=np.ones(80))   # 80 singleton groups
    pt = oracle.plan_system(t, 0.1)
    assert pt.ngroups == 80
    with pytest.raises(obk.ObkError):
        obk.banded_emulate_host(pt.rp, pt.ci, pt.v, pt.f, pt.inv, pt.group, pt.ngroups, 1, 1, np.zeros(80))
