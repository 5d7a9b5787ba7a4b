"""GPU parity of the block form of Algorithm 4 (k uniform blocks, exact block
projections) against the oracle's block form (through the C ABI).

Bar: the RCM permutation, the block ranges, the Oclass pairs (in the order
formed) and Nclass are exact; the |cos| table of the block centroids agrees
to 1e-12 absolute (both FP64; the two sides sum in different orders); the
iterate after K sweeps is within 1e-10 of the oracle's, relative in the
2-norm and element-wise (max |difference| over max |oracle entry|).
The oracle projects with the dense pseudo-inverse; the library runs
conjugate gradients on A_t A_t^T y = r to a relative residual of 1e-14 per
projection, so each projection carries an error of about 1e-14 times the
condition number of the block; over K k projections on these well
conditioned blocks that stays below 1e-11 (observed at most a few 1e-15
for the direct projections).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
import paper_2401_00672_amd as obk

pytestmark = pytest.mark.gpu

TOL_X = 1e-10
TOL_COS = 1e-12


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.init()


def _rel(a, b):
    """The larger of the 2-norm relative error and the element-wise one."""
    nb = np.linalg.norm(b)
    mb = np.abs(b).max() if b.size else 0.0
    return max(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0),
               (np.abs(a - b).max() if b.size else 0.0) / (mb if mb > 0 else 1.0))


def _check_plan(P, bp, k):
    assert np.array_equal(P.perm()[:bp.n], bp.p)
    info = P.blocks()
    assert info["k"] == k
    assert np.array_equal(info["bptr"], bp.bptr)
    assert info["pairs"] == [tuple(int(v) for v in pr) for pr in bp.pairs]
    assert info["nclass"] == [int(v) for v in bp.nclass]
    assert np.max(np.abs(info["cos"] - bp.cos)) <= TOL_COS
    g, ng = P.groups()
    assert ng == k
    assert np.array_equal(g, np.repeat(np.arange(k), np.diff(bp.bptr)))
    return info


CASES = [
    # (name, system maker, k, thr, sweeps)
    ("c1-companion-600/k1", lambda: synth.c1(n=600, companion=True), 1, 0.02, 2),
    ("c1-companion-600/k3", lambda: synth.c1(n=600, companion=True), 3, 0.02, 3),
    ("c1-companion-600/k10", lambda: synth.c1(n=600, companion=True), 10, 0.02, 3),
    ("c1-companion-600/k10/thr0.1", lambda: synth.c1(n=600, companion=True), 10, 0.1, 3),
    ("c1-601/k6-ragged", lambda: synth.c1(n=601), 6, 0.1, 2),
    ("stencil24/k6", lambda: synth.c2(grid=24), 6, 0.02, 3),
    ("stencil24/k16", lambda: synth.c2(grid=24), 16, 0.02, 3),
    ("c1-40/k40-rows", lambda: synth.c1(n=40, companion=True), 40, 0.1, 2),
]


WIDE_BAND = {"c1-companion-600/k1", "c1-companion-600/k3"}
NARROW_BAND = {"c1-601/k6-ragged", "stencil24/k6", "stencil24/k16", "c1-40/k40-rows"}


@pytest.mark.parametrize("solver", ["direct", "cg"])
@pytest.mark.parametrize("name,maker,k,thr,sweeps", CASES, ids=[c[0] for c in CASES])
def test_block_form_matches_oracle(name, maker, k, thr, sweeps, solver):
    s = maker()
    _say(f"[block] {name} ({solver}): n={s.n} nnz={s.nnz} k={k} thr={thr} sweeps={sweeps}")
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, thr)
    x_o = oracle.block_solve(bp, sweeps)
    with obk.plan_system(s, thr, block_k=k, block_solver=solver) as P:
        info_b = _check_plan(P, bp, k)
        x, info = P.solve(maxit=sweeps)
        b = P.blocks()
        it, direct = b["cg_iters"], b["direct"]
        err = _rel(x, x_o)
        _say(f"[block] {name} ({solver}): |x - x_oracle| / |x_oracle| = {err:.3e}, direct blocks "
             f"{int(direct.sum())}/{k} (bandwidths {b['factor_bandwidth'].tolist()}), CG iterations {it.tolist()}")
        assert info.sweeps == sweeps
        assert err <= TOL_X
        if solver == "cg":
            assert not direct.any()
        else:
            assert direct.all()               # these blocks have full row rank
            assert not it.any()
            # both triangular-solve forms are exercised: one-wave window for
            # bands under 64, panels for wider ones
            if name in WIDE_BAND:
                assert (b["factor_bandwidth"] >= 64).all()
            if name in NARROW_BAND:
                assert (b["factor_bandwidth"] < 64).all()
        # bitwise repeatable
        x2, _ = P.solve(maxit=sweeps)
        assert np.array_equal(x, x2)


def test_block_form_direct_at_block_size_1024():
    """Blocks of 1024 rows of a stencil: in the global order their Gram
    matrix has a band of about twice the grid side, and the block's own
    reverse Cuthill-McKee order brings the factor's band below the grid side.
    The direct projections reproduce the oracle's pseudo-inverse projections
    and agree with the CG ones."""
    s = synth.c2(grid=64)
    k, thr, sweeps = 4, 0.02, 2
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, thr)
    x_o = oracle.block_solve(bp, sweeps)
    with obk.plan_system(s, thr, block_k=k) as P:
        x, _ = P.solve(maxit=sweeps)
        b = P.blocks()
    with obk.plan_system(s, thr, block_k=k, block_solver="cg") as P:
        x_cg, _ = P.solve(maxit=sweeps)
    _say(f"[block] stencil64 k=4 direct: err {_rel(x, x_o):.3e}, vs CG {_rel(x, x_cg):.3e}, "
         f"bandwidths {b['factor_bandwidth'].tolist()}")
    assert b["direct"].all() and (b["factor_bandwidth"] < 64).all()
    assert _rel(x, x_o) <= TOL_X and _rel(x, x_cg) <= TOL_X


def test_block_form_mixed_direct_and_cg_blocks():
    """Rows 3 and 7 made identical land in one of three blocks (RCM
    positions 227 and 204 of 300): that block keeps CG, the other two are
    projected from their factors in the same launch, and the iterate is the
    oracle's."""
    base = synth.c1(n=300, companion=True)
    A = base.scipy().tolil()
    A[7, :] = A[3, :]
    A = A.tocsr()
    A.sort_indices()
    s = synth.from_scipy(A, base.x_star, name="dup-row")
    k, sweeps = 3, 3
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, 0.02)
    x_o = oracle.block_solve(bp, sweeps)
    with obk.plan_system(s, 0.02, block_k=k) as P:
        x, _ = P.solve(maxit=sweeps)
        x2, _ = P.solve(maxit=sweeps)
        b = P.blocks()
        import torch
        prof = P.sweep_profile(torch.zeros(s.n, dtype=torch.float64, device="cuda"), 1)
    _say(f"[block] mixed: direct {b['direct'].tolist()}, CG iterations {b['cg_iters'].tolist()}, "
         f"err {_rel(x, x_o):.3e}, kernel {prof[0]['name']}")
    assert b["direct"].tolist() == [True, True, False]
    assert b["cg_iters"][2] > 0 and b["cg_iters"][0] == 0 and b["cg_iters"][1] == 0
    assert prof[0]["name"] == "k_block_sweeps"
    assert _rel(x, x_o) <= TOL_X and np.array_equal(x, x2)


def test_block_form_dense_column_keeps_cg():
    """A single 4,200-row block whose first column is dense has 4,200^2 row
    pairs sharing that column, over the 2^24 limit of the factor's Gram
    graph: the block keeps CG, and one projection onto the whole consistent
    system still lands on its minimum-norm solution."""
    n = 4200
    rng = np.random.default_rng(23)
    A = sp.lil_matrix((n, n))
    A.setdiag(rng.uniform(1, 2, n) + n ** 0.5)
    A[0, :] = rng.standard_normal(n)
    A[:, 0] = rng.standard_normal((n, 1))
    A[0, 0] = n
    s = synth.from_scipy(A.tocsr(), rng.standard_normal(n), name="arrow-4200")
    with obk.plan_system(s, 0.02, block_k=1) as P:
        x, info = P.solve(maxit=1)
        b = P.blocks()
    _say(f"[block] dense column: direct {b['direct'].tolist()}, CG iterations {b['cg_iters'].tolist()}, "
         f"relres {info.relres:.3e}, |x - x*| / |x*| = {_rel(x, s.x_star):.3e}")
    assert not b["direct"].any() and b["cg_iters"][0] > 0
    assert info.relres <= 1e-11 and _rel(x, s.x_star) <= 1e-10


def test_block_form_rank_deficient_block_keeps_cg():
    """A block with two identical rows has no Cholesky factor (the pivot
    test fails): it is projected by CG, and the least-norm projection is
    still the oracle's."""
    base = synth.c1(n=300, companion=True)
    A = base.scipy().tolil()
    A[7, :] = A[3, :]
    A = A.tocsr()
    A.sort_indices()
    s = synth.from_scipy(A, base.x_star, name="dup-row")
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, 1, 0.02)
    x_o = oracle.block_solve(bp, 1)
    with obk.plan_system(s, 0.02, block_k=1) as P:
        x, _ = P.solve(maxit=1)
        b = P.blocks()
    _say(f"[block] duplicated row, k=1: direct {b['direct'].tolist()}, err {_rel(x, x_o):.3e}")
    assert not b["direct"].any() and b["cg_iters"].sum() > 0
    assert _rel(x, x_o) <= TOL_X


def test_block_form_single_block_is_the_least_norm_solution():
    """k = 1: one projection onto the whole consistent system lands on the
    minimum-norm solution from x0 = 0 (eq. 3.3 with A_t = A)."""
    s = synth.c1(n=500, companion=True)
    with obk.plan_system(s, 0.02, block_k=1) as P:
        x, info = P.solve(maxit=1)
    _say(f"[block] k=1: |x - x*| / |x*| = {_rel(x, s.x_star):.3e}, relres {info.relres:.3e}")
    assert _rel(x, s.x_star) <= 1e-11
    assert info.relres <= 1e-11


@pytest.mark.parametrize("wgs", [2, 7, 32])
def test_block_form_multi_workgroup_launch(wgs):
    """The projection launch split over several workgroups (grid barriers
    between the CG phases) gives the oracle's iterate as well."""
    s = synth.c1(n=3001, companion=True)
    k, thr, sweeps = 4, 0.02, 2
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, thr)
    x_o = oracle.block_solve(bp, sweeps)
    with obk.plan_system(s, thr, block_k=k, block_wgs=wgs) as P:
        _check_plan(P, bp, k)
        x, _ = P.solve(maxit=sweeps)
        x2, _ = P.solve(maxit=sweeps)
        P.set_opts(block_wgs=1)
        x1, _ = P.solve(maxit=sweeps)
    _say(f"[block] wgs={wgs}: err {_rel(x, x_o):.3e}, vs one workgroup {_rel(x, x1):.3e}")
    assert _rel(x, x_o) <= TOL_X
    assert np.array_equal(x, x2)
    assert _rel(x, x1) <= TOL_X


def test_block_form_underdetermined():
    """m < n (Algorithm 6): [A; O] appends zero rows with a zero right-hand
    side; they take no part in a projection."""
    s = synth.rect(150, 200, 0.05)
    k, thr, sweeps = 8, 0.02, 3
    N, rp, ci, v, f = oracle.pad_square(s.m, s.n, s.row_ptr, s.col, s.val, s.f)
    bp = oracle.block_plan(N, rp, ci, v, f, k, thr)
    x_o = oracle.block_solve(bp, sweeps)
    with obk.plan_system(s, thr, block_k=k) as P:
        _check_plan(P, bp, k)
        x, _ = P.solve(maxit=sweeps)
    _say(f"[block] UOBK 150x200 k=8: err {_rel(x, x_o):.3e}")
    assert _rel(x, x_o) <= TOL_X


@pytest.mark.parametrize("solver", ["direct", "cg"])
def test_block_form_all_zero_blocks(solver):
    """Isolated unknowns (an empty row and an empty column each) come last in
    the RCM order, so the last blocks hold only zero rows: their centroid is
    0, their cosine with every block is 0 and their projection is empty
    (no CG iteration; a unit factor and y = 0 in the direct form)."""
    base = synth.c1(n=300, companion=True)
    A = sp.bmat([[base.scipy(), None], [None, sp.csr_matrix((100, 100))]]).tocsr()
    xs = np.concatenate([base.x_star, np.zeros(100)])
    s = synth.from_scipy(A, xs)
    k, thr, sweeps = 8, 0.02, 3
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, thr)
    x_o = oracle.block_solve(bp, sweeps)
    zero_blocks = [b for b in range(k) if not np.any(bp.cos[b] > 0)]
    assert zero_blocks == [6, 7]
    with obk.plan_system(s, thr, block_k=k, block_solver=solver) as P:
        _check_plan(P, bp, k)
        x, _ = P.solve(maxit=sweeps)
        it, direct = P.blocks()["cg_iters"], P.blocks()["direct"]
    _say(f"[block] zero blocks {zero_blocks} ({solver}): CG iterations {it.tolist()}, err {_rel(x, x_o):.3e}")
    if solver == "cg":
        assert all(it[b] == 0 for b in zero_blocks) and all(it[b] > 0 for b in range(6))
    else:
        assert direct.all() and not it.any()
    assert _rel(x, x_o) <= TOL_X


def test_block_form_overdetermined():
    """m > n (Algorithm 5): [A, O], x = x^(1:n)."""
    s = synth.rect(300, 200, 0.03)
    k, thr, sweeps = 5, 0.05, 3
    N, rp, ci, v, f = oracle.pad_square(s.m, s.n, s.row_ptr, s.col, s.val, s.f)
    bp = oracle.block_plan(N, rp, ci, v, f, k, thr)
    x_o = oracle.block_solve(bp, sweeps)[:s.n]
    with obk.plan_system(s, thr, block_k=k) as P:
        _check_plan(P, bp, k)
        x, _ = P.solve(maxit=sweeps)
    _say(f"[block] SOBK 300x200 k=5: err {_rel(x, x_o):.3e}")
    assert _rel(x, x_o) <= TOL_X


def test_block_form_tolerance_stops_and_converges():
    """Checked solve: the residual falls below tol on a consistent system and
    the sweep count is the oracle's (the first sweep count at which the
    oracle's iterate meets tol)."""
    s = synth.c1(n=600, companion=True)
    k, thr, tol = 10, 0.02, 1e-8
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, thr)
    A = s.scipy()
    xs = np.zeros(s.n)
    xt = oracle.permute_vec(bp.p, xs)
    want = None
    for sw in range(1, 200):
        xt = oracle.block_sweep(bp, xt, 1)
        x = oracle.unpermute(bp.p, xt)
        if np.linalg.norm(s.f - A @ x) / np.linalg.norm(s.f) <= tol:
            want = sw
            break
    assert want is not None
    with obk.plan_system(s, thr, block_k=k) as P:
        x, info = P.solve(maxit=500, tol=tol)
    _say(f"[block] c1-companion-600 k=10 to {tol}: {info.sweeps} sweeps (oracle {want}), relres {info.relres:.3e}")
    assert info.status == "converged" and info.relres <= tol
    assert info.sweeps == want


@pytest.mark.parametrize("solver", ["direct", "cg"])
def test_block_form_sweep_device_and_profile(solver):
    """Device-resident sweeps and the per-kernel profile of the block form
    (one launch; bytes from the factor bands, or from the CG iteration
    counts)."""
    import torch
    s = synth.c2(grid=48)
    k, thr, sweeps = 8, 0.02, 2
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, thr)
    xt_o = oracle.block_sweep(bp, np.zeros(s.n), sweeps)
    with obk.plan_system(s, thr, block_k=k, block_solver=solver) as P:
        xt = torch.zeros(s.n, dtype=torch.float64, device="cuda")
        P.sweep_device(xt, sweeps)
        torch.cuda.synchronize()
        assert _rel(xt.cpu().numpy(), xt_o) <= TOL_X
        it0 = P.blocks()["cg_iters"].sum()
        prof = P.sweep_profile(xt, 1)
        it1 = P.blocks()["cg_iters"].sum()
    _say(f"[block] profile ({solver}) {prof}, CG iterations {it1 - it0}")
    assert len(prof) == 1 and prof[0]["seconds"] > 0 and prof[0]["bytes"] > 0
    if solver == "cg":
        assert prof[0]["name"] == "k_block_sweeps" and it1 > it0
    else:
        assert prof[0]["name"] == "k_block_direct" and it1 == it0


def test_block_form_rejected_by_batch():
    s = synth.c1(n=200, companion=True)
    with obk.plan_system(s, 0.02, block_k=2) as P:
        with pytest.raises(obk.ObkError) as ei:
            obk.Batch([P])
        assert ei.value.code == -1
        with pytest.raises(obk.ObkError):
            P.set_opts(precision=obk.FP32_IR)


@pytest.mark.parametrize("name,maker,thr", [
    ("stencil24", lambda: synth.c2(grid=24), 0.02),
    ("c1-companion-600", lambda: synth.c1(n=600, companion=True), 0.02),
    ("c1-500", lambda: synth.c1(n=500), 0.1),
])
def test_block_count_selection_matches_oracle(name, maker, thr):
    """Section 3.6: zn and nn of every candidate k, and the chosen k, equal the
    oracle's (zn exactly: it counts exact zeros of the cosine table)."""
    s = maker()
    cands = list(range(2, 20))
    want = oracle.block_k_scores(s.n, s.row_ptr, s.col, s.val, s.f, thr, cands)
    k_o = oracle.select_block_k(want)
    k, got = obk.select_block_k(s, thr, cands)
    _say(f"[block] {name}: chosen k {k} (oracle {k_o}); zn/nn {[(a, round(b, 4), round(c, 4)) for a, b, c in got]}")
    for (ka, za, na), (kb, zb, nb) in zip(got, want):
        assert ka == kb and za == zb and abs(na - nb) <= 1e-12
    assert k == k_o
    with obk.plan_system(s, thr, block_k=k) as P:
        zn, nn = P.block_zn_nn()
    assert (zn, nn) == next((z, q) for kk, z, q in got if kk == k)


def test_block_form_iteration_cap_and_budget():
    """block_maxit caps every projection's CG iterations (the result is then
    an approximate projection, still repeatable); an HBM budget below the
    plan's footprint is refused."""
    s = synth.c2(grid=32)
    k = 4
    with obk.plan_system(s, 0.02, block_k=k, block_maxit=3, block_solver="cg") as P:
        x1, _ = P.solve(maxit=2)
        it = P.blocks()["cg_iters"]
        x2, _ = P.solve(maxit=2)
        assert np.array_equal(x1, x2)
    assert all(0 < v <= 3 * 2 for v in it), it      # 2 sweeps x at most 3 iterations
    with pytest.raises(obk.ObkError) as ei:
        obk.plan_system(s, 0.02, block_k=k, hbm_budget=1 << 16)
    assert ei.value.code == -5
