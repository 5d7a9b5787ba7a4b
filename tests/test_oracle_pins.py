"""Pins of the FP64 CPU oracle against facts fixed outside it.

Each test names what it pins: a hand-worked case, a closed form, a textbook
routine (numpy pseudo-inverse, dense Gram matrix, classic row Kaczmarz) or an
invariant the paper states.  None of them re-types the oracle's own formula.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
import synth
from conftest import parse_golden


def _csr(M):
    A = sp.csr_matrix(np.asarray(M, dtype=np.float64))
    A.sort_indices()
    return (np.ascontiguousarray(A.indptr, np.int64), np.ascontiguousarray(A.indices, np.int32),
            np.ascontiguousarray(A.data, np.float64))


def _identity_plan(M, f, delta):
    """Plan steps O5-O7 on a matrix taken as already reordered (P = I)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    rp, ci, v = _csr(M)
    nu, inv = oracle.norms(n, rp, v)
    cptr, cidx = oracle.conflicts(n, rp, ci, v, nu, delta)
    g, ng = oracle.groups(n, nu, cptr, cidx)
    return oracle.Plan(n, np.arange(n, dtype=np.int32), rp, ci, v, np.asarray(f, np.float64),
                       nu, inv, cptr, cidx, g, ng)


def _bandwidth(rp, ci):
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return int(np.abs(rows - ci).max()) if ci.size else 0


def _kaczmarz_textbook(M, f, x, order):
    """Classic row Kaczmarz, eq. (1.2), dense, one row after another."""
    x = np.array(x, dtype=np.float64)
    for i in order:
        a = M[i]
        x = x + (f[i] - a @ x) / (a @ a) * a
    return x


# ----------------------------------------------------------------- P8: RCM
@pytest.mark.parametrize("case", parse_golden("rcm_hand.txt"), ids=lambda c: c["name"])
def test_rcm_hand_worked(case):
    """O3 against orders worked by hand from the tie-break rule (Section 3.2)."""
    n = int(case["n"])
    M = np.eye(n)
    for e in case["stored"].split():
        r, c = map(int, e.split("-"))
        M[r, c] = 1.0
    rp, ci, v = _csr(M)
    p = oracle.rcm(n, rp, ci)
    assert p.tolist() == [int(t) for t in case["p"].split()]
    assert p[::-1].tolist() == [int(t) for t in case["cm"].split()]


def test_rcm_scrambled_path_has_bandwidth_one():
    """A randomly labelled path is a band of width 1 after RCM."""
    n = 500
    perm = np.random.default_rng(7).permutation(n)
    M = sp.lil_matrix((n, n))
    for t in range(n):
        M[perm[t], perm[t]] = 2.0
        if t + 1 < n:
            M[perm[t], perm[t + 1]] = -1.0
            M[perm[t + 1], perm[t]] = -1.0
    s = synth.from_scipy(M.tocsr())
    pl = oracle.plan_system(s, 0.1)
    assert _bandwidth(pl.rp, pl.ci) == 1


@pytest.mark.parametrize("grid", [8, 32, 64])
def test_rcm_grid_bandwidth(grid):
    """A scrambled N x N grid comes back with bandwidth N (a level-set band;
    Table 1 and Fig. 2 show RCM restoring a band)."""
    s = synth.c2(grid=grid)
    before = _bandwidth(s.row_ptr, s.col)
    pl = oracle.plan_system(s, 0.1)
    after = _bandwidth(pl.rp, pl.ci)
    assert after <= 2 * grid - 1
    assert after == grid
    assert before > 4 * grid


def test_rcm_is_a_permutation_and_close_to_scipy():
    """Sanity against scipy's RCM (different tie-break, so not parity)."""
    for s in (synth.c1(), synth.c2(grid=48)):
        p = oracle.rcm(s.n, s.row_ptr, s.col)
        assert np.array_equal(np.sort(p), np.arange(s.n))
        A = s.scipy()
        pat = ((A + A.T) != 0).astype(np.int8).tocsr()
        ps = csg.reverse_cuthill_mckee(pat, symmetric_mode=True)
        bw_o = _bandwidth(*_csr_perm(A, p))
        bw_s = _bandwidth(*_csr_perm(A, ps))
        assert bw_o <= 1.5 * bw_s


def _csr_perm(A, p):
    B = A[p][:, p].tocsr()
    B.sort_indices()
    return B.indptr.astype(np.int64), B.indices.astype(np.int32)


# ------------------------------------------------------------- O4 permute
def test_permute_matches_dense_symmetric_permutation():
    """A~ = P A P^T, f~ = P f (eqs. 3.1-3.2) against dense fancy indexing."""
    s = synth.c1(n=300)
    p = oracle.rcm(s.n, s.row_ptr, s.col)
    trp, tci, tv, tf = oracle.permute(s.n, s.row_ptr, s.col, s.val, s.f, p)
    D = s.scipy().toarray()
    Dt = D[p][:, p]
    got = sp.csr_matrix((tv, tci, trp), shape=(s.n, s.n)).toarray()
    assert np.array_equal(got, Dt)
    assert np.array_equal(tf, s.f[p])
    for i in range(s.n):
        row = tci[trp[i]:trp[i + 1]]
        assert np.all(np.diff(row) > 0)


def test_error_norm_invariant_under_permutation():
    """eq. (3.4): ||x_j - x*|| is the same in reordered and original coordinates."""
    s = synth.c1(n=400)
    pl = oracle.plan_system(s, 0.1)
    xt = oracle.sweep(pl, np.zeros(s.n), 7)
    xs_t = oracle.permute_vec(pl.p, s.x_star)
    x = oracle.unpermute(pl.p, xt)
    assert np.linalg.norm(xt - xs_t) == np.linalg.norm(x - s.x_star)
    assert np.array_equal(oracle.permute_vec(pl.p, x), xt)


# ------------------------------------------------- P9: norms and cosines
def test_cosines_against_dense_gram():
    """O5-O6 against |D^-1/2 A A^T D^-1/2| from a dense Gram matrix."""
    for s in (synth.c1(n=250), synth.c2(grid=12), synth.c1(n=200, companion=True)):
        n = s.n
        rp, ci, v = s.row_ptr, s.col, s.val
        nu, inv = oracle.norms(n, rp, v)
        D = s.scipy().toarray()
        assert np.allclose(nu, (D * D).sum(1), rtol=4e-16 * 16, atol=0)
        G = D @ D.T
        C = np.abs(G) / np.sqrt(np.outer(nu, nu))
        pattern = ((np.abs(D) > 0).astype(float) @ (np.abs(D) > 0).T.astype(float)) > 0
        for delta in (0.02, 0.1, 0.3):
            cptr, cidx = oracle.conflicts(n, rp, ci, v, nu, delta)
            got = set()
            for i in range(n):
                for j in cidx[cptr[i]:cptr[i + 1]]:
                    got.add((i, int(j)))
            near = np.abs(C - delta) < 1e-12
            want = set()
            for i in range(n):
                for j in range(i):
                    if pattern[i, j] and C[i, j] >= delta:
                        want.add((i, j))
            ambiguous = {(i, j) for i in range(n) for j in range(i) if near[i, j]}
            assert got - ambiguous == want - ambiguous
        # individual cosines within a few ulp of the dense value
        rng = np.random.default_rng(1)
        for _ in range(200):
            i, j = rng.integers(0, n, 2)
            c = oracle.cosine(i, j, rp, ci, v, nu)
            if pattern[i, j]:
                assert abs(c - C[i, j]) <= 8 * np.finfo(float).eps * max(C[i, j], 1e-300) + 1e-17
            else:
                assert c == 0.0


@pytest.mark.parametrize("case", [c for c in parse_golden("hand_cases.txt") if "conflicts" in c],
                         ids=lambda c: c["name"])
def test_conflicts_groups_pairs_hand_worked(case):
    """O6, O7 and the literal pair rule of Section 3.3 on cases worked by hand."""
    M = np.array(case["row"])
    n = M.shape[0]
    delta = float(case["delta"])
    pl = _identity_plan(M, np.zeros(n), delta)
    want = {}
    for tok in case["conflicts"].split():
        i, js = tok.split(":")
        want[int(i)] = [int(j) for j in js.split(",")]
    for i in range(n):
        assert pl.cidx[pl.cptr[i]:pl.cptr[i + 1]].tolist() == want.get(i, [])
    assert pl.group.tolist() == [int(t) for t in case["groups"].split()]
    got_pairs = oracle.pairs(n, pl.rp, pl.ci, pl.v, pl.nu, delta)
    assert got_pairs.tolist() == [int(t) for t in case["pairs"].split()]


# --------------------------------------------------------- P10: groups
def _mis_peeling(n, conflict_sets):
    """Independent statement of the class{i} rule taken to maximal classes:
    repeatedly open a class at the first unassigned row and add every later
    unassigned row that conflicts with none of the class so far."""
    group = [-1] * n
    g = 0
    while True:
        members = []
        for i in range(n):
            if group[i] != -1:
                continue
            if all(j not in conflict_sets[i] for j in members):
                members.append(i)
        if not members:
            break
        for i in members:
            group[i] = g
        g += 1
        if all(x != -1 for x in group):
            break
    return group


@pytest.mark.parametrize("maker", [lambda: synth.c1(n=600), lambda: synth.c2(grid=20),
                                   lambda: synth.c1(n=300, companion=True)])
def test_groups_valid_first_fit_and_peeling(maker):
    s = maker()
    pl = oracle.plan_system(s, 0.1)
    n = s.n
    conf = [set() for _ in range(n)]
    for i in range(n):
        for j in pl.cidx[pl.cptr[i]:pl.cptr[i + 1]]:
            conf[i].add(int(j))
            conf[int(j)].add(i)
    g = pl.group
    # validity: no conflict inside a group
    for i in range(n):
        for j in conf[i]:
            assert g[i] != g[j]
    # first-fit property: a row of group c has an earlier conflicting row in every group < c
    for i in range(n):
        earlier = {int(g[j]) for j in conf[i] if j < i}
        assert set(range(g[i])) <= earlier
    # equality with the peeling statement of the class rule
    assert _mis_peeling(n, conf) == g.tolist()


# --------------------------------------- P1/P4: hand-worked sweeps (Fig. 1)
@pytest.mark.parametrize("case", [c for c in parse_golden("hand_cases.txt") if "x1" in c],
                         ids=lambda c: c["name"])
def test_sweep_hand_worked(case):
    M = np.array(case["row"])
    f = np.array([float(t) for t in case["f"].split()])
    xs = np.array([float(t) for t in case["xstar"].split()])
    s = synth.from_dense(M, xs, f)
    pl = oracle.plan_system(s, float(case["delta"]))
    if "p" in case:
        assert pl.p.tolist() == [int(t) for t in case["p"].split()]
    assert pl.group.tolist() == [int(t) for t in case["groups"].split()]
    x1 = oracle.solve(pl, 1)
    np.testing.assert_allclose(x1, [float(t) for t in case["x1"].split()], rtol=0, atol=4e-16)
    if "x2" in case:
        x2 = oracle.solve(pl, 2)
        np.testing.assert_allclose(x2, [float(t) for t in case["x2"].split()], rtol=0, atol=4e-16)
    if "rate" in case:
        # eq. (3.15): each projection multiplies the error by cos(theta)
        errs = [np.linalg.norm(oracle.solve(pl, k) - xs) for k in range(1, 8)]
        ratios = np.array(errs[1:]) / np.array(errs[:-1])
        np.testing.assert_allclose(ratios, float(case["rate"]), rtol=1e-10)


def test_single_row_projection_lands_on_hyperplane():
    """eq. (1.2): after projecting row i, a_i x = f_i (to rounding)."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        M = np.diag(rng.uniform(1, 2, 4))
        M[0] = rng.standard_normal(4)
        M[0, 0] = 3.0
        f = rng.standard_normal(4)
        pl = _identity_plan(M, f, 0.1)
        x0 = rng.standard_normal(4)
        rows = np.array([0], np.int32)
        x = oracle.rowwise(4, pl.rp, pl.ci, pl.v, f, pl.inv, rows, x0)
        assert abs(M[0] @ x - f[0]) <= 8e-16 * (np.abs(M[0]) @ np.abs(x) + abs(f[0]))
        np.testing.assert_allclose(x, _kaczmarz_textbook(M, f, x0, [0]), rtol=1e-15, atol=1e-15)


# ---------------------------------- P2/P3/P5: exactly orthogonal groups
def _hadamard(k):
    H = np.array([[1.0]])
    while H.shape[0] < k:
        H = np.block([[H, H], [H, -H]])
    return H


def _one_group_plan(M, f, rows):
    """A plan whose only group is `rows` (other rows left out)."""
    pl = _identity_plan(M, f, 0.1)
    g = np.full(M.shape[0], -1, np.int32)
    g[np.asarray(rows)] = 0
    pl.group = g
    pl.ngroups = 1
    return pl


@pytest.mark.parametrize("kind", ["hadamard", "disjoint", "orthogonal_dense"])
def test_group_step_equals_pseudoinverse_projection(kind):
    """O8 on an exactly orthogonal group equals eq. (1.3) with numpy's pinv,
    equals sequential eq. (1.2) in any order (P3), and obeys the Pythagorean
    identity of eq. (3.8) (P5)."""
    rng = np.random.default_rng({"hadamard": 1, "disjoint": 2, "orthogonal_dense": 3}[kind])
    n = 8
    M = np.diag(rng.uniform(1, 2, n))
    if kind == "hadamard":
        rows = [0, 2, 5, 7]
        H = _hadamard(8)
        for t, r in enumerate(rows):
            M[r] = H[t] * rng.choice([1.0, 2.0, 0.5])
    elif kind == "disjoint":
        rows = [0, 1, 2]
        M[0] = 0; M[1] = 0; M[2] = 0
        M[0, [0, 3]] = rng.standard_normal(2)
        M[1, [1, 4, 6]] = rng.standard_normal(3)
        M[2, [2, 5, 7]] = rng.standard_normal(3)
    else:
        rows = [1, 3, 4, 6]
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        for t, r in enumerate(rows):
            M[r] = Q[t] * rng.uniform(0.5, 2)
    f = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    pl = _one_group_plan(M, f, rows)
    x1 = oracle.sweep(pl, x0, 1)
    Ag = M[rows]
    want = x0 + np.linalg.pinv(Ag) @ (f[rows] - Ag @ x0)
    np.testing.assert_allclose(x1, want, rtol=1e-14, atol=1e-14 * np.abs(want).max())
    for order in (rows, rows[::-1], list(rng.permutation(rows))):
        np.testing.assert_allclose(x1, _kaczmarz_textbook(M, f, x0, order), rtol=1e-14,
                                   atol=1e-14 * np.abs(want).max())
    # eq. (3.8) with x* any point on all the group's hyperplanes
    xs = rng.standard_normal(n)
    f2 = f.copy()
    f2[rows] = Ag @ xs
    pl2 = _one_group_plan(M, f2, rows)
    x1 = oracle.sweep(pl2, x0, 1)
    lhs = np.linalg.norm(x1 - xs) ** 2
    rhs = np.linalg.norm(x0 - xs) ** 2 - np.linalg.norm(x1 - x0) ** 2
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(x0 - xs) ** 2


def test_all_orthogonal_rows_solve_in_one_sweep():
    """Fig. 1 (right) and bcsstm39's IT = 1 (Table 4; nnz = rows, Table 3):
    mutually orthogonal rows form one group and one sweep is exact."""
    rng = np.random.default_rng(5)
    n = 64
    cases = []
    cases.append(np.diag(rng.uniform(0.5, 3, n)))                      # diagonal
    P = np.eye(n)[rng.permutation(n)] * rng.uniform(0.5, 3, n)[:, None]  # scaled permutation
    cases.append(P)
    Q, _ = np.linalg.qr(rng.standard_normal((16, 16)))                   # dense orthogonal
    cases.append(Q)
    for M in cases:
        xs = rng.standard_normal(M.shape[0])
        s = synth.from_dense(M, xs)
        pl = oracle.plan_system(s, 0.1)
        assert pl.ngroups == 1
        x = oracle.solve(pl, 1)
        np.testing.assert_allclose(x, xs, rtol=0, atol=1e-13 * np.abs(xs).max())


def test_identity_gives_f_after_one_sweep():
    """Identity: one group, x = f after one sweep (exactly)."""
    n = 50
    f = np.random.default_rng(8).standard_normal(n)
    s = synth.from_dense(np.eye(n), f=f)
    pl = oracle.plan_system(s, 0.1)
    assert pl.ngroups == 1
    assert np.array_equal(oracle.solve(pl, 1), f)


def test_identical_rows_are_singletons_and_sequential():
    """All rows identical: every pair has |cos| = 1, so n singleton groups and
    the sweep is classic sequential Kaczmarz; a consistent f is met after one
    sweep."""
    n = 12
    rng = np.random.default_rng(9)
    a = rng.standard_normal(n)
    M = np.tile(a, (n, 1))
    xs = rng.standard_normal(n)
    f = M @ xs
    pl = _identity_plan(M, f, 0.1)
    assert pl.ngroups == n
    assert sorted(pl.group.tolist()) == list(range(n))
    x0 = rng.standard_normal(n)
    x = oracle.sweep(pl, x0, 1)
    np.testing.assert_allclose(x, _kaczmarz_textbook(M, f, x0, list(range(n))), rtol=1e-13, atol=1e-13)
    assert np.abs(M @ x - f).max() < 1e-12 * np.abs(f).max()


def test_threshold_above_one_gives_single_simultaneous_step():
    """delta > 1: no pair can conflict (|cos| <= 1), one group, and one sweep is
    the simultaneous step x + A^T D^-1 (f - A x) of all rows."""
    s = synth.c1(n=150)
    pl = oracle.plan_system(s, 1.5)
    assert pl.ngroups == 1
    D = sp.csr_matrix((pl.v, pl.ci, pl.rp), shape=(s.n, s.n)).toarray()
    x0 = np.random.default_rng(2).standard_normal(s.n)
    want = x0 + D.T @ ((pl.f - D @ x0) / (D * D).sum(1))
    np.testing.assert_allclose(oracle.sweep(pl, x0, 1), want, rtol=1e-12, atol=1e-12)


# -------------------------------------------- P7: convergence (Theorem 1)
def test_converges_to_generating_solution():
    """Theorem 1: consistent systems converge to x* (= A^+ f, A nonsingular)."""
    s = synth.c1(companion=True)
    pl = oracle.plan_system(s, 0.1)
    x = oracle.solve(pl, 60)
    assert np.linalg.norm(x - s.x_star) / np.linalg.norm(s.x_star) < 1e-10
    s = synth.c2(grid=16)
    pl = oracle.plan_system(s, 0.1)
    x = oracle.solve(pl, 20000)
    assert np.linalg.norm(x - s.x_star) / np.linalg.norm(s.x_star) < 1e-10


def test_minimum_norm_limit_for_singular_consistent_system():
    """Theorem 1: from x0 = 0 the limit is the minimum-norm solution A^+ f."""
    rng = np.random.default_rng(11)
    n = 30
    B = sp.random(n, n, density=0.15, random_state=3).toarray() + np.diag(rng.uniform(1, 2, n))
    B[5] = B[3] + B[7]              # rank deficient, still consistent
    B[20] = 0.0                     # a zero row, left out of every group
    xs = rng.standard_normal(n)
    f = B @ xs
    s = synth.from_dense(B, f=f)
    pl = oracle.plan_system(s, 0.1)
    assert pl.group[np.nonzero(pl.p == 20)[0][0]] == -1
    x = oracle.solve(pl, 40000)
    want = np.linalg.pinv(B) @ f
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-7 * np.abs(want).max())


def test_error_non_increasing_each_sweep():
    """Every group step is non-expansive in the error when the group's unit rows
    have lambda_max < 2 (Gershgorin bound checked here); the error norm then
    never grows from sweep to sweep (eq. 3.8 for exact groups)."""
    s = synth.c1()
    pl = oracle.plan_system(s, 0.1)
    D = sp.csr_matrix((pl.v, pl.ci, pl.rp), shape=(s.n, s.n))
    B = sp.diags(1 / np.sqrt(pl.nu)) @ D
    for g in range(pl.ngroups):
        rows = np.nonzero(pl.group == g)[0]
        Bg = B[rows]
        G = abs(Bg @ Bg.T)
        assert G.sum(1).max() < 2.0
    xs_t = oracle.permute_vec(pl.p, s.x_star)
    x = np.zeros(s.n)
    e_prev = np.linalg.norm(x - xs_t)
    for _ in range(30):
        x = oracle.sweep(pl, x, 1)
        e = np.linalg.norm(x - xs_t)
        assert e <= e_prev * (1 + 1e-14)
        e_prev = e


# ---------------------------------------------- O9 residual, O11 refine
def test_relres_against_scipy():
    s = synth.c1(n=500)
    x = np.random.default_rng(4).standard_normal(s.n)
    r = s.f - s.scipy() @ x
    np.testing.assert_allclose(oracle.relres(s.n, s.row_ptr, s.col, s.val, s.f, x),
                               np.linalg.norm(r) / np.linalg.norm(s.f), rtol=1e-13)


# ------------------------------------------------- relaxation (omega)
def test_relaxed_step_on_the_identity():
    """With omega, each row step moves omega times the projection: on the
    identity (one group) one sweep from 0 gives x = omega f exactly (one
    rounding per entry), and omega = 1 is the unrelaxed step of eq. 1.2."""
    f = np.arange(1.0, 34.0) / 7.0
    s = synth.from_dense(np.eye(33), f=f)
    for om in (0.5, 1.3, 1.0):
        pl = oracle.plan_system(s, 0.1, omega=om)
        assert pl.ngroups == 1
        x = oracle.sweep(pl, np.zeros(33), 1)
        assert np.array_equal(x, om * pl.f)


def test_relaxed_single_group_step_is_relaxed_cimmino():
    """delta > 1 puts every row in one group: one sweep is the relaxed
    simultaneous step x + omega A^T D^-1 (f - A x), D = diag(||a_i||^2),
    formed here with dense numpy."""
    s = synth.c1(n=80)
    for om in (0.6, 1.7):
        pl = oracle.plan_system(s, 1.5, omega=om)
        assert pl.ngroups == 1
        A = sp.csr_matrix((pl.v, pl.ci, pl.rp), shape=(s.n, s.n)).toarray()
        x0 = np.random.default_rng(8).standard_normal(s.n)
        want = x0 + om * (A.T @ ((pl.f - A @ x0) / np.einsum("ij,ij->i", A, A)))
        got = oracle.sweep(pl, x0, 1)
        assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


def test_relaxed_orthonormal_group_scales_the_residual():
    """For one group of orthonormal rows the relaxed step leaves the residual
    (1 - omega) r: ||r_1|| = |1 - omega| ||r_0||."""
    rng = np.random.default_rng(12)
    Q, _ = np.linalg.qr(rng.standard_normal((24, 24)))
    s = synth.from_dense(Q, x_star=rng.standard_normal(24))
    for om in (0.25, 1.5):
        pl = oracle.plan_system(s, 1.5, omega=om)
        x1, inf = oracle.solve_tol(pl, 0.0, 1, 1)
        assert inf.relres == pytest.approx(abs(1.0 - om) * inf.relres0, rel=1e-10)


# ------------------------------------------------- O9: the stopping rule
def _two_row_case():
    """A = [[1, 1], [0, 1]], x* = (1, 1), f = (2, 1).  RCM reverses the two
    vertices, so A~ = [[1, 0], [1, 1]], f~ = (1, 2), x~* = (1, 1); the rows'
    cosine is 1/sqrt(2) >= 0.1, so each row is its own group, row (1, 0)
    first.  Worked by hand from x~ = 0: the first projection sets x~_0 = 1,
    the second moves x~ along (1, 1) onto x~_0 + x~_1 = 2, and after every
    sweep the error lies along (1, -1) with the residual of row 0 equal to
    -(x~_0 - 1) and that of row 1 zero.  Sweep 1 ends at (3/2, 1/2), sweep 2
    at (5/4, 3/4): each sweep halves the error (alternating projections onto
    two lines at 45 degrees, |cos|^2 = 1/2), so ||r_k|| = 2^-k exactly
    (dyadic values) and relres_k = 2^-k / sqrt(5)."""
    return synth.from_dense(np.array([[1.0, 1.0], [0.0, 1.0]]), f=np.array([2.0, 1.0]))


# ------------------------------------------- relaxation bound (one-row groups)
def _tri(sign):
    return sp.csr_matrix(np.array([[2.0, sign, 0.0], [sign, 2.0, sign], [0.0, sign, 2.0]]))


@pytest.mark.parametrize("sign", [-1.0, 1.0])
def test_lambda_bound_hand_worked_tridiagonal(sign):
    """tridiag(s, 2, s): |a_1|^2 = |a_3|^2 = 5, |a_2|^2 = 6, |cos(a_1, a_2)| =
    |cos(a_2, a_3)| = 4 / sqrt(30) ~ 0.730, |cos(a_1, a_3)| = 1 / 5, whatever
    the sign s.  delta = 0.75: one group, bound 1 + 8 / sqrt(30) (row 2);
    delta = 0.5: groups {1, 3} and {2}, bounds 1.2 and 1."""
    s = synth.from_scipy(_tri(sign))
    b, per = oracle.lambda_bound(oracle.plan_system(s, 0.75))
    assert per.size == 1 and b == pytest.approx(1.0 + 8.0 / np.sqrt(30.0), rel=1e-14)
    b, per = oracle.lambda_bound(oracle.plan_system(s, 0.5))
    assert np.sort(per) == pytest.approx([1.0, 1.2], rel=1e-14) and b == pytest.approx(1.2, rel=1e-14)


def test_lambda_bound_of_orthogonal_rows_is_one():
    """Rows with disjoint supports (and a zero row): every Gram matrix is the
    identity, so every bound is exactly 1."""
    M = np.diag([3.0, -2.0, 0.0, 5.0, 1.5])[[4, 0, 3, 2, 1]]
    pl = oracle.plan_system(synth.from_dense(M), 0.1)
    b, per = oracle.lambda_bound(pl)
    assert pl.ngroups == 1 and b == 1.0 and np.array_equal(per, [1.0])


def test_lambda_bound_hand_worked_complex():
    """a_1 = (1, i, 0), a_2 = (i, 2, 0), a_3 = (0, 1, 1); squared norms 2, 5, 2.
    |a_1^H a_2| = |i - 2i| = 1, |a_1^H a_3| = |-i| = 1, |a_2^H a_3| = 2, so the
    cosines are 1/sqrt(10), 1/2 and 2/sqrt(10) (the plain bilinear products
    would give 3, 1 and 2).  delta = 0.7: one group; the row sums are
    1 + 1/sqrt(10) + 1/2, 1 + 3/sqrt(10) and 1 + 1/2 + 2/sqrt(10), the last
    the largest."""
    M = np.array([[1.0, 1j, 0.0], [1j, 2.0, 0.0], [0.0, 1.0, 1.0]])
    A = sp.csr_matrix(M)
    n = 3
    pl = oracle.plan_complex(n, A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data,
                             M @ np.ones(n), 0.7, use_rcm=False)
    b, per = oracle.lambda_bound(pl)
    assert pl.ngroups == 1 and b == pytest.approx(1.5 + 2.0 / np.sqrt(10.0), rel=1e-14)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_lambda_bound_bounds_the_largest_eigenvalue(seed):
    """Gershgorin: per group, lambda_max of the dense B_g B_g^T lies in
    [1, bound] (the diagonal is 1, the bound is the largest absolute row sum)."""
    s = synth.random_rows(120, 4, seed)
    pl = oracle.plan_system(s, 0.3)
    b, per = oracle.lambda_bound(pl)
    A = sp.csr_matrix((pl.v, pl.ci, pl.rp), shape=(pl.n, pl.n)).toarray()
    for g in range(pl.ngroups):
        rows = np.flatnonzero(pl.group == g)
        B = A[rows] / np.sqrt(pl.nu[rows])[:, None]
        lam = np.linalg.eigvalsh(B @ B.T).max()
        assert 1.0 - 1e-12 <= lam <= per[g] * (1 + 1e-12)
    assert b == per.max() and b < 1.0 + 0.3 * 12


def test_stop_rule_two_row_hand_case():
    """Section 3.5's stopping rule read as relres <= tol: 2^-k / sqrt(5) <= 1e-10
    first at k = 33 (2^-32 / sqrt(5) = 1.04e-10); checked every 5 sweeps it
    stops at 35; with maxit = 20 it stops there, unconverged; tol <= 0 runs
    exactly maxit sweeps."""
    pl = oracle.plan_system(_two_row_case(), 0.1)
    assert pl.p.tolist() == [1, 0] and pl.group.tolist() == [0, 1]
    for every, k in ((1, 33), (5, 35)):
        x, inf = oracle.solve_tol(pl, 1e-10, 100, every)
        assert (inf.status, inf.sweeps, inf.checks) == ("converged", k, k // every)
        assert inf.relres0 == 1.0
        assert inf.relres == pytest.approx(2.0 ** -k / np.sqrt(5.0), rel=1e-14)
        assert np.array_equal(x, np.array([1.0 + 2.0 ** -k, 1.0 - 2.0 ** -k]))
    x, inf = oracle.solve_tol(pl, 1e-10, 20, 1)
    assert (inf.status, inf.sweeps) == ("maxit", 20)
    assert inf.relres == pytest.approx(2.0 ** -20 / np.sqrt(5.0), rel=1e-14)
    x, inf = oracle.solve_tol(pl, 0.0, 7, 3)
    assert (inf.status, inf.sweeps, inf.checks) == ("maxit", 7, 0)
    assert inf.relres == pytest.approx(2.0 ** -7 / np.sqrt(5.0), rel=1e-14)


def test_stop_rule_divergence_and_nonfinite_hand_case():
    """Three identical rows (1, 1, 1), f = (3, 3, 3), delta = 2: no pair
    reaches |cos| = 1 >= 2, so one group projects all three rows from the
    same iterate.  With s = sum x, each w_i = (3 - s) / 3 and x_c grows by
    3 w, so s becomes 9 - 2 s: s = 0, 9, -9, 27, ... and every residual entry
    is 3 (-2)^k, relres_k = 2^k.  The rule declares divergence at the first
    check with relres > 1e3: sweep 10 (1024) when checked every sweep, sweep 12
    (4096) when checked every 4.  Checked only after 1100 sweeps, the values
    have overflowed (3 * 2^1100 > DBL_MAX): NONFINITE.  A NaN start is
    NONFINITE before any sweep."""
    s = synth.from_dense(np.ones((3, 3)), f=np.full(3, 3.0))
    pl = oracle.plan_system(s, 2.0)
    assert pl.ngroups == 1
    for every, k in ((1, 10), (4, 12)):
        _, inf = oracle.solve_tol(pl, 1e-10, 100, every)
        assert (inf.status, inf.sweeps, inf.relres) == ("diverged", k, 2.0 ** k)
    _, inf = oracle.solve_tol(pl, 1e-10, 2000, 1100)
    assert (inf.status, inf.sweeps, inf.checks) == ("nonfinite", 1100, 1)
    x0 = np.array([0.0, np.nan, 0.0])
    _, inf = oracle.solve_tol(pl, 1e-10, 50, 1, x0t=x0)
    assert (inf.status, inf.sweeps) == ("nonfinite", 0)


def test_stop_rule_residual_against_scipy():
    """The relative residual the rule reports equals ||f - A x|| / ||f|| formed
    by scipy in original coordinates from the returned iterate, and the
    iterate of a tol <= 0 run is the plain K-sweep iterate."""
    s = synth.c1(n=800, companion=True)
    pl = oracle.plan_system(s, 0.1)
    xt, inf = oracle.solve_tol(pl, 1e-6, 500, 3)
    assert inf.status == "converged" and inf.sweeps % 3 == 0
    x = oracle.unpermute(pl.p, xt)
    ref = np.linalg.norm(s.f - s.scipy() @ x) / np.linalg.norm(s.f)
    assert inf.relres == pytest.approx(ref, rel=1e-12)
    assert ref <= 1e-6
    _, prev = oracle.solve_tol(pl, 0.0, inf.sweeps - 3, 1)
    assert prev.relres > 1e-6          # not converged at the previous check
    xk, _ = oracle.solve_tol(pl, 0.0, 17, 1)
    assert np.array_equal(xk, oracle.sweep(pl, np.zeros(s.n), 17))


def test_refinement_reaches_tolerance():
    """Iterative refinement around the sweep reaches relative residual 1e-10."""
    s = synth.c1(companion=True)
    pl = oracle.plan_system(s, 0.1)
    xt, steps, rho = oracle.refine(pl, inner=8, outer=50, tol=1e-10)
    assert rho <= 1e-10
    assert steps >= 2
    x = oracle.unpermute(pl.p, xt)
    assert np.linalg.norm(x - s.x_star) / np.linalg.norm(s.x_star) < 1e-9


# ---------------------------------------------------------- O1 validate
def test_validate_rejects_bad_input():
    rp = np.array([0, 2, 3], np.int64)
    assert oracle.validate(2, rp, np.array([0, 1, 1], np.int32), np.ones(3)) == 0
    assert oracle.validate(2, rp, np.array([0, 0, 1], np.int32), np.ones(3)) == -2       # duplicate
    assert oracle.validate(2, rp, np.array([0, 2, 1], np.int32), np.ones(3)) == -2       # out of range
    assert oracle.validate(2, rp, np.array([0, 1, 1], np.int32), np.array([1, np.nan, 1])) == -4
    assert oracle.validate(2, rp, np.array([0, 1, 1], np.int32), np.ones(3), np.array([1, np.inf])) == -4
    assert oracle.validate(2, np.array([0, 3, 2], np.int64), np.array([0, 1, 1], np.int32), np.ones(3)) == -2


# ------------------------------------------------------------------ Section 4
def test_pad_square_matches_dense_extension():
    """Eqs. 4.1 and 4.3: [A, O] for m > n and [A; O] with f^ = [f; 0] for m < n,
    checked against dense numpy blocks."""
    import scipy.sparse as sp
    for m, n in ((30, 20), (20, 30), (25, 25)):
        s = synth.rect(m, n, 0.2, index=m)
        A = s.scipy().toarray()
        N, rp, ci, v, f = oracle.pad_square(m, n, s.row_ptr, s.col, s.val, s.f)
        Ah = sp.csr_matrix((v, ci, rp), shape=(N, N)).toarray()
        if m > n:
            want, fw = np.hstack([A, np.zeros((m, m - n))]), s.f
        elif m < n:
            want, fw = np.vstack([A, np.zeros((n - m, n))]), np.concatenate([s.f, np.zeros(n - m)])
        else:
            want, fw = A, s.f
        assert N == max(m, n)
        assert np.array_equal(Ah, want) and np.array_equal(f, fw)


def test_sobk_recovers_solution_and_leaves_extension_unknowns():
    """Algorithm 5 on a consistent overdetermined system with full column rank
    (the 200 x 150, density 0.2 size of Table 6): x^(1:n) -> x*, and the
    extension unknowns x^(n+1:m), whose columns are zero, never move."""
    s = synth.rect(200, 150, 0.2)
    assert np.linalg.matrix_rank(s.scipy().toarray()) == 150
    pl = oracle.plan_rect(s.m, s.n, s.row_ptr, s.col, s.val, s.f, 0.1)
    xh = oracle.solve(pl, 400, np.zeros(pl.n))
    assert np.array_equal(xh[s.n:], np.zeros(s.m - s.n))
    x = oracle.solve_rect(pl, s.n, 400)
    assert np.array_equal(x, xh[:s.n])
    assert np.linalg.norm(x - s.x_star) / np.linalg.norm(s.x_star) <= 1e-8


def test_uobk_converges_to_minimum_norm_solution():
    """Algorithm 6 on a consistent underdetermined system (the 500 x 2000,
    density 0.002 size of Table 8): from x0 = 0 the iterate stays in the row
    space, so it converges to the minimum-norm solution pinv(A) f (Theorem 1),
    not to the generating x*."""
    s = synth.rect(500, 2000, 0.002)
    A = s.scipy().toarray()
    x_mn = np.linalg.pinv(A) @ s.f
    pl = oracle.plan_rect(s.m, s.n, s.row_ptr, s.col, s.val, s.f, 0.1)
    x = oracle.solve_rect(pl, s.n, 2000)
    assert np.linalg.norm(x - x_mn) / np.linalg.norm(x_mn) <= 1e-10
    assert np.linalg.norm(x - s.x_star) / np.linalg.norm(s.x_star) > 0.1


def test_extension_rows_are_zero_rows():
    """The n - m appended rows of [A; O] have no entries: they join no group
    (zero rows, Q15) and their right-hand side is 0, so the system stays
    consistent."""
    s = synth.rect(300, 700, 0.01)
    pl = oracle.plan_rect(s.m, s.n, s.row_ptr, s.col, s.val, s.f, 0.1)
    new_of_old = np.empty(pl.n, dtype=np.int64)
    new_of_old[pl.p] = np.arange(pl.n)
    ext = new_of_old[s.m:]                          # reordered positions of appended rows
    assert np.all(pl.group[ext] == -1)
    assert np.all(pl.f[ext] == 0.0)
    lens = np.diff(s.row_ptr)
    real = new_of_old[:s.m][lens > 0]
    assert np.all(pl.group[real] >= 0)


# ------------------------------------------- block mode (Section 3.3, Algorithm 4)
def test_block_ranges_floor_rule():
    """The first k - 1 blocks take floor(m / k) rows, the k-th the rest."""
    assert oracle.block_ranges(10, 3).tolist() == [0, 3, 6, 10]
    assert oracle.block_ranges(12, 4).tolist() == [0, 3, 6, 9, 12]
    assert oracle.block_ranges(7, 1).tolist() == [0, 7]
    assert oracle.block_ranges(5, 5).tolist() == [0, 1, 2, 3, 4, 5]


def test_block_projection_lands_on_block_hyperplanes():
    """Eq. 1.3: after x + pinv(A_tau)(f_tau - A_tau x) on a consistent system,
    A_tau x = f_tau."""
    s = synth.c1(n=300, companion=True)
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, 5, 0.1)
    A = sp.csr_matrix((bp.v, bp.ci, bp.rp), shape=(s.n, s.n))
    x = np.random.default_rng(1).standard_normal(s.n)
    for tau in range(5):
        y = oracle.block_project(bp, tau, x)
        r0, r1 = bp.bptr[tau], bp.bptr[tau + 1]
        assert np.linalg.norm(A[r0:r1] @ y - bp.f[r0:r1]) <= 1e-10 * np.linalg.norm(bp.f[r0:r1])


def test_one_row_blocks_are_sequential_kaczmarz():
    """k = m: every block is one row, so a block sweep is eq. 1.2 row by row in
    the order the pairs and Nclass give."""
    s = synth.c1(n=60)
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, s.n, 0.1)
    order = [t for pr in bp.pairs for t in pr] + list(bp.nclass)
    assert sorted(order) == list(range(s.n))
    x0 = np.random.default_rng(2).standard_normal(s.n)
    xb = oracle.block_sweep(bp, x0, 2)
    nu, inv = oracle.norms(s.n, bp.rp, bp.v)
    xr = oracle.rowwise(s.n, bp.rp, bp.ci, bp.v, bp.f, inv, np.array(order * 2, dtype=np.int32), x0)
    assert np.linalg.norm(xb - xr) <= 1e-12 * np.linalg.norm(xr)


def test_block_pair_rule_hand_cases():
    """Blocks with disjoint column supports have centroid cosine 0 and pair up
    in order; blocks of identical dense rows have cosine 1 and all go to
    Nclass."""
    n = 12
    D = np.zeros((n, n))
    for i in range(n):
        D[i, i] = 2.0
        D[i, (i + 1) % 3 + 3 * (i // 3)] += 0.5     # stays inside each block of 3 rows and 3 columns
    s = synth.from_dense(D, np.ones(n))
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, 4, 0.1)
    # the RCM order keeps the four 3x3 blocks contiguous, so the chunks are them
    assert np.allclose(bp.cos - np.eye(4), 0.0)
    assert bp.pairs == [(0, 1), (2, 3)] and bp.nclass == []
    E = np.ones((8, 8)) + 7 * np.eye(8)
    se = synth.from_dense(E, np.ones(8))
    be = oracle.block_plan(se.n, se.row_ptr, se.col, se.val, se.f, 4, 0.1)
    assert be.pairs == [] and be.nclass == [0, 1, 2, 3]


def _tridiag_blocks(n=40, k=5):
    T = sp.diags([np.full(n - 1, -1.0), np.full(n, 4.0), np.full(n - 1, -1.0)], [-1, 0, 1]).tocsr()
    return synth.from_scipy(T, np.linspace(-1.0, 1.0, n)), k


def test_block_centroid_cosines_hand_worked():
    """Centroid cosines of Section 3.3 (Algorithm 4, step 3) on tridiag(-1, 4, -1)
    with n = 40 cut into k = 5 blocks of s = 8 rows.  RCM reverses the path,
    which leaves this matrix unchanged.  The row sum of an inner block is -1
    at the column before the block, 3 at its first and last columns, 2 at the
    s - 2 columns between and -1 at the column after: squared norm
    1 + 9 + 4 (s - 2) + 9 + 1 = 4 s + 12 = 44; the first and last blocks lack
    one outer -1: 4 s + 11 = 43.  Neighbouring sums overlap at two columns
    with products 3 (-1) each: G = -6 (-6 / s^2 for the mean rows; the scale
    cancels).  Blocks two apart share no column.  Hence |cos| = 6 / sqrt(43 * 44)
    for the pairs (0, 1) and (3, 4), 6 / 44 = 3 / 22 for (1, 2) and (2, 3),
    0 beyond, 1 on the diagonal."""
    s, k = _tridiag_blocks()
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, 0.1)
    want = np.eye(k)
    edge, inner = 6.0 / np.sqrt(43.0 * 44.0), 3.0 / 22.0
    for a, b, c in ((0, 1, edge), (1, 2, inner), (2, 3, inner), (3, 4, edge)):
        want[a, b] = want[b, a] = c
    assert np.abs(bp.cos - want).max() <= 1e-15
    # pair rule on these values: at thr = 0.1 the neighbours (|cos| ~ 0.14)
    # conflict, so 0 pairs with 2 and 1 with 3; at thr = 0.2 neighbours pair
    assert bp.pairs == [(0, 2), (1, 3)] and bp.nclass == [4]
    bp2 = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, 0.2)
    assert bp2.pairs == [(0, 1), (2, 3)] and bp2.nclass == [4]


def test_block_sweep_order_is_pairs_then_nclass():
    """Algorithm 4's order: each pair's tau1 then tau2 (in the order the pairs
    were formed), then the Nclass blocks.  The blocks of the thr = 0.2 plan
    overlap their neighbours, so the projections do not commute and the order
    shows; the expected iterate is formed with dense numpy pseudo-inverses
    in that order."""
    s, k = _tridiag_blocks()
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, k, 0.2)
    A = sp.csr_matrix((bp.v, bp.ci, bp.rp), shape=(s.n, s.n)).toarray()
    x = np.random.default_rng(9).standard_normal(s.n)
    want = x.copy()
    for t in (0, 1, 2, 3, 4):
        r0, r1 = bp.bptr[t], bp.bptr[t + 1]
        want = want + np.linalg.pinv(A[r0:r1]) @ (bp.f[r0:r1] - A[r0:r1] @ want)
    got = oracle.block_sweep(bp, x, 1)
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)
    other = x.copy()
    for t in (4, 1, 0, 3, 2):                        # a different order lands elsewhere
        r0, r1 = bp.bptr[t], bp.bptr[t + 1]
        other = other + np.linalg.pinv(A[r0:r1]) @ (bp.f[r0:r1] - A[r0:r1] @ other)
    assert np.linalg.norm(other - want) > 1e-6 * np.linalg.norm(want)


def test_orthogonal_pair_equals_joint_projection():
    """For two blocks whose rows are mutually orthogonal, the two half steps of
    Algorithm 4 equal one projection onto both blocks (eq. 1.3 with the
    stacked block)."""
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    A = Q[:20]                                       # 20 orthonormal rows
    f = A @ rng.standard_normal(40)
    x = rng.standard_normal(40)
    A1, A2, f1, f2 = A[:10], A[10:], f[:10], f[10:]
    y = x + np.linalg.pinv(A1) @ (f1 - A1 @ x)
    y = y + np.linalg.pinv(A2) @ (f2 - A2 @ y)
    z = x + np.linalg.pinv(A) @ (f - A @ x)
    assert np.linalg.norm(y - z) <= 1e-12 * np.linalg.norm(z)


def test_block_mode_converges_to_generating_solution():
    """Theorem 1 for the block iteration: a consistent, well-conditioned system."""
    s = synth.c1(n=400, companion=True)
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, 8, 0.1)
    x = oracle.block_solve(bp, 60)
    assert np.linalg.norm(x - s.x_star) / np.linalg.norm(s.x_star) <= 1e-10


# ------------------------------------------ block-count criteria (Section 3.6)
def test_zn_nn_of_disjoint_blocks():
    """Definitions 1-2 on the block-diagonal hand case: C = I_4 gives
    n1 = 12 zero entries of 16 (zn = 0.75) and four nonzero entries of
    mean 1 (nn = 4 / 16)."""
    n = 12
    D = np.zeros((n, n))
    for i in range(n):
        D[i, i] = 2.0
        D[i, (i + 1) % 3 + 3 * (i // 3)] += 0.5
    s = synth.from_dense(D, np.ones(n))
    bp = oracle.block_plan(s.n, s.row_ptr, s.col, s.val, s.f, 4, 0.1)
    zn, nn = oracle.block_zn_nn(bp.cos)
    assert zn == pytest.approx(0.75, abs=1e-15)
    assert nn == pytest.approx(0.25, abs=1e-12)


def test_zn_nn_of_a_dense_matrix_and_of_a_band():
    """A dense matrix of equal positive rows has no zero cosine (zn = 0) and
    every cosine 1 (nn = 1).  A tridiagonal matrix cut into k blocks has
    nonzero cosines only between a block and itself or a neighbour:
    n2 = 3k - 2, so zn = 1 - (3k - 2) / k^2."""
    E = np.ones((8, 8))
    se = synth.from_dense(E, np.ones(8))
    zn, nn = oracle.block_zn_nn(oracle.block_plan(se.n, se.row_ptr, se.col, se.val, se.f, 4, 0.1).cos)
    assert zn == 0.0 and nn == pytest.approx(1.0, abs=1e-12)
    n = 60
    T = sp.diags([np.full(n - 1, -1.0), np.full(n, 4.0), np.full(n - 1, -1.0)], [-1, 0, 1]).tocsr()
    st = synth.from_scipy(T, np.ones(n))
    for k in (3, 5, 6, 10):
        bp = oracle.block_plan(st.n, st.row_ptr, st.col, st.val, st.f, k, 0.1)
        zn, nn = oracle.block_zn_nn(bp.cos)
        assert zn == pytest.approx(1.0 - (3 * k - 2) / k ** 2, abs=1e-15), k
        off = np.array([bp.cos[b, b + 1] for b in range(k - 1)])
        assert np.all(off > 0) and nn == pytest.approx((np.trace(bp.cos) + 2 * off.sum()) / k ** 2, abs=1e-15)


def test_block_k_selection_rule():
    """Largest zn first, then least nn, then least k; one candidate that is
    best on both criteria is always chosen (the muu example of Section 3.6)."""
    assert oracle.select_block_k([(2, 0.5, 0.10), (3, 0.4, 0.05), (4, 0.5, 0.20)]) == 2
    assert oracle.select_block_k([(2, 0.5, 0.30), (3, 0.5, 0.20), (4, 0.5, 0.20)]) == 3
    assert oracle.select_block_k([(5, 0.1, 0.9), (2, 0.7, 0.1), (9, 0.6, 0.05)]) == 2
    with pytest.raises(ValueError):
        oracle.select_block_k([])



# ------------------------------------------------ complex systems (kim1 case)
def _as_complex(s):
    return synth.ComplexSystem(s.n, s.row_ptr, s.col, s.val.astype(np.complex128), s.f.astype(np.complex128),
                               s.x_star.astype(np.complex128), s.name + "-as-complex", s.seed)


def test_complex_oracle_on_a_real_system_is_the_real_oracle():
    """Imaginary parts 0: every complex operation reduces exactly to its real
    counterpart, so the permutation, the groups and the iterate equal the
    (separately pinned) real oracle's bit for bit."""
    s = synth.c1(n=300)
    pr = oracle.plan_system(s, 0.1)
    pz = oracle.plan_system_complex(_as_complex(s), 0.1)
    assert np.array_equal(pr.p, pz.p) and np.array_equal(pr.group, pz.group) and pr.ngroups == pz.ngroups
    xr = oracle.solve(pr, 5)
    xz = oracle.solve_complex(pz, 5)
    assert np.array_equal(xz.real, xr) and not np.any(xz.imag)


def test_complex_cosine_is_the_hermitian_cosine():
    """|a_i^H a_j| / (||a_i|| ||a_j||), against numpy's conjugating dot."""
    s = synth.c1z(n=200)
    pz = oracle.plan_system_complex(s, 0.1)
    A = sp.csr_matrix((pz.vr + 1j * pz.vi, pz.ci, pz.rp), shape=(s.n, s.n)).toarray()
    rng = np.random.default_rng(3)
    checked = 0
    for _ in range(400):
        i, j = rng.integers(0, s.n, 2)
        if i == j or not np.any((A[i] != 0) & (A[j] != 0)):
            continue
        want = abs(np.vdot(A[i], A[j])) / (np.linalg.norm(A[i]) * np.linalg.norm(A[j]))
        assert oracle.cosine_complex(i, j, pz.rp, pz.ci, pz.vr, pz.vi, pz.nu) == pytest.approx(want, rel=1e-13)
        checked += 1
    assert checked > 20
    assert np.allclose(pz.nu, np.sum(np.abs(A) ** 2, axis=1), rtol=1e-14)


def test_complex_orthogonal_group_step_is_the_pseudo_inverse_projection():
    """Rows of a unitary (DFT) matrix are mutually orthogonal: they form one
    group, and one sweep is x + pinv(A)(f - A x) over C (eq. 1.3)."""
    m = 16
    F = np.exp(-2j * np.pi * np.outer(np.arange(m), np.arange(m)) / m) / np.sqrt(m)
    A = F[:8] * np.array([1.0, 2.0, 0.5, 3.0, 1.5, 1.0, 0.25, 2.5])[:, None]
    A = np.vstack([A, np.zeros((m - 8, m))])       # square, with zero rows
    xs = np.random.default_rng(5).standard_normal(m) + 1j * np.random.default_rng(6).standard_normal(m)
    S = sp.csr_matrix(A)
    S.sort_indices()
    z = synth.ComplexSystem(m, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data.astype(np.complex128),
                            S @ xs, xs, "dft", -1)
    pz = oracle.plan_system_complex(z, 0.1, use_rcm=False)
    assert pz.ngroups == 1
    x0 = np.random.default_rng(7).standard_normal(m) + 0j
    x1 = oracle.solve_complex(pz, 1, x0)
    want = x0 + np.linalg.pinv(A) @ (z.f - A @ x0)
    assert np.linalg.norm(x1 - want) <= 1e-12 * np.linalg.norm(want)


def test_complex_projection_is_phase_invariant():
    """Scaling row i and f_i by e^{i theta} leaves the hyperplane, hence every
    projection, unchanged (a missing conjugate in the update breaks this)."""
    s = synth.c1z(n=200, companion=True)
    rng = np.random.default_rng(8)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, s.n))
    rows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    t = synth.ComplexSystem(s.n, s.row_ptr, s.col, s.val * ph[rows], s.f * ph, s.x_star, "phased", -1)
    pa = oracle.plan_system_complex(s, 0.1)
    pb = oracle.plan_system_complex(t, 0.1)
    assert np.array_equal(pa.group, pb.group)
    xa = oracle.solve_complex(pa, 4)
    xb = oracle.solve_complex(pb, 4)
    assert np.linalg.norm(xa - xb) <= 1e-12 * np.linalg.norm(xa)


def test_complex_sweep_converges_to_generating_solution():
    """Theorem 1 over C on a consistent, well-conditioned complex system."""
    s = synth.c1z(n=400, companion=True)
    pz = oracle.plan_system_complex(s, 0.1)
    x = oracle.solve_complex(pz, 80)
    assert np.linalg.norm(x - s.x_star) / np.linalg.norm(s.x_star) <= 1e-10
    assert oracle.relres_complex(s.n, s.row_ptr, s.col, s.val, s.f, x) <= 1e-10
