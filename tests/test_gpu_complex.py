"""GPU parity of complex systems (the paper's kim1 case) against the oracle's
complex path (through the C ABI).

Bar, as for real systems: the RCM permutation and the group of every row are
bit-exact (complex cosines in FP64 on both sides, summed in the same order);
the iterate after K sweeps is within 1e-10 relative (2-norm) of the oracle's.
Both sides use the same complex operations in the same order without FMA
contraction, so the iterates are expected to agree to the last bit; the
tolerance is the stated contract, the bitwise result is reported.
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
    return max(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300),
               np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


CASES = [
    ("c1z-2000", lambda: synth.c1z(), 0.1, 20),
    ("c1z-companion-2000", lambda: synth.c1z(companion=True), 0.1, 20),
    ("c2z-grid64", lambda: synth.c2z(grid=64), 0.1, 10),
    ("c2z-grid196-kim1-order", lambda: synth.c2z(grid=196), 0.1, 10),
    ("c1z-37-ragged", lambda: synth.c1z(n=37), 0.3, 5),
]


@pytest.mark.parametrize("name,maker,delta,sweeps", CASES, ids=[c[0] for c in CASES])
def test_complex_plan_and_sweeps_match_oracle(name, maker, delta, sweeps):
    s = maker()
    _say(f"[complex] {name}: n={s.n} nnz={s.nnz} delta={delta} sweeps={sweeps}")
    po = oracle.plan_system_complex(s, delta)
    x_o = oracle.solve_complex(po, sweeps)
    with obk.plan_system(s, delta) as P:
        assert P.cplx
        assert np.array_equal(P.perm(), po.p)
        g, ng = P.groups()
        assert ng == po.ngroups and np.array_equal(g, po.group)
        x, info = P.solve(maxit=sweeps)
    err = _rel(x, x_o)
    _say(f"[complex] {name}: {ng} groups, |x - x_oracle| / |x_oracle| = {err:.3e}, "
         f"bitwise {np.array_equal(x, x_o)}, relres {info.relres:.3e}")
    assert x.dtype == np.complex128 and info.sweeps == sweeps
    assert err <= TOL_X


def test_complex_plan_of_a_real_system_equals_the_real_plan():
    """Imaginary parts 0: the complex path gives the real path's groups and
    iterate bit for bit (every complex operation reduces exactly)."""
    s = synth.c1(n=3000)
    z = synth.ComplexSystem(s.n, s.row_ptr, s.col, s.val.astype(np.complex128), s.f.astype(np.complex128),
                            s.x_star.astype(np.complex128))
    with obk.plan_system(s, 0.1) as Pr, obk.plan_system(z, 0.1) as Pz:
        assert np.array_equal(Pr.groups()[0], Pz.groups()[0])
        xr, _ = Pr.solve(maxit=7)
        xz, _ = Pz.solve(maxit=7)
    assert np.array_equal(xz.real, xr) and not np.any(xz.imag)


def test_complex_solve_to_tolerance_and_from_x0():
    """Checked solve on the well-conditioned complex family: converges, and
    the sweep count and iterate match the oracle's; a start x0 is honoured."""
    s = synth.c1z(companion=True)
    po = oracle.plan_system_complex(s, 0.1)
    want = None
    xt = np.zeros(s.n, dtype=np.complex128)
    for sw in range(1, 200):
        xt = oracle.sweep_complex(po, xt, 1)
        x = np.empty_like(xt)
        x[po.p] = xt
        if oracle.relres_complex(s.n, s.row_ptr, s.col, s.val, s.f, x) <= 1e-10:
            want = sw
            break
    assert want is not None
    x0 = np.random.default_rng(11).standard_normal(s.n) + 1j * np.random.default_rng(12).standard_normal(s.n)
    with obk.plan_system(s, 0.1) as P:
        x, info = P.solve(maxit=500, tol=1e-10)
        x1, _ = P.solve(x0=x0, maxit=3)
    _say(f"[complex] tolerance solve: {info.sweeps} sweeps (oracle {want}), relres {info.relres:.3e}")
    assert info.status == "converged" and info.sweeps == want
    assert _rel(x, s.x_star) <= 1e-9
    assert _rel(x1, oracle.solve_complex(po, 3, x0)) <= TOL_X


def test_complex_device_inputs_sweep_device_and_profile():
    import torch
    s = synth.c2z(grid=96)
    po = oracle.plan_system_complex(s, 0.1)
    dev = [torch.from_numpy(a).cuda() for a in (s.row_ptr, s.col, s.val, s.f)]
    P = obk.plan_complex(*dev, 0.1)
    try:
        assert np.array_equal(P.perm(), po.p)
        x, _ = P.solve(maxit=4)
        assert x.is_cuda and x.dtype == torch.complex128
        assert _rel(x.cpu().numpy(), oracle.solve_complex(po, 4)) <= TOL_X
        xt = torch.zeros(s.n, dtype=torch.complex128, device="cuda")
        P.sweep_device(xt, 9)
        torch.cuda.synchronize()
        assert _rel(xt.cpu().numpy(), oracle.sweep_complex(po, np.zeros(s.n, dtype=np.complex128), 9)) <= TOL_X
        prof = P.sweep_profile(xt, 2)
        _say(f"[complex] profile {prof}")
        assert {k["name"] for k in prof} == {"k_phase_r_z", "k_phase_s_z"}
        with pytest.raises(obk.ObkError):
            obk.Batch([P])
        with pytest.raises(obk.ObkError):
            P.set_opts(precision=obk.FP32_IR)
    finally:
        P.free()


@pytest.mark.parametrize("m,n", [(120, 200), (260, 150)])
def test_complex_non_square_systems(m, n):
    """Section 4 over C: the complex plan of an m x n system is that of the
    extended square system ([A; O] with f^ = [f; 0], or [A, O]); x = x^(1:n)."""
    rng = np.random.default_rng(m + n)
    nnz = int(0.05 * m * n)
    pos = np.sort(rng.choice(m * n, size=nnz, replace=False))
    rows, cols = pos // n, pos % n
    vals = rng.standard_normal(nnz) + 1j * rng.standard_normal(nnz)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    xs = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    f = A @ xs
    N = max(m, n)
    rp_ext = np.concatenate([A.indptr, np.full(N - m, A.indptr[-1])]).astype(np.int64)
    f_ext = np.concatenate([f, np.zeros(N - m, dtype=np.complex128)])
    ext = synth.ComplexSystem(N, rp_ext, A.indices.astype(np.int32), A.data.astype(np.complex128), f_ext,
                              np.zeros(N, dtype=np.complex128))
    po = oracle.plan_system_complex(ext, 0.1)
    x_o = oracle.solve_complex(po, 6)[:n]
    P = obk.plan_complex(A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, f, 0.1, n=m, n_cols=n)
    try:
        assert np.array_equal(P.perm(), po.p)
        assert np.array_equal(P.groups()[0], po.group)
        x, _ = P.solve(maxit=6)
    finally:
        P.free()
    _say(f"[complex] {m}x{n}: err {_rel(x, x_o):.3e}, bitwise {np.array_equal(x, x_o)}")
    assert x.shape == (n,) and _rel(x, x_o) <= TOL_X
