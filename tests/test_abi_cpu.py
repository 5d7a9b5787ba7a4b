"""CPU checks of libobk: it loads, exports every declared entry point, rejects
bad arguments before touching a GPU, and its host plan stages (RCM order,
first-fit grouping) are bit-exact with the oracle's independent code."""
import os
import re

import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth
import paper_2401_00672_amd as obk
from conftest import ROOT, parse_golden

HEADER = os.path.join(ROOT, "include", "obk.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"OBK_API[^;(]*?\b(obk_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 12
    L = obk.lib()
    for name in names:
        assert hasattr(L, name), name


def test_opts_default_and_free_null():
    L = obk.lib()
    o = obk._Opts()
    assert L.obk_opts_default(o) == 0
    assert (o.use_rcm, o.precision, o.inner_sweeps, o.check_every, o.reject_inconsistent, o.hbm_budget) == \
        (1, 0, 8, 1, 0, 0)
    assert (o.block_k, o.block_wgs, o.block_maxit, o.block_tol) == (0, 0, 0, 1e-14)
    assert (o.sweep_kernel, o.omega, o.max_group, o.deterministic) == (0, 1.0, 0, 1)
    assert (o.alloc, o.dealloc, o.ctx) == (None, None, None)
    L.obk_free(None)
    assert L.obk_opts_default(None) == -1


@pytest.mark.parametrize("kw,code", [
    (dict(n_cols=-1), -1),              # negative size
    (dict(delta=0.0), -1),              # delta must be > 0
    (dict(delta=float("nan")), -1),
    (dict(precision=7), -1),
    (dict(check_every=0), -1),
    (dict(block_k=-1), -1),             # block form: k in [1, 4096], at most the rows
    (dict(block_k=4097), -1),
    (dict(block_k=7), -1),              # 6 rows
    (dict(block_k=2, precision=1), -1), # block form is FP64 only
    (dict(block_k=2, block_tol=-1.0), -1),
    (dict(block_k=2, block_maxit=-3), -1),
    (dict(omega=0.0), -1),              # relaxation in (0, 2)
    (dict(omega=2.0), -1),
    (dict(omega=float("nan")), -1),
    (dict(block_k=2, omega=0.5), -1),   # the block form takes no relaxation
    (dict(max_group=3), -1),            # 0 (first fit) or 2 (the paper's pairs)
    (dict(max_group=2, block_k=2), -1),
    (dict(sweep_kernel="banded", block_k=2), -1),
])
def test_plan_rejects_bad_arguments_before_any_gpu_work(kw, code):
    s = synth.c1(n=6)
    delta = kw.pop("delta", 0.1)
    with pytest.raises(obk.ObkError) as ei:
        obk.plan(s.row_ptr, s.col, s.val, s.f, delta, **kw)
    assert ei.value.code == code
    assert obk.lib().obk_last_error().decode() != ""


@pytest.mark.parametrize("use_rcm", [-1, 4])
def test_plan_rejects_unknown_rcm_engine_before_any_gpu_work(use_rcm):
    s = synth.c1(n=6)
    csr = obk._Csr(s.n, s.n, s.nnz, s.row_ptr.ctypes.data, s.col.ctypes.data, s.val.ctypes.data, 0)
    o = obk._Opts()
    obk.lib().obk_opts_default(ctypes.byref(o))
    o.use_rcm = use_rcm
    h = ctypes.c_void_p()
    rc = obk.lib().obk_plan(ctypes.byref(csr), s.f.ctypes.data, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert "use_rcm" in obk.lib().obk_last_error().decode()
    with pytest.raises(ValueError):
        obk.plan(s.row_ptr, s.col, s.val, s.f, 0.1, rcm_engine="gpu")


@pytest.mark.parametrize("solver", [-1, 2])
def test_plan_rejects_unknown_block_solver_before_any_gpu_work(solver):
    s = synth.c1(n=6)
    csr = obk._Csr(s.n, s.n, s.nnz, s.row_ptr.ctypes.data, s.col.ctypes.data, s.val.ctypes.data, 0)
    o = obk._Opts()
    obk.lib().obk_opts_default(ctypes.byref(o))
    assert o.block_solver == 0
    o.block_k, o.block_solver = 2, solver
    h = ctypes.c_void_p()
    rc = obk.lib().obk_plan(ctypes.byref(csr), s.f.ctypes.data, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert "block_solver" in obk.lib().obk_last_error().decode()
    with pytest.raises(ValueError):
        obk.plan(s.row_ptr, s.col, s.val, s.f, 0.1, block_k=2, block_solver="lu")


def _graph(s):
    A = s.scipy()
    G = ((A + A.T) != 0).astype(np.int8).tolil()
    G.setdiag(0)
    G = sp.csr_matrix(G)
    G.eliminate_zeros()
    G.sort_indices()
    return G.indptr.astype(np.int64), G.indices.astype(np.int32)


@pytest.mark.parametrize("maker", [lambda: synth.c1(), lambda: synth.c2(grid=64), lambda: synth.c1(n=37),
                                   lambda: synth.c4_system(3, n=3000),
                                   lambda: synth.from_dense(np.eye(9))])
def test_host_rcm_bit_exact_with_oracle(maker):
    s = maker()
    gptr, gadj = _graph(s)
    assert np.array_equal(obk.rcm_host(gptr, gadj), oracle.rcm(s.n, s.row_ptr, s.col))


@pytest.mark.parametrize("case", parse_golden("rcm_hand.txt"), ids=lambda c: c["name"])
def test_host_rcm_hand_worked(case):
    n = int(case["n"])
    M = np.eye(n)
    for e in case["stored"].split():
        r, c = map(int, e.split("-"))
        M[r, c] = 1.0
    gptr, gadj = _graph(synth.from_dense(M))
    assert obk.rcm_host(gptr, gadj).tolist() == [int(t) for t in case["p"].split()]


def test_host_rcm_random_graphs():
    rng = np.random.default_rng(0)
    for trial in range(30):
        n = int(rng.integers(1, 80))
        M = sp.random(n, n, density=float(rng.uniform(0, 0.15)), random_state=trial, format="csr")
        M = M + sp.eye(n)
        s = synth.from_scipy(M)
        gptr, gadj = _graph(s)
        assert np.array_equal(obk.rcm_host(gptr, gadj), oracle.rcm(s.n, s.row_ptr, s.col))


@pytest.mark.parametrize("maker,delta", [(lambda: synth.c1(), 0.1), (lambda: synth.c2(grid=64), 0.1),
                                         (lambda: synth.c1(n=500), 0.02), (lambda: synth.c1(n=300), 0.5)])
def test_host_first_fit_bit_exact_with_oracle(maker, delta):
    s = maker()
    pl = oracle.plan_system(s, delta)
    rng = np.random.default_rng(5)
    # conflict lists in scrambled order: the grouping must not depend on it
    cidx = pl.cidx.copy()
    for i in range(s.n):
        seg = cidx[pl.cptr[i]:pl.cptr[i + 1]]
        rng.shuffle(seg)
    g, ng = obk.first_fit_host(pl.cptr, cidx, (pl.nu != 0).astype(np.uint8))
    assert ng == pl.ngroups
    assert np.array_equal(g, pl.group)


def test_host_stage_argument_errors():
    assert obk.lib().obk_rcm_host(-1, None, None, None) == -1
    assert obk.lib().obk_first_fit_host(3, None, None, None, None, None) == -1
    assert obk.rcm_host(np.zeros(1, np.int64), np.zeros(0, np.int32)).size == 0


def test_block_select_k_rejects_bad_candidates_before_any_gpu_work():
    s = synth.c1(n=6)
    for cands in ([], [0], [4097], [2, -1]):
        with pytest.raises(obk.ObkError) as ei:
            obk.select_block_k(s, 0.1, cands)
        assert ei.value.code == -1


@pytest.mark.parametrize("kw", [dict(precision=1), dict(block_k=2)])
def test_complex_plan_rejects_fp32_and_block_form_before_any_gpu_work(kw):
    s = synth.c1z(n=6)
    with pytest.raises(obk.ObkError) as ei:
        obk.plan_complex(s.row_ptr, s.col, s.val, s.f, 0.1, **kw)
    assert ei.value.code == -1


@pytest.mark.parametrize("cands,tol,maxit", [([], 1e-8, 10), ([0.1, 0.0], 1e-8, 10), ([0.1, float("nan")], 1e-8, 10),
                                             ([0.1], 0.0, 10), ([0.1], 1e-8, 0)])
def test_select_delta_rejects_bad_arguments_before_any_gpu_work(cands, tol, maxit):
    s = synth.c1(n=6)
    with pytest.raises(obk.ObkError) as ei:
        obk.select_delta(s, cands, tol=tol, maxit=maxit)
    assert ei.value.code == -1


def test_header_is_plain_c(tmp_path):
    """include/obk.h is a C ABI: it compiles as C99 with -pedantic next to
    <math.h> (no C++ or torch types leak into it)."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not installed")
    src = tmp_path / "use_obk.c"
    src.write_text('#include <math.h>\n#include "obk.h"\n'
                   'int main(void) { obk_opts o; obk_opts_default(&o); return o.block_k + (int)cos(0.0) - 1; }\n')
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I",
                        os.path.join(ROOT, "include"), "-c", str(src), "-o", str(tmp_path / "use_obk.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def _opts_plan_rc(**fields):
    """obk_plan on a 6-row host system with raw option fields; returns the
    status (the options are checked before any device work)."""
    s = synth.c1(n=6)
    csr = obk._Csr(s.n, s.n, s.nnz, s.row_ptr.ctypes.data, s.col.ctypes.data, s.val.ctypes.data, 0)
    o = obk._Opts()
    obk.lib().obk_opts_default(ctypes.byref(o))
    for k, v in fields.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    rc = obk.lib().obk_plan(ctypes.byref(csr), s.f.ctypes.data, 0.1, ctypes.byref(o), None, ctypes.byref(h))
    assert not h.value
    return rc


def test_plan_rejects_bad_option_fields_before_any_gpu_work():
    """deterministic takes 0 or 1; alloc and dealloc come together; a pair
    rule (max_group = 2) beyond 4096 rows is refused; sweep_kernel is 0..2."""
    keep = obk.ALLOC_FN(lambda n, ctx: None)
    assert _opts_plan_rc(deterministic=2) == -1
    assert "deterministic" in obk.lib().obk_last_error().decode()
    assert _opts_plan_rc(alloc=ctypes.cast(keep, ctypes.c_void_p)) == -1
    assert "alloc and dealloc" in obk.lib().obk_last_error().decode()
    assert _opts_plan_rc(sweep_kernel=3) == -1
    s = synth.c1(n=5000)
    with pytest.raises(obk.ObkError) as ei:
        obk.plan(s.row_ptr, s.col, s.val, s.f, 0.1, max_group=2)
    assert ei.value.code == -1 and "4096" in str(ei.value)


def test_binding_declares_argument_types_of_every_call():
    """Every library call of the binding that takes arguments has ctypes
    argument types declared (a float passed without them fails at call time,
    which only a device run would show)."""
    src = open(os.path.join(os.path.dirname(HEADER), "..", "paper_2401_00672_amd", "__init__.py")).read()
    called = set(re.findall(r"lib\(\)\.(obk_\w+)\((?!\))", src))
    declared = set(re.findall(r"L\.(obk_\w+)\.argtypes", src))
    assert called <= declared, sorted(called - declared)
