"""ctypes front end of the FP64 CPU oracle (``oracle/obk_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
CPU-baseline leg of ``bench.py``; never by the library.  It shares no code
with the HIP path.  Each function states the step of the paper it follows;
the C file carries the details of every step.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "obk_oracle.c")

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f64 = ctypes.c_double
_p = ctypes.c_void_p

_lib = None


def build(force: bool = True) -> str:
    from .build import build as _b
    return _b(force=force)


def lib():
    """The compiled oracle.  OBK_ORACLE_LIB names another build of the same
    source (the mutation tests load deliberately broken copies this way)."""
    global _lib
    if _lib is None:
        path = os.environ.get("OBK_ORACLE_LIB", LIB_PATH)
        if path == LIB_PATH and not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(path)
        L.orc_validate.restype = ctypes.c_int
        L.orc_validate.argtypes = [_i64, _p, _p, _p, _p]
        L.orc_rcm.restype = ctypes.c_int
        L.orc_rcm.argtypes = [_i64, _p, _p, _p]
        L.orc_permute.restype = ctypes.c_int
        L.orc_permute.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_norms.restype = None
        L.orc_norms.argtypes = [_i64, _p, _p, _p, _p]
        L.orc_cosine.restype = _f64
        L.orc_cosine.argtypes = [_i64, _i64, _p, _p, _p, _p]
        L.orc_conflicts.restype = _i64
        L.orc_conflicts.argtypes = [_i64, _p, _p, _p, _p, _f64, _p, _p]
        L.orc_groups.restype = _i32
        L.orc_groups.argtypes = [_i64, _p, _p, _p, _p]
        L.orc_pairs.restype = ctypes.c_int
        L.orc_pairs.argtypes = [_i64, _p, _p, _p, _p, _f64, _p]
        L.orc_sweep.restype = ctypes.c_int
        L.orc_sweep.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _i32, _f64, _p, _i64]
        L.orc_rowwise.restype = None
        L.orc_rowwise.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _i64, _p]
        L.orc_relres.restype = _f64
        L.orc_relres.argtypes = [_i64, _p, _p, _p, _p, _p, _p]
        L.orc_unpermute.restype = None
        L.orc_unpermute.argtypes = [_i64, _p, _p, _p]
        L.orc_permute_vec.restype = None
        L.orc_permute_vec.argtypes = [_i64, _p, _p, _p]
        L.orc_norms_z.restype = None
        L.orc_norms_z.argtypes = [_i64, _p, _p, _p, _p, _p]
        L.orc_cosine_z.restype = _f64
        L.orc_cosine_z.argtypes = [_i64, _i64, _p, _p, _p, _p, _p]
        L.orc_conflicts_z.restype = _i64
        L.orc_conflicts_z.argtypes = [_i64, _p, _p, _p, _p, _p, _f64, _p, _p]
        L.orc_sweep_z.restype = ctypes.c_int
        L.orc_sweep_z.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _p, _i32, _f64, _p, _p, _i64]
        L.orc_rowwise_z.restype = None
        L.orc_rowwise_z.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _p, _i64, _p, _p]
        L.orc_relres_z.restype = _f64
        L.orc_relres_z.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _p, _p]
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_max_threads.argtypes = []
        L.orc_mt_prepare.restype = _p
        L.orc_mt_prepare.argtypes = [_i64, _p, _p, _p, _p, _i32]
        L.orc_mt_sweep.restype = ctypes.c_int
        L.orc_mt_sweep.argtypes = [_p, _p, _p, _p, _p, _p, _f64, _p, _i64]
        L.orc_mt_free.restype = None
        L.orc_mt_free.argtypes = [_p]
        L.orc_solve_tol.restype = ctypes.c_int
        L.orc_solve_tol.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _i32, _f64, _p, _f64, _i64, _i64, _p, _p]
        L.orc_refine.restype = _i64
        L.orc_refine.argtypes = [_i64, _p, _p, _p, _p, _p, _p, _i32, _f64, _p, _i64, _i64, _f64, _p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def validate(n, rp, ci, v, f=None) -> int:
    """O1 (square CSR, columns in range, no duplicates, finite). 0 = valid."""
    rp, ci, v = _c(rp, np.int64), _c(ci, np.int32), _c(v, np.float64)
    f = None if f is None else _c(f, np.float64)
    return lib().orc_validate(n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(f))


def rcm(n, rp, ci) -> np.ndarray:
    """O2-O3: reverse Cuthill-McKee permutation p (new -> old), Section 3.2."""
    rp, ci = _c(rp, np.int64), _c(ci, np.int32)
    p = np.empty(n, dtype=np.int32)
    rc = lib().orc_rcm(n, _ptr(rp), _ptr(ci), _ptr(p))
    if rc != 0:
        raise RuntimeError(f"orc_rcm failed: {rc}")
    return p


def permute(n, rp, ci, v, f, p):
    """O4: A~ = P A P^T with sorted rows, f~ = P f (eqs. 3.1-3.2)."""
    rp, ci, v = _c(rp, np.int64), _c(ci, np.int32), _c(v, np.float64)
    f = _c(f, np.float64)
    p = _c(p, np.int32)
    nnz = int(rp[n])
    trp = np.empty(n + 1, np.int64)
    tci = np.empty(nnz, np.int32)
    tv = np.empty(nnz, np.float64)
    tf = np.empty(n, np.float64)
    rc = lib().orc_permute(n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(f), _ptr(p), _ptr(trp), _ptr(tci),
                           _ptr(tv), _ptr(tf))
    if rc != 0:
        raise RuntimeError(f"orc_permute failed: {rc}")
    return trp, tci, tv, tf


def norms(n, rp, v):
    """O5: nu_i = ||a_i||^2 (denominator of eq. 1.2), inv_i = 1/nu_i."""
    rp, v = _c(rp, np.int64), _c(v, np.float64)
    nu = np.empty(n, np.float64)
    inv = np.empty(n, np.float64)
    lib().orc_norms(n, _ptr(rp), _ptr(v), _ptr(nu), _ptr(inv))
    return nu, inv


def cosine(i, j, rp, ci, v, nu) -> float:
    """O6: |cos| of the angle between rows i and j (cosine table of Section 3.3)."""
    return lib().orc_cosine(int(i), int(j), _ptr(rp), _ptr(ci), _ptr(v), _ptr(nu))


def conflicts(n, rp, ci, v, nu, delta):
    """O6: for each row i the rows j < i with |cos_ij| >= delta (CSR form)."""
    rp, ci, v, nu = _c(rp, np.int64), _c(ci, np.int32), _c(v, np.float64), _c(nu, np.float64)
    cptr = np.empty(n + 1, np.int64)
    total = lib().orc_conflicts(n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(nu), float(delta), _ptr(cptr), None)
    if total < 0:
        raise RuntimeError(f"orc_conflicts failed: {total}")
    cidx = np.empty(max(total, 1), np.int32)
    total2 = lib().orc_conflicts(n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(nu), float(delta), _ptr(cptr),
                                 _ptr(cidx))
    assert total2 == total
    return cptr, cidx[:total]


def groups(n, nu, cptr, cidx):
    """O7: first-fit grouping (maximal Oclass/Nclass of Section 3.3)."""
    nu, cptr, cidx = _c(nu, np.float64), _c(cptr, np.int64), _c(cidx, np.int32)
    if cidx.size == 0:
        cidx = np.zeros(1, np.int32)
    g = np.empty(n, np.int32)
    ng = lib().orc_groups(n, _ptr(nu), _ptr(cptr), _ptr(cidx), _ptr(g))
    if ng < 0:
        raise RuntimeError(f"orc_groups failed: {ng}")
    return g, int(ng)


def pairs(n, rp, ci, v, nu, delta):
    """Literal pair rule of Section 3.3: partner of each row, -1 Nclass, -2 zero row."""
    rp, ci, v, nu = _c(rp, np.int64), _c(ci, np.int32), _c(v, np.float64), _c(nu, np.float64)
    out = np.empty(n, np.int32)
    lib().orc_pairs(n, _ptr(rp), _ptr(ci), _ptr(v), _ptr(nu), float(delta), _ptr(out))
    return out


@dataclasses.dataclass
class Plan:
    n: int
    p: np.ndarray          # new -> old
    rp: np.ndarray
    ci: np.ndarray
    v: np.ndarray
    f: np.ndarray          # permuted right-hand side
    nu: np.ndarray
    inv: np.ndarray
    cptr: np.ndarray
    cidx: np.ndarray
    group: np.ndarray      # group of each reordered row (-1: zero row)
    ngroups: int
    omega: float = 1.0     # relaxation of every row step (the paper's step: 1)


def plan(n, rp, ci, v, f, delta, *, use_rcm: bool = True, omega: float = 1.0) -> Plan:
    """Algorithm 4, first four steps, with one-row blocks: RCM, reorder,
    norms, cosine conflicts, grouping."""
    if validate(n, rp, ci, v, f) != 0:
        raise ValueError("invalid system")
    p = rcm(n, rp, ci) if use_rcm else np.arange(n, dtype=np.int32)
    trp, tci, tv, tf = permute(n, rp, ci, v, f, p)
    nu, inv = norms(n, trp, tv)
    cptr, cidx = conflicts(n, trp, tci, tv, nu, delta)
    g, ng = groups(n, nu, cptr, cidx)
    return Plan(n, p, trp, tci, tv, tf, nu, inv, cptr, cidx, g, ng, float(omega))


def plan_system(s, delta, **kw) -> Plan:
    return plan(s.n, s.row_ptr, s.col, s.val, s.f, delta, **kw)


def sweep(pl: Plan, xt: np.ndarray, sweeps: int, f: np.ndarray | None = None) -> np.ndarray:
    """O8: `sweeps` OBK sweeps in reordered coordinates; returns a new array."""
    x = np.array(xt, dtype=np.float64, copy=True)
    ff = pl.f if f is None else _c(f, np.float64)
    rc = lib().orc_sweep(pl.n, _ptr(pl.rp), _ptr(pl.ci), _ptr(pl.v), _ptr(ff), _ptr(pl.inv),
                         _ptr(pl.group), pl.ngroups, pl.omega, _ptr(x), int(sweeps))
    if rc != 0:
        raise RuntimeError(f"orc_sweep failed: {rc}")
    return x


def set_threads(t: int) -> None:
    """Threads of the oracle's row-parallel loops (conflicts, ThreadedSweep)."""
    lib().orc_set_threads(int(t))


def max_threads() -> int:
    return int(lib().orc_max_threads())


class ThreadedSweep:
    """O8 on several threads: phase (i) over the rows of a group, phase (ii)
    over its touched columns, each column's sum in ascending row order --
    the same operations as `sweep`, so the iterate is the same bit for bit
    (checked by the CPU tests).  Used for timing on all cores and for the
    full-size checks."""

    def __init__(self, pl: Plan):
        self.pl = pl
        self._h = lib().orc_mt_prepare(pl.n, _ptr(pl.rp), _ptr(pl.ci), _ptr(pl.v), _ptr(pl.group), pl.ngroups)
        if not self._h:
            raise MemoryError("orc_mt_prepare failed")

    def sweep(self, x: np.ndarray, sweeps: int, f: np.ndarray | None = None) -> np.ndarray:
        """`sweeps` sweeps in place on x (float64, contiguous); returns x."""
        assert x.dtype == np.float64 and x.flags.c_contiguous
        ff = self.pl.f if f is None else _c(f, np.float64)
        rc = lib().orc_mt_sweep(self._h, _ptr(self.pl.rp), _ptr(self.pl.ci), _ptr(self.pl.v), _ptr(ff),
                                _ptr(self.pl.inv), self.pl.omega, _ptr(x), int(sweeps))
        if rc != 0:
            raise RuntimeError(f"orc_mt_sweep failed: {rc}")
        return x

    def close(self) -> None:
        if self._h:
            lib().orc_mt_free(self._h)
            self._h = None

    def __del__(self):
        self.close()


def rowwise(n, rp, ci, v, f, inv, rows, x):
    """Sequential eq. (1.2) projections over `rows` in the given order."""
    x = np.array(x, dtype=np.float64, copy=True)
    rows = _c(rows, np.int32)
    lib().orc_rowwise(n, _ptr(_c(rp, np.int64)), _ptr(_c(ci, np.int32)), _ptr(_c(v, np.float64)),
                      _ptr(_c(f, np.float64)), _ptr(_c(inv, np.float64)), _ptr(rows), rows.size,
                      _ptr(x))
    return x


def relres(n, rp, ci, v, f, x, want_r: bool = False):
    """O9: ||f - A x|| / ||f||."""
    r = np.empty(n, np.float64) if want_r else None
    rho = lib().orc_relres(n, _ptr(_c(rp, np.int64)), _ptr(_c(ci, np.int32)), _ptr(_c(v, np.float64)),
                           _ptr(_c(f, np.float64)), _ptr(_c(x, np.float64)), _ptr(r))
    return (rho, r) if want_r else rho


def unpermute(p, xt):
    """O10: x = P^T x~."""
    xt = _c(xt, np.float64)
    x = np.empty_like(xt)
    lib().orc_unpermute(xt.size, _ptr(_c(p, np.int32)), _ptr(xt), _ptr(x))
    return x


def permute_vec(p, x):
    x = _c(x, np.float64)
    xt = np.empty_like(x)
    lib().orc_permute_vec(x.size, _ptr(_c(p, np.int32)), _ptr(x), _ptr(xt))
    return xt


def solve(pl: Plan, sweeps: int, x0: np.ndarray | None = None) -> np.ndarray:
    """Plan + `sweeps` sweeps from x0 (default 0, Section 3.5), original ordering."""
    xt = np.zeros(pl.n) if x0 is None else permute_vec(pl.p, x0)
    return unpermute(pl.p, sweep(pl, xt, sweeps))


def pad_square(m, n, rp, ci, v, f):
    """The extended square system of Section 4 for an m x n system.

    m > n (Algorithm 5): A^ = [A, O] with an m x (m - n) zero block, f^ = f;
    the unknowns become x^ = [x; x2] and x = x^(1:n).
    m < n (Algorithm 6): A^ = [A; O] with an (n - m) x n zero block,
    f^ = [f; 0]; x = x^.
    A zero block adds no entries: [A, O] is the same CSR read as m x m, and
    [A; O] appends n - m empty rows.  Returns (N, rp^, ci, v, f^), N = max(m, n)."""
    rp = _c(rp, np.int64)
    f = _c(f, np.float64)
    N = max(int(m), int(n))
    if m < N:
        rp = np.concatenate([rp, np.full(N - m, rp[-1], dtype=np.int64)])
        f = np.concatenate([f, np.zeros(N - m)])
    return N, rp, _c(ci, np.int32), _c(v, np.float64), f


def plan_rect(m, n, rp, ci, v, f, delta, **kw) -> Plan:
    """Plan of the extended square system (Algorithms 5 and 6, first step)."""
    N, rp2, ci2, v2, f2 = pad_square(m, n, rp, ci, v, f)
    return plan(N, rp2, ci2, v2, f2, delta, **kw)


def solve_rect(pl: Plan, n: int, sweeps: int, x0: np.ndarray | None = None) -> np.ndarray:
    """Sweeps on the extended system from x^0 = [x0; 0] (x0 default 0); returns
    x = x^(1:n) (Algorithm 5; for Algorithm 6 n = N and x = x^)."""
    x0h = np.zeros(pl.n)
    if x0 is not None:
        x0h[:n] = x0
    return solve(pl, sweeps, x0h)[:n]


SOLVE_STATUS = {0: "converged", 1: "maxit", 2: "diverged", 3: "nonfinite"}


@dataclasses.dataclass
class SolveInfo:
    sweeps: int
    checks: int
    relres0: float
    relres: float
    status: str


def solve_tol(pl: Plan, tol: float, maxit: int, check_every: int = 1,
              x0t: np.ndarray | None = None) -> tuple[np.ndarray, SolveInfo]:
    """O9: sweeps from x~0 (default 0, Section 3.5) until the relative residual
    is <= tol, checked every `check_every` sweeps, or `maxit` sweeps are done;
    DIVERGED when it exceeds 1e3 times its initial value, NONFINITE on NaN or
    Inf.  tol <= 0 runs exactly maxit sweeps.  Reordered coordinates."""
    x = np.zeros(pl.n) if x0t is None else np.array(x0t, dtype=np.float64, copy=True)
    out = np.zeros(2, np.int64)
    rho = np.zeros(2, np.float64)
    st = lib().orc_solve_tol(pl.n, _ptr(pl.rp), _ptr(pl.ci), _ptr(pl.v), _ptr(pl.f), _ptr(pl.inv),
                             _ptr(pl.group), pl.ngroups, pl.omega, _ptr(x), float(tol), int(maxit),
                             int(check_every), _ptr(out), _ptr(rho))
    if st < 0:
        raise RuntimeError(f"orc_solve_tol failed: {st}")
    return x, SolveInfo(int(out[0]), int(out[1]), float(rho[0]), float(rho[1]), SOLVE_STATUS[st])


def refine(pl: Plan, inner: int, outer: int, tol: float, x0t: np.ndarray | None = None):
    """O11 iterative refinement schedule in FP64; returns (x~, steps, relres)."""
    x = np.zeros(pl.n) if x0t is None else np.array(x0t, dtype=np.float64, copy=True)
    rho = ctypes.c_double(0.0)
    steps = lib().orc_refine(pl.n, _ptr(pl.rp), _ptr(pl.ci), _ptr(pl.v), _ptr(pl.f), _ptr(pl.inv),
                             _ptr(pl.group), pl.ngroups, pl.omega, _ptr(x), int(inner), int(outer), float(tol),
                             ctypes.byref(rho))
    return x, int(steps), float(rho.value)


# ------------------------------------------------- block mode (Algorithm 4)
@dataclasses.dataclass
class BlockPlan:
    """Paper-literal block form of Algorithm 4 (k uniform row blocks)."""
    n: int
    p: np.ndarray          # RCM permutation, new -> old
    rp: np.ndarray         # reordered CSR
    ci: np.ndarray
    v: np.ndarray
    f: np.ndarray
    bptr: np.ndarray       # block row ranges, k + 1
    cos: np.ndarray        # k x k table of |cos| between block centroids
    pairs: list            # Oclass: (tau1, tau2) in the order formed
    nclass: list           # Nclass: blocks left unpaired, ascending


def block_ranges(m: int, k: int) -> np.ndarray:
    """Uniform chunking in order (Section 3.3): the first k - 1 blocks take
    floor(m / k) rows each, the k-th block the rest."""
    if k < 1 or k > max(m, 1):
        raise ValueError("need 1 <= k <= m")
    size = m // k
    b = np.arange(k + 1, dtype=np.int64) * size
    b[k] = m
    return b


def block_plan(n, rp, ci, v, f, k, thr) -> BlockPlan:
    """Algorithm 4, steps 1-4 in block form: RCM, uniform chunking, the cosine
    table of the block centroids, and the pairing of Section 3.3 (each block
    not yet in a class takes the first later block not yet in a class whose
    centroid is near-orthogonal to its own, |cos| < thr; blocks left over form
    Nclass)."""
    if validate(n, rp, ci, v, f) != 0:
        raise ValueError("invalid system")
    p = rcm(n, rp, ci)
    trp, tci, tv, tf = permute(n, rp, ci, v, f, p)
    bptr = block_ranges(n, k)
    A = sp.csr_matrix((tv, tci, trp), shape=(n, n))
    cen = np.zeros((k, n))
    for b in range(k):
        # the centroid is the mean row of the block (its scale does not enter the cosine)
        cen[b] = np.asarray(A[bptr[b]:bptr[b + 1]].sum(axis=0)).ravel() / max(bptr[b + 1] - bptr[b], 1)
    nrm = np.sqrt(np.einsum("ij,ij->i", cen, cen))
    G = cen @ cen.T
    cos = np.zeros((k, k))
    for i in range(k):
        for j in range(k):
            if nrm[i] > 0 and nrm[j] > 0:
                cos[i, j] = abs(G[i, j]) / (nrm[i] * nrm[j])
    taken = [False] * k
    pairs = []
    for i in range(k):
        if taken[i]:
            continue
        for j in range(i + 1, k):
            if not taken[j] and cos[i, j] < thr:
                pairs.append((i, j))
                taken[i] = taken[j] = True
                break
    nclass = [i for i in range(k) if not taken[i]]
    return BlockPlan(n, p, trp, tci, tv, tf, bptr, cos, pairs, nclass)


def block_project(bp: BlockPlan, tau: int, x: np.ndarray) -> np.ndarray:
    """Eq. 1.3 / 3.3: x + pinv(A_tau) (f_tau - A_tau x), with the dense
    pseudo-inverse of the block."""
    r0, r1 = int(bp.bptr[tau]), int(bp.bptr[tau + 1])
    A = sp.csr_matrix((bp.v, bp.ci, bp.rp), shape=(bp.n, bp.n))[r0:r1].toarray()
    return x + np.linalg.pinv(A) @ (bp.f[r0:r1] - A @ x)


def block_sweep(bp: BlockPlan, xt: np.ndarray, sweeps: int) -> np.ndarray:
    """Sweeps of the block iteration in reordered coordinates: each Oclass
    pair projected in turn (tau1 then tau2, the two half steps of Algorithm 4),
    then every Nclass block, in the order formed (deterministic reading of the
    selection steps)."""
    x = np.array(xt, dtype=np.float64, copy=True)
    for _ in range(int(sweeps)):
        for t1, t2 in bp.pairs:
            x = block_project(bp, t1, x)
            x = block_project(bp, t2, x)
        for t in bp.nclass:
            x = block_project(bp, t, x)
    return x


def block_solve(bp: BlockPlan, sweeps: int, x0: np.ndarray | None = None) -> np.ndarray:
    """Block plan + sweeps from x0 (default 0), original ordering."""
    xt = np.zeros(bp.n) if x0 is None else permute_vec(bp.p, x0)
    return unpermute(bp.p, block_sweep(bp, xt, sweeps))


# ------------------------------------------ block-count criteria (Section 3.6)
def block_zn_nn(cos: np.ndarray) -> tuple[float, float]:
    """Definitions 1 and 2 on a k x k cosine table C: the orthogonality
    proportion zn = n1 / k^2 (n1 = entries of C exactly zero) and the
    non-orthogonality severity nn = n2 * nm / k^2 (n2 = nonzero entries, nm
    their mean), i.e. the sum of the nonzero entries over k^2."""
    C = np.asarray(cos, dtype=np.float64)
    k = C.shape[0]
    num = k * k
    nz = C[C != 0.0]
    n1 = num - nz.size
    nm = nz.mean() if nz.size else 0.0
    return n1 / num, nz.size * nm / num


def select_block_k(scores) -> int:
    """The block count that maximises zn and minimises nn (Section 3.6), read
    as: the largest zn, then among those the least nn, then the least k.
    scores: iterable of (k, zn, nn)."""
    best = None
    for k, zn, nn in scores:
        key = (-zn, nn, k)
        if best is None or key < best[0]:
            best = (key, k)
    if best is None:
        raise ValueError("no candidate block counts")
    return int(best[1])


def block_k_scores(n, rp, ci, v, f, thr, candidates):
    """(k, zn, nn) of the block plan for every candidate k."""
    out = []
    for k in candidates:
        bp = block_plan(n, rp, ci, v, f, int(k), thr)
        zn, nn = block_zn_nn(bp.cos)
        out.append((int(k), zn, nn))
    return out



# ----------------------------------------------------- complex systems (kim1)
@dataclasses.dataclass
class ComplexPlan:
    """Plan of a complex system: the real plan's steps with the complex norm and
    cosine (orc_*_z in the C file); values in separate real/imaginary arrays."""
    n: int
    p: np.ndarray
    rp: np.ndarray
    ci: np.ndarray
    vr: np.ndarray
    vi: np.ndarray
    fr: np.ndarray
    fi: np.ndarray
    nu: np.ndarray
    inv: np.ndarray
    group: np.ndarray
    ngroups: int
    omega: float = 1.0


def norms_complex(n, rp, vr, vi):
    nu = np.empty(n)
    inv = np.empty(n)
    lib().orc_norms_z(n, _ptr(_c(rp, np.int64)), _ptr(_c(vr, np.float64)), _ptr(_c(vi, np.float64)),
                      _ptr(nu), _ptr(inv))
    return nu, inv


def cosine_complex(i, j, rp, ci, vr, vi, nu) -> float:
    """|a_i^H a_j| / (||a_i|| ||a_j||) over the common columns."""
    return float(lib().orc_cosine_z(int(i), int(j), _ptr(rp), _ptr(ci), _ptr(vr), _ptr(vi), _ptr(nu)))


def plan_complex(n, rp, ci, vz, fz, delta, *, use_rcm: bool = True, omega: float = 1.0) -> ComplexPlan:
    """Algorithm 4, first four steps, over C: RCM on the pattern (as for real
    systems), the same symmetric permutation of the real and imaginary parts,
    complex norms and cosines, first-fit grouping."""
    vz = np.asarray(vz, dtype=np.complex128)
    fz = np.asarray(fz, dtype=np.complex128)
    vr, vi = _c(vz.real, np.float64), _c(vz.imag, np.float64)
    fr, fi = _c(fz.real, np.float64), _c(fz.imag, np.float64)
    if validate(n, rp, ci, vr, fr) != 0 or validate(n, rp, ci, vi, fi) != 0:
        raise ValueError("invalid system")
    p = rcm(n, rp, ci) if use_rcm else np.arange(n, dtype=np.int32)
    trp, tci, tvr, tfr = permute(n, rp, ci, vr, fr, p)
    _, _, tvi, tfi = permute(n, rp, ci, vi, fi, p)
    nu, inv = norms_complex(n, trp, tvr, tvi)
    cptr = np.zeros(n + 1, dtype=np.int64)
    total = lib().orc_conflicts_z(n, _ptr(trp), _ptr(tci), _ptr(tvr), _ptr(tvi), _ptr(nu), float(delta),
                                  _ptr(cptr), None)
    cidx = np.zeros(max(int(total), 1), dtype=np.int32)
    lib().orc_conflicts_z(n, _ptr(trp), _ptr(tci), _ptr(tvr), _ptr(tvi), _ptr(nu), float(delta), _ptr(cptr),
                          _ptr(cidx))
    group, ng = groups(n, nu, cptr, cidx[:total])
    return ComplexPlan(n, p, trp, tci, tvr, tvi, tfr, tfi, nu, inv, group, ng, float(omega))


def sweep_complex(pl: ComplexPlan, xt: np.ndarray, sweeps: int) -> np.ndarray:
    """O8 over C on a reordered complex iterate."""
    xr = np.array(np.real(xt), dtype=np.float64, copy=True)
    xi = np.array(np.imag(xt), dtype=np.float64, copy=True)
    rc = lib().orc_sweep_z(pl.n, _ptr(pl.rp), _ptr(pl.ci), _ptr(pl.vr), _ptr(pl.vi), _ptr(pl.fr), _ptr(pl.fi),
                           _ptr(pl.inv), _ptr(pl.group), pl.ngroups, pl.omega, _ptr(xr), _ptr(xi), int(sweeps))
    if rc != 0:
        raise RuntimeError(f"orc_sweep_z failed: {rc}")
    return xr + 1j * xi


def rowwise_complex(pl: ComplexPlan, rows, xt: np.ndarray) -> np.ndarray:
    xr = np.array(np.real(xt), dtype=np.float64, copy=True)
    xi = np.array(np.imag(xt), dtype=np.float64, copy=True)
    rows = _c(rows, np.int32)
    lib().orc_rowwise_z(pl.n, _ptr(pl.rp), _ptr(pl.ci), _ptr(pl.vr), _ptr(pl.vi), _ptr(pl.fr), _ptr(pl.fi),
                        _ptr(pl.inv), _ptr(rows), len(rows), _ptr(xr), _ptr(xi))
    return xr + 1j * xi


def relres_complex(n, rp, ci, vz, fz, xz) -> float:
    vz, fz, xz = (np.asarray(a, dtype=np.complex128) for a in (vz, fz, xz))
    return float(lib().orc_relres_z(n, _ptr(_c(rp, np.int64)), _ptr(_c(ci, np.int32)), _ptr(_c(vz.real, np.float64)),
                                    _ptr(_c(vz.imag, np.float64)), _ptr(_c(fz.real, np.float64)),
                                    _ptr(_c(fz.imag, np.float64)), _ptr(_c(xz.real, np.float64)),
                                    _ptr(_c(xz.imag, np.float64))))


def solve_complex(pl: ComplexPlan, sweeps: int, x0: np.ndarray | None = None) -> np.ndarray:
    """Plan + sweeps from x0 (default 0), original ordering."""
    xt = np.zeros(pl.n, dtype=np.complex128) if x0 is None else np.asarray(x0, dtype=np.complex128)[pl.p]
    xt = sweep_complex(pl, xt, sweeps)
    x = np.empty(pl.n, dtype=np.complex128)
    x[pl.p] = xt
    return x


def plan_system_complex(s, delta, **kw) -> ComplexPlan:
    return plan_complex(s.n, s.row_ptr, s.col, s.val, s.f, delta, **kw)


# ------------------------------------------- relaxation bound (one-row groups)
def lambda_bound(pl) -> tuple[float, np.ndarray]:
    """Gershgorin bound on lambda_max(B_g B_g^H) for every group g, B_g being
    the rows of g scaled to unit norm: max over the rows i of g of
    sum_j |(B_g B_g^H)_ij| (the diagonal entry 1 plus the row's cosines).

    The paper is silent on relaxation (it steps with omega = 1); the group
    step e <- (I - omega B_g^H B_g) e does not expand the error when
    omega * lambda_max <= 2, which this bound certifies.  The bound of a plan
    is the largest over its groups (0 with no groups).  Real or complex
    plans; the product B B^H is a library sparse product."""
    n = pl.n
    vals = (pl.vr + 1j * pl.vi) if isinstance(pl, ComplexPlan) else pl.v
    A = sp.csr_matrix((vals, pl.ci, pl.rp), shape=(n, n))
    act = pl.group >= 0
    scale = np.zeros(n)
    scale[act] = 1.0 / np.sqrt(pl.nu[act])
    B = sp.diags(scale) @ A
    C = abs(B @ B.conj().T).tocoo()
    same = (pl.group[C.row] == pl.group[C.col]) & (pl.group[C.row] >= 0)
    rowsum = np.zeros(n)
    np.add.at(rowsum, C.row[same], C.data[same])
    per = np.zeros(pl.ngroups)
    np.maximum.at(per, pl.group[act], rowsum[act])
    return (float(per.max()) if per.size else 0.0), per
