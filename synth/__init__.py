"""Seeded synthetic sparse systems ``A x = f`` (problem statement, eq. 1.1).

This module only draws random inputs; it holds none of the solver's
arithmetic.  Both the FP64 CPU oracle and the HIP path are fed from here,
so that the two see bit-identical CSR matrices and right-hand sides.

The paper evaluates on SuiteSparse matrices (Section 3.5, Table 3) that are
not available here; the families below stand in for them:

* ``c1``        2,000 rows, diagonal U(1,2) plus 4 off-diagonal N(0,1) entries
                per row at distinct uniform columns, then a random symmetric
                permutation (scattered pattern).
* ``c2``        2-D 5-point stencil on a 1024x1024 grid (diagonal 4+U(0,0.1),
                -1 to each N/S/E/W neighbour, Dirichlet), random symmetric
                permutation.  ``grid`` sets the side for smaller cases.
* ``c3``        2,000,000 rows, diagonal U(1,2) plus 11 distinct uniform
                off-diagonal N(0,1) entries per row (12 nnz/row).
* ``c4``        512 systems, n log-uniform in [1e3, 2e5], 4..16 nnz per row
                including the diagonal.
* ``c5``        serving requests, n log-uniform in [500, 5e5], 4..16 nnz/row.
* ``companion=True`` replaces the diagonal by U(1,2) + sum_j |a_ij| (row
  diagonal dominance), keeping pattern, off-diagonal values and seeds.
* ``c1z``, ``c2z`` complex counterparts of ``c1`` and ``c2`` (the paper also
  solves the complex matrix kim1): same patterns, complex values, complex
  x*; ``c2z(grid=196)`` has kim1's order (38,416 rows against 38,415).

Conventions: ``numpy.random.Generator(PCG64(seed))`` with
``seed = 1000*config + system_index``.  Draw order per system: per-row nnz
(families with variable rows), off-diagonal columns, off-diagonal values,
diagonal values, symmetric permutation (where used), x* ~ N(0,1).
f = A x* is formed in FP64 by scipy's CSR product.

CSR layout everywhere: int64 ``row_ptr[n+1]``, int32 ``col[nnz]`` sorted
ascending within each row, float64 ``val[nnz]``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp

__all__ = [
    "System", "seed_for", "random_rows", "stencil", "c1", "c2", "c3",
    "c4_sizes", "c4_system", "c5_sizes", "c5_system", "c5_arrivals",
    "from_dense", "from_scipy", "RectSystem", "rect", "ComplexSystem", "c1z", "c2z",
]


@dataclasses.dataclass
class System:
    """A square sparse system in CSR form with its generating solution."""
    n: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [nnz]
    val: np.ndarray          # float64 [nnz]
    f: np.ndarray            # float64 [n]
    x_star: np.ndarray       # float64 [n]
    name: str = ""
    seed: int = -1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


@dataclasses.dataclass
class RectSystem:
    """A consistent m x n sparse system (m != n allowed) in CSR form."""
    m: int
    n: int
    row_ptr: np.ndarray      # int64 [m+1]
    col: np.ndarray          # int32 [nnz], values < n
    val: np.ndarray          # float64 [nnz]
    f: np.ndarray            # float64 [m]
    x_star: np.ndarray       # float64 [n]
    name: str = ""
    seed: int = -1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.m, self.n))


def seed_for(config: int, index: int = 0) -> int:
    return 1000 * int(config) + int(index)


def _pack(A: sp.spmatrix, x_star: np.ndarray, name: str, seed: int) -> System:
    A = sp.csr_matrix(A)
    A.sum_duplicates()
    A.sort_indices()
    f = A @ x_star
    return System(
        n=A.shape[0],
        row_ptr=np.ascontiguousarray(A.indptr, dtype=np.int64),
        col=np.ascontiguousarray(A.indices, dtype=np.int32),
        val=np.ascontiguousarray(A.data, dtype=np.float64),
        f=np.ascontiguousarray(f, dtype=np.float64),
        x_star=np.ascontiguousarray(x_star, dtype=np.float64),
        name=name, seed=seed)


def from_scipy(A: sp.spmatrix, x_star: np.ndarray | None = None, f: np.ndarray | None = None,
               name: str = "custom") -> System:
    """Wrap an explicit matrix.  If ``f`` is given it is kept as-is."""
    A = sp.csr_matrix(A)
    A.sort_indices()
    n = A.shape[0]
    if x_star is None:
        x_star = np.zeros(n)
    s = _pack(A, np.asarray(x_star, dtype=np.float64), name, -1)
    if f is not None:
        s.f = np.ascontiguousarray(f, dtype=np.float64)
    return s


def from_dense(M: np.ndarray, x_star: np.ndarray | None = None, f: np.ndarray | None = None,
               name: str = "dense") -> System:
    """CSR of a small dense matrix; exact zeros are not stored."""
    return from_scipy(sp.csr_matrix(np.asarray(M, dtype=np.float64)), x_star, f, name)


def _distinct_offdiag_columns(rng: np.random.Generator, n: int, k: np.ndarray):
    """Per row i, k[i] distinct columns uniform over {0..n-1} minus {i}.

    Rows are drawn as a batch of k_max candidates with replacement from
    {0..n-2}; a row whose first k[i] candidates repeat is redrawn whole
    (rejection keeps the subset uniform).  Candidates v >= i map to v+1.
    Returns the candidate matrix and the mask of its used entries.
    """
    kmax = int(k.max()) if len(k) else 0
    if kmax > n - 1:
        raise ValueError("more off-diagonals than columns")
    cand = rng.integers(0, max(n - 1, 1), size=(n, kmax), dtype=np.int64)
    mask = np.arange(kmax)[None, :] < k[:, None]
    filler = (n + 7 + np.arange(kmax, dtype=np.int64))[None, :]

    def dup_rows(c: np.ndarray, m: np.ndarray) -> np.ndarray:
        if kmax < 2:
            return np.zeros(0, dtype=np.int64)
        s = np.sort(np.where(m, c, filler), axis=1)
        return np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0]

    bad = dup_rows(cand, mask)
    while bad.size:
        cand[bad] = rng.integers(0, n - 1, size=(bad.size, kmax), dtype=np.int64)
        bad = bad[dup_rows(cand[bad], mask[bad])]
    rows = np.arange(n, dtype=np.int64)
    cand = np.where(cand >= rows[:, None], cand + 1, cand)
    return cand, mask


def _random_rows_from(rng: np.random.Generator, n: int, k: np.ndarray, *, permute: bool,
                      companion: bool, name: str, seed: int) -> System:
    cols, mask = _distinct_offdiag_columns(rng, n, k)
    offv = rng.standard_normal(size=cols.shape)
    diag = rng.uniform(1.0, 2.0, size=n)
    rr = np.repeat(np.arange(n, dtype=np.int64), k)
    cc = cols[mask]
    vv = offv[mask]
    if companion:
        diag = diag + np.bincount(rr, weights=np.abs(vv), minlength=n)
    r_all = np.concatenate([rr, np.arange(n, dtype=np.int64)])
    c_all = np.concatenate([cc, np.arange(n, dtype=np.int64)])
    v_all = np.concatenate([vv, diag])
    A = sp.csr_matrix((v_all, (r_all, c_all)), shape=(n, n))
    if permute:
        perm = rng.permutation(n)          # new -> old
        A = A[perm][:, perm]
    x_star = rng.standard_normal(n)
    return _pack(A, x_star, name + ("-companion" if companion else ""), seed)


def random_rows(n: int, k_off: int, seed: int, *, permute: bool = False, companion: bool = False,
                name: str = "random") -> System:
    """Diagonal U(1,2) plus ``k_off`` off-diagonal N(0,1) entries on every row."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.full(n, int(k_off), dtype=np.int64)
    return _random_rows_from(rng, n, k, permute=permute, companion=companion, name=name, seed=seed)


def stencil(grid: int, seed: int, *, permute: bool = True, name: str = "stencil") -> System:
    """5-point stencil on a grid x grid mesh, natural index r*grid + c.

    Diagonal 4 + U(0, 0.1); -1 to each existing N/S/E/W neighbour.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = grid * grid
    idx = np.arange(n, dtype=np.int64).reshape(grid, grid)
    rows, cols = [], []
    for dr, dc in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        r0, r1 = max(0, -dr), grid - max(0, dr)
        c0, c1 = max(0, -dc), grid - max(0, dc)
        src = idx[r0:r1, c0:c1].ravel()
        dst = idx[r0 + dr:r1 + dr, c0 + dc:c1 + dc].ravel()
        rows.append(src)
        cols.append(dst)
    rr = np.concatenate(rows)
    cc = np.concatenate(cols)
    diag = 4.0 + rng.uniform(0.0, 0.1, size=n)
    A = sp.csr_matrix((np.concatenate([-np.ones(rr.size), diag]),
                       (np.concatenate([rr, np.arange(n)]), np.concatenate([cc, np.arange(n)]))),
                      shape=(n, n))
    if permute:
        perm = rng.permutation(n)
        A = A[perm][:, perm]
    x_star = rng.standard_normal(n)
    return _pack(A, x_star, f"{name}{grid}", seed)


def c1(index: int = 0, *, n: int = 2000, companion: bool = False) -> System:
    """2,000 rows, 4 off-diagonals per row, scattered by a symmetric permutation."""
    return random_rows(n, 4, seed_for(1, index), permute=True, companion=companion, name=f"c1-n{n}")


def c2(index: int = 0, *, grid: int = 1024) -> System:
    """1024x1024 5-point stencil under a random symmetric permutation."""
    return stencil(grid, seed_for(2, index), permute=True, name="c2-grid")


def c3(index: int = 0, *, n: int = 2_000_000, companion: bool = False) -> System:
    """n rows, 12 nnz per row (diagonal plus 11 uniform off-diagonals)."""
    return random_rows(n, 11, seed_for(3, index), permute=False, companion=companion, name=f"c3-n{n}")


def _loguniform_sizes(rng: np.random.Generator, count: int, lo: float, hi: float) -> np.ndarray:
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def c4_sizes(count: int = 512, lo: float = 1e3, hi: float = 2e5) -> np.ndarray:
    """System sizes of the batched family (drawn from seed 4000)."""
    return _loguniform_sizes(np.random.Generator(np.random.PCG64(seed_for(4, 0))), count, lo, hi)


def _variable_rows(n: int, seed: int, companion: bool, name: str) -> System:
    """4..16 nnz per row including the diagonal; the per-row count is drawn first."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nnz_row = rng.integers(4, 17, size=n)
    k_off = np.minimum(nnz_row - 1, n - 1).astype(np.int64)
    return _random_rows_from(rng, n, k_off, permute=False, companion=companion, name=name, seed=seed)


def c4_system(index: int, n: int | None = None, *, companion: bool = False) -> System:
    """System ``index`` of the batched family (seed 4000 + 1 + index)."""
    if n is None:
        n = int(c4_sizes()[index])
    return _variable_rows(n, seed_for(4, 1 + index), companion, f"c4-{index}-n{n}")


def c5_sizes(count: int = 8192, lo: float = 500, hi: float = 5e5) -> np.ndarray:
    return _loguniform_sizes(np.random.Generator(np.random.PCG64(seed_for(5, 0))), count, lo, hi)


def c5_system(index: int, n: int | None = None, *, companion: bool = True) -> System:
    if n is None:
        n = int(c5_sizes()[index])
    return _variable_rows(n, seed_for(5, 1 + index), companion, f"c5-{index}-n{n}")


def c5_arrivals(count: int, rate_per_s: float) -> np.ndarray:
    """Poisson arrival times (seconds) at ``rate_per_s``, from seed 5000."""
    rng = np.random.Generator(np.random.PCG64(5000))
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=count))


def rect(m: int, n: int, density: float, index: int = 0) -> RectSystem:
    """Rectangular family of the non-square experiments (the row, column and
    density figures of Tables 6 and 8): round(density * m * n) distinct
    positions uniform over the m x n grid, N(0,1) values, x* ~ N(0,1),
    f = A x*.  Seed 1000 * 6 + index; draw order: positions, values, x*."""
    seed = seed_for(6, index)
    rng = np.random.Generator(np.random.PCG64(seed))
    nnz = int(round(density * m * n))
    pos = np.sort(rng.choice(m * n, size=nnz, replace=False))
    rows, cols = pos // n, pos % n
    vals = rng.standard_normal(nnz)
    x_star = rng.standard_normal(n)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    f = A @ x_star
    return RectSystem(m=m, n=n, row_ptr=np.ascontiguousarray(A.indptr, dtype=np.int64),
                      col=np.ascontiguousarray(A.indices, dtype=np.int32),
                      val=np.ascontiguousarray(A.data, dtype=np.float64),
                      f=np.ascontiguousarray(f, dtype=np.float64),
                      x_star=np.ascontiguousarray(x_star, dtype=np.float64),
                      name=f"rect-{m}x{n}-d{density}", seed=seed)


# ------------------------------------------------------------ complex systems
@dataclasses.dataclass
class ComplexSystem:
    """A square sparse complex system in CSR form with its generating solution."""
    n: int
    row_ptr: np.ndarray      # int64 [n+1]
    col: np.ndarray          # int32 [nnz]
    val: np.ndarray          # complex128 [nnz]
    f: np.ndarray            # complex128 [n]
    x_star: np.ndarray       # complex128 [n]
    name: str = ""
    seed: int = -1

    @property
    def nnz(self) -> int:
        return int(self.col.size)

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _pack_z(A, x_star, name: str, seed: int) -> ComplexSystem:
    A = sp.csr_matrix(A, dtype=np.complex128)
    A.sum_duplicates()
    A.sort_indices()
    f = A @ x_star
    return ComplexSystem(n=A.shape[0],
                         row_ptr=np.ascontiguousarray(A.indptr, dtype=np.int64),
                         col=np.ascontiguousarray(A.indices, dtype=np.int32),
                         val=np.ascontiguousarray(A.data, dtype=np.complex128),
                         f=np.ascontiguousarray(f, dtype=np.complex128),
                         x_star=np.ascontiguousarray(x_star, dtype=np.complex128), name=name, seed=seed)


def c1z(index: int = 0, *, n: int = 2000, companion: bool = False) -> ComplexSystem:
    """Complex counterpart of c1: 4 off-diagonals per row at distinct uniform
    columns with N(0,1) + i N(0,1) values, a diagonal of modulus U(1,2) (plus
    sum_j |a_ij| for the companion) and phase U(0, 2 pi), then a random
    symmetric permutation.  Seed 1000 * 7 + index; draw order: columns,
    off-diagonal real parts, imaginary parts, diagonal moduli, phases,
    permutation, x* real parts, imaginary parts."""
    seed = seed_for(7, index)
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.full(n, 4, dtype=np.int64)
    cols, mask = _distinct_offdiag_columns(rng, n, k)
    off_re = rng.standard_normal(size=cols.shape)
    off_im = rng.standard_normal(size=cols.shape)
    mod = rng.uniform(1.0, 2.0, size=n)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n)
    rr = np.repeat(np.arange(n, dtype=np.int64), k)
    vv = off_re[mask] + 1j * off_im[mask]
    if companion:
        mod = mod + np.bincount(rr, weights=np.abs(vv), minlength=n)
    diag = mod * np.exp(1j * phase)
    A = sp.csr_matrix((np.concatenate([vv, diag]),
                       (np.concatenate([rr, np.arange(n)]), np.concatenate([cols[mask], np.arange(n)]))),
                      shape=(n, n), dtype=np.complex128)
    perm = rng.permutation(n)
    A = A[perm][:, perm]
    x_star = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return _pack_z(A, x_star, f"c1z-n{n}" + ("-companion" if companion else ""), seed)


def c2z(index: int = 0, *, grid: int = 1024) -> ComplexSystem:
    """Complex counterpart of c2: the 5-point stencil pattern with -1 + 0.25 i g
    (g ~ N(0,1)) to each neighbour and 4 + U(0, 0.1) + i U(-0.5, 0.5) on the
    diagonal, under a random symmetric permutation.  Seed 1000 * 8 + index;
    draw order: neighbour imaginary parts, diagonal real parts, diagonal
    imaginary parts, permutation, x* real parts, imaginary parts."""
    seed = seed_for(8, index)
    rng = np.random.Generator(np.random.PCG64(seed))
    n = grid * grid
    idx = np.arange(n, dtype=np.int64).reshape(grid, grid)
    rows, cols = [], []
    for dr, dc in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        r0, r1 = max(0, -dr), grid - max(0, dr)
        c0, c1 = max(0, -dc), grid - max(0, dc)
        rows.append(idx[r0:r1, c0:c1].ravel())
        cols.append(idx[r0 + dr:r1 + dr, c0 + dc:c1 + dc].ravel())
    rr = np.concatenate(rows)
    cc = np.concatenate(cols)
    off = -1.0 + 0.25j * rng.standard_normal(rr.size)
    dre = 4.0 + rng.uniform(0.0, 0.1, size=n)
    dim = rng.uniform(-0.5, 0.5, size=n)
    A = sp.csr_matrix((np.concatenate([off, dre + 1j * dim]),
                       (np.concatenate([rr, np.arange(n)]), np.concatenate([cc, np.arange(n)]))),
                      shape=(n, n), dtype=np.complex128)
    perm = rng.permutation(n)
    A = A[perm][:, perm]
    x_star = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return _pack_z(A, x_star, f"c2z-grid{grid}", seed)
