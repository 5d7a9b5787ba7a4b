"""The oracle's pins must catch plausible mistakes.

Each mutant is a copy of ``oracle/obk_oracle.c`` with one planted mistake (a
dropped term, a wrong sign, index or direction, a transposed operand), built
on the CPU into a temporary library.  The pin suite is run against it in a
subprocess and must fail.  Nothing here touches the GPU or the library.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "obk_oracle.c")

# each pin run is single-threaded, so that parallel mutant runs do not
# oversubscribe the cores with BLAS threads
_ONE_THREAD = {"OMP_NUM_THREADS": "1", "OPENBLAS_NUM_THREADS": "1", "MKL_NUM_THREADS": "1"}

# (name, exact text in the source, replacement)
MUTANTS = [
    ("rcm_not_reversed", "p[t] = order[n - 1 - t];", "p[t] = order[t];"),
    ("rcm_ignores_degree", "if (da != db) return da < db ? -1 : 1;", "(void)da; (void)db;"),
    ("permute_no_relabel", "buf[k].c = q[ci[rp[old] + k]];", "buf[k].c = ci[rp[old] + k];"),
    ("norm_abs_not_square", "s = s + v[k] * v[k];", "s = s + fabs(v[k]);"),
    ("cosine_no_sqrt", "return fabs(d) / sqrt(nu[i] * nu[j]);", "return fabs(d) / (nu[i] * nu[j]);"),
    ("cosine_signed", "return fabs(d) / sqrt(nu[i] * nu[j]);", "return d / sqrt(nu[i] * nu[j]);"),
    ("threshold_strict", "if (orc_cosine(i, j, rp, ci, v, nu) >= delta) {",
     "if (orc_cosine(i, j, rp, ci, v, nu) > delta) {"),
    ("firstfit_skips_zero", "int32_t g = 0;\n        while (used[g]) g++;",
     "int32_t g = 1;\n        while (used[g]) g++;"),
    ("sweep_sign", "w[i] = ((f[i] - s) * inv[i]) * omega;\n            }\n            /* (ii)",
     "w[i] = ((s - f[i]) * inv[i]) * omega;\n            }\n            /* (ii)"),
    ("sweep_omega_dropped", "w[i] = ((f[i] - s) * inv[i]) * omega;\n            }\n            /* (ii)",
     "w[i] = ((f[i] - s) * inv[i]);\n            }\n            /* (ii)"),
    ("sweep_gathers_wrong_x", "for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[ci[k]];\n"
     "                w[i] = ((f[i] - s) * inv[i]) * omega;\n            }\n            /* (ii)",
     "for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[i];\n"
     "                w[i] = ((f[i] - s) * inv[i]) * omega;\n            }\n            /* (ii)"),
    ("sweep_drops_update", "x[c] = x[c] + t[c];", "x[c] = t[c];"),
    ("sweep_sequential_within_group", "x[c] = x[c] + t[c];", "x[c] = x[c];"),
    ("relres_no_sqrt", "? 0.0 : -1.0;\n    return sqrt(rr) / sqrt(ff);", "? 0.0 : -1.0;\n    return rr / ff;"),
    ("unpermute_wrong_direction", "for (int64_t t = 0; t < n; t++) x[p[t]] = xt[t];",
     "for (int64_t t = 0; t < n; t++) x[t] = xt[p[t]];"),
    ("refine_unscaled", "x[i] = x[i] + sigma * d[i];", "x[i] = x[i] + d[i];"),
    ("stop_ignores_check_every", "if (tol > 0.0 && check_every < c) c = check_every;",
     "if (tol > 0.0 && 1 < c) c = 1;"),
    ("stop_divergence_factor", "else if (rho0 > 0.0 && cur > 1e3 * rho0) status = ORC_DIVERGED;",
     "else if (rho0 > 0.0 && cur > 1e2 * rho0) status = ORC_DIVERGED;"),
    ("stop_misses_nonfinite", "*nonfinite = !isfinite(rr);", "*nonfinite = 0;"),
    ("stop_squared_residual", "    if (ff == 0.0) return rr == 0.0 ? 0.0 : INFINITY;\n    return sqrt(rr) / sqrt(ff);",
     "    if (ff == 0.0) return rr == 0.0 ? 0.0 : INFINITY;\n    return rr / ff;"),
    ("z_cosine_no_conjugate", "di = di + (vr[a] * vi[b] - vi[a] * vr[b]);",
     "di = di + (vr[a] * vi[b] + vi[a] * vr[b]);"),
    ("z_norm_real_part_only", "s = s + (vr[k] * vr[k] + vi[k] * vi[k]);", "s = s + vr[k] * vr[k];"),
    ("z_update_no_conjugate", "ti[c] = ti[c] + (wi[i] * vr[k] - wr[i] * vi[k]);",
     "ti[c] = ti[c] + (wi[i] * vr[k] + wr[i] * vi[k]);"),
    ("z_product_sign", "sr = sr + (vr[k] * xr[c] - vi[k] * xi[c]);\n"
     "                    si = si + (vr[k] * xi[c] + vi[k] * xr[c]);\n                }\n                wr[i]",
     "sr = sr + (vr[k] * xr[c] + vi[k] * xi[c]);\n"
     "                    si = si + (vr[k] * xi[c] + vi[k] * xr[c]);\n                }\n                wr[i]"),
]


def _apply(src, old, new, name):
    assert src.count(old) == 1, f"mutation site for {name} is not unique"
    return src.replace(old, new)


@pytest.fixture(scope="module")
def source():
    with open(SRC) as fh:
        return fh.read()


def _sequential_patch(src):
    # within a group, apply each row's update at once (the mistake of running
    # the class rows one after another from the latest iterate)
    old = "                w[i] = ((f[i] - s) * inv[i]) * omega;\n            }\n            /* (ii)"
    new = ("                w[i] = ((f[i] - s) * inv[i]) * omega;\n"
           "                for (int64_t k = rp[i]; k < rp[i + 1]; k++) x[ci[k]] = x[ci[k]] + w[i] * v[k];"
           "\n            }\n            /* (ii)")
    src = _apply(src, old, new, "seq")
    return src


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(source, name, old, new, tmp_path):
    src = _apply(source, old, new, name)
    if name == "sweep_sequential_within_group":
        src = _sequential_patch(src)
    csrc = tmp_path / "mutant.c"
    so = tmp_path / "libmutant.so"
    csrc.write_text(src)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-shared", "-fPIC", "-o", str(so),
                    str(csrc), "-lm"], check=True)
    env = dict(os.environ, OBK_ORACLE_LIB=str(so), **_ONE_THREAD)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"


# Mistakes planted in the Python half of the oracle (oracle/__init__.py: the
# block form, its criteria, the non-square extension and the relaxation bound).
PY_MUTANTS = [
    ("centroid_of_abs_values", "cen[b] = np.asarray(A[bptr[b]:bptr[b + 1]].sum(axis=0))",
     "cen[b] = np.asarray(abs(A[bptr[b]:bptr[b + 1]]).sum(axis=0))"),
    ("centroid_is_first_row", "cen[b] = np.asarray(A[bptr[b]:bptr[b + 1]].sum(axis=0))",
     "cen[b] = np.asarray(A[bptr[b]:bptr[b] + 1].sum(axis=0))"),
    ("tau2_before_tau1", "            x = block_project(bp, t1, x)\n            x = block_project(bp, t2, x)",
     "            x = block_project(bp, t2, x)\n            x = block_project(bp, t1, x)"),
    ("nclass_before_pairs",
     "        for t1, t2 in bp.pairs:\n            x = block_project(bp, t1, x)\n            x = block_project(bp, t2, x)\n"
     "        for t in bp.nclass:\n            x = block_project(bp, t, x)",
     "        for t in bp.nclass:\n            x = block_project(bp, t, x)\n"
     "        for t1, t2 in bp.pairs:\n            x = block_project(bp, t1, x)\n            x = block_project(bp, t2, x)"),
    ("block_projection_sign", "return x + np.linalg.pinv(A) @ (bp.f[r0:r1] - A @ x)",
     "return x - np.linalg.pinv(A) @ (bp.f[r0:r1] - A @ x)"),
    ("chunks_ceil", "size = m // k", "size = -(-m // k)"),
    ("zn_counts_nonzeros", "return n1 / num, nz.size * nm / num", "return nz.size / num, nz.size * nm / num"),
    ("nn_mean_only", "return n1 / num, nz.size * nm / num", "return n1 / num, nm / num"),
    ("select_least_zn", "key = (-zn, nn, k)", "key = (zn, nn, k)"),
    ("pad_rhs_ones", "f = np.concatenate([f, np.zeros(N - m)])", "f = np.concatenate([f, np.ones(N - m)])"),
    ("stop_status_names_swapped", 'SOLVE_STATUS = {0: "converged", 1: "maxit", 2: "diverged", 3: "nonfinite"}',
     'SOLVE_STATUS = {0: "converged", 1: "diverged", 2: "maxit", 3: "nonfinite"}'),
    ("lambda_signed_cosines", "C = abs(B @ B.conj().T).tocoo()", "C = (B @ B.conj().T).real.tocoo()"),
    ("lambda_no_conjugate", "C = abs(B @ B.conj().T).tocoo()", "C = abs(B @ B.T).tocoo()"),
    ("lambda_rows_not_scaled", "scale[act] = 1.0 / np.sqrt(pl.nu[act])", "scale[act] = 1.0 / pl.nu[act]"),
    ("lambda_across_groups", "same = (pl.group[C.row] == pl.group[C.col]) & (pl.group[C.row] >= 0)",
     "same = (pl.group[C.row] >= 0) & (pl.group[C.col] >= 0)"),
    ("lambda_without_diagonal", "same = (pl.group[C.row] == pl.group[C.col]) & (pl.group[C.row] >= 0)",
     "same = (pl.group[C.row] == pl.group[C.col]) & (pl.group[C.row] >= 0) & (C.row != C.col)"),
]


@pytest.fixture(scope="module")
def py_source():
    with open(os.path.join(ROOT, "oracle", "__init__.py")) as fh:
        return fh.read()


def _run_pins_on_copy(tmp_path, init_text):
    import shutil
    import oracle
    oracle.lib()                        # builds liboracle.so if it is missing
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("build.py", "obk_oracle.c", "liboracle.so"):
        shutil.copy(os.path.join(ROOT, "oracle", f), pkg / f)
    (pkg / "__init__.py").write_text(init_text)
    env = dict(os.environ, OBK_ORACLE_PKG=str(tmp_path), **_ONE_THREAD)
    env.pop("OBK_ORACLE_LIB", None)
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                          env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)


def test_python_mutant_harness_imports_the_copy(py_source, tmp_path):
    """Control: the pins import the planted copy, not the package in the tree."""
    r = _run_pins_on_copy(tmp_path, py_source + '\nraise ImportError("planted copy loaded")\n')
    assert r.returncode != 0 and "planted copy loaded" in r.stdout + r.stderr


@pytest.mark.parametrize("name,old,new", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_pins_catch_python_mutant(py_source, name, old, new, tmp_path):
    r = _run_pins_on_copy(tmp_path, _apply(py_source, old, new, name))
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
