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
    ("sweep_sign", "w[i] = (f[i] - s) * inv[i];", "w[i] = (s - f[i]) * inv[i];"),
    ("sweep_gathers_wrong_x", "for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[ci[k]];\n"
     "                w[i]", "for (int64_t k = rp[i]; k < rp[i + 1]; k++) s = s + v[k] * x[i];\n"
     "                w[i]"),
    ("sweep_drops_update", "x[c] = x[c] + t[c];", "x[c] = t[c];"),
    ("sweep_sequential_within_group", "x[c] = x[c] + t[c];", "x[c] = x[c];"),
    ("relres_no_sqrt", "return sqrt(rr) / sqrt(ff);", "return rr / ff;"),
    ("unpermute_wrong_direction", "for (int64_t t = 0; t < n; t++) x[p[t]] = xt[t];",
     "for (int64_t t = 0; t < n; t++) x[t] = xt[p[t]];"),
    ("refine_unscaled", "x[i] = x[i] + sigma * d[i];", "x[i] = x[i] + d[i];"),
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
    old = "                w[i] = (f[i] - s) * inv[i];"
    new = ("                w[i] = (f[i] - s) * inv[i];\n"
           "                for (int64_t k = rp[i]; k < rp[i + 1]; k++) x[ci[k]] = x[ci[k]] + w[i] * v[k];")
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
    env = dict(os.environ, OBK_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant {name} survived the pins:\n{r.stdout[-2000:]}"
