"""obk_solve_noalloc (the solve that allocates no device memory: residual
partials in a static device array) against obk_solve, through the C ABI:
the same iterate, sweeps and residuals, on two calls in a row, the second on
a smaller system (the static array keeps the first call's contents)."""
import sys

import numpy as np
import pytest

import synth
import paper_2401_00672_amd as obk

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("kw", [dict(), dict(sweep_kernel="phases"), dict(precision=1, inner_sweeps=8)],
                         ids=["fp64-auto-engine", "fp64-phase-kernels", "fp32-refinement"])
def test_noalloc_solve_equals_solve(kw):
    import torch
    big = synth.c2(grid=256) if "precision" not in kw else synth.c1(n=20000, companion=True)
    small = synth.c2(grid=40) if "precision" not in kw else synth.c1(n=700, companion=True)
    tol = 1e-6 if "precision" not in kw else 1e-10
    for name, s in (("first (larger)", big), ("second (smaller)", small)):
        _say(f"[noalloc] {kw} {name}: n={s.n}")
        P = obk.plan_system(s, 0.1, **kw)
        try:
            x0 = torch.tensor(np.random.default_rng(5).standard_normal(s.n) * 1e-3, device="cuda")
            xa, ia = P.solve(x0=x0.cpu().numpy(), tol=tol, maxit=400)
            xb, ib = P.solve_noalloc(x0=x0, tol=tol, maxit=400)
            xb = xb.cpu().numpy()
            _say(f"[noalloc] {name}: {ia.status} {ia.sweeps} sweeps relres {ia.relres:.3e} | noalloc {ib.status} "
                 f"{ib.sweeps} relres {ib.relres:.3e} bitwise {np.array_equal(xa, xb)}")
            assert (ia.status, ia.sweeps, ia.outer_steps) == (ib.status, ib.sweeps, ib.outer_steps)
            assert ia.relres0 == ib.relres0 and ia.relres == ib.relres
            assert np.abs(xa - xb).max() <= 1e-10 * np.abs(xa).max()
            # tol <= 0: a fixed number of sweeps (refinement steps of 8 inner
            # sweeps for an FP32 plan) from zero
            xc, ic = P.solve(maxit=7)
            xd, idd = P.solve_noalloc(maxit=7)
            assert (ic.sweeps, ic.outer_steps) == (idd.sweeps, idd.outer_steps)
            assert ic.sweeps == (7 * 8 if "precision" in kw else 7)
            assert np.array_equal(xc, xd.cpu().numpy())
        finally:
            P.free()
