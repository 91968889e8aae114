"""Parity of the timed workload itself: Cook 64x64x4 (98,304 P1 tets),
lambda/mu = 5000, dead traction schedule tau = 1, 2, 4, 8, 16 with halving
of a failed increment, solved exactly as the benchmark solves it, against the
oracle's root of the same schedule (stored in tests/golden/ by
tests/golden/make_golden.py, which runs exact Newton with a complex-step
tangent and sparse LU to ||r|| <= 1e-13 ||r_0||).

Gates: displacement relative error (2-norm) <= 1e-6 for the mixed-precision
methods, <= 1e-8 for the FP64 methods, at the schedule's own stopping rule
||r|| <= 1e-8 ||r_0||.  No tighter rule is used here: at lambda/mu = 5000 the
FP64 residual's rounding floor lies near 1e-9 of ||r_0|| (the oracle's exact
Newton stalls at 3e-9, the GPU's at 5e-10), and at the 1e-8 rule the roots
already agree to ~1e-13.  Where paths could land on different equilibria at this load
(both residuals converged but u apart), the failure message says so
("branch") with both potentials.
"""

import os

import numpy as np
import pytest

import synthetic as syn
from oracle import fem
from tests.gpu_common import MU

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import bench  # noqa: E402
from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "cook64x64x4_l5000_tau16.npy")


@pytest.fixture(scope="module")
def cook64():
    mesh = syn.cook_mesh(*bench.GRID)
    P = fem.cook_problem(mesh, mu=MU, lam=bench.RATIO * MU, tau=1.0)
    ustar = np.load(GOLDEN)
    assert ustar.shape == (P.n_dofs,)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, bench.RATIO * MU, 1.0, block_size=bench.HEAD_BLOCK)
    yield mesh, P, ustar, ctx
    ctx.close()


def _check(P, ustar, uh, tol, method):
    err = float(np.linalg.norm(uh - ustar) / np.linalg.norm(ustar))
    if err > tol:
        r = np.linalg.norm(P.residual(uh, 16.0)) / np.linalg.norm(P.residual(P.lift(0 * uh), 16.0))
        branch = r <= 1e-6
        raise AssertionError(
            f"{method}: |u - u*|/|u*| = {err:.3e} > {tol:g}; oracle residual of the GPU root "
            f"{r:.2e} relative; " + (f"branch: Pi(u) = {P.energy(uh, 16.0):.10e}, "
                                     f"Pi(u*) = {P.energy(ustar, 16.0):.10e}" if branch else
                                     "not a root"))
    return err


@pytest.mark.parametrize("method", ["ink_mixed_cg3_amg", "ink_mixed_cg_amg", "ink_fp64_cg_amg",
                                    "nk_fp64_minres_amg"])
def test_headline_schedule_matches_oracle_root(cook64, method):
    mesh, P, ustar, ctx = cook64
    solver, prec, kw = bench.METHODS[method]
    opts = problems.make_opts(solver, prec, **{"pc": "jacobi", **kw})
    fp64 = prec == "fp64"
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    sched = bench.load_schedule()
    reps = problems.solve_schedule(ctx, u, solver, opts, sched)
    assert problems.schedule_ok(reps, sched), [(r["load_scale"], r["status_name"], r["nit"],
                                                r["rnorm_final"] / max(r["rnorm0"], 1e-300))
                                               for r in reps]
    err = _check(P, ustar, u.cpu().numpy(), 1e-8 if fp64 else 1e-6, method)
    print(f"{method}: rel. error {err:.2e}, attempts "
          f"{[(r['load_scale'], r['status_name'], r['nit']) for r in reps]}")
