"""GPU parity of the follower Cook traction (fixed direction, per unit current
area; the Cook load in the deformed configuration of Sec. 4) against the FP64
oracle: residual, Jacobian action (FP64, FP32), diagonal and nodal blocks at
seeded states and load scales, and solves (NK / iNK / inexact BFGS with GMRES)
against the oracle's exact-Newton roots.

Tolerances: kernels FP64 <= 1e-12 (max-norm relative to the largest entry),
FP32 Jacobian action <= 1e-5 (2-norm); solutions <= 1e-8 (FP64 at a 1e-11
stopping rule) and <= 1e-6 (mixed).
"""

import numpy as np
import pytest

import synthetic as syn
from oracle import fem, newton, precond
from tests.gpu_common import MU, assert_fp32_entrywise, relmax, relnorm, row_magnitude, smooth_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402


def _t(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _setup(nx, ny, nz, ratio, be, tau):
    mesh = syn.cook_mesh(nx, ny, nz)
    P = fem.cook_problem(mesh, mu=MU, lam=ratio * MU, tau=tau, follower=True)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, ratio * MU, tau, block_size=be, follower=True)
    return mesh, P, ctx


@pytest.mark.parametrize("grid,be", [((6, 5, 2, 5.0), 64), ((12, 10, 3, 50.0), 512)])
def test_follower_kernels_parity(grid, be):
    mesh, P, ctx = _setup(*grid, be=be, tau=4.0)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=91, amp=0.05))
    for s in (0.3, 1.0):
        nl.nle_set_load_scale(ctx, s)
        r = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
        rn = nl.nle_residual(ctx, _t(u), r)
        ref = P.residual(u, s)
        assert relmax(r.cpu().numpy(), ref) < 1e-12, s
        assert abs(rn - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    s = 0.8
    nl.nle_set_load_scale(ctx, s)
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    nl.nle_set_load_scale(ctx, 0.2)  # the Jacobian keeps the linearization's load scale
    K = P.stiffness(u, load_scale=s)
    v = syn.random_field(P.n_dofs, 1.0, seed=92)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_jv(ctx, _t(v), y, nl.NLE_FP64)
    assert relmax(y.cpu().numpy(), K @ v) < 1e-12
    y32 = torch.empty(P.n_dofs, dtype=torch.float32, device="cuda")
    nl.nle_jv(ctx, _t(v, torch.float32), y32, nl.NLE_FP32)
    assert relnorm(y32.double().cpu().numpy(), K @ v) < 1e-5
    assert_fp32_entrywise(y32.cpu().numpy(), K @ v, row_magnitude(K, v, P, u),
                          dir_dofs=P.ddofs, v=v)
    d = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_diag(ctx, d)
    assert relmax(d.cpu().numpy(), K.diagonal()) < 1e-12
    b = torch.empty(6 * mesh.n_nodes, dtype=torch.float64, device="cuda")
    nl.nle_block_diag(ctx, b)
    B = precond.node_blocks(K, mesh.n_nodes)
    ref6 = np.stack([B[:, 0, 0], B[:, 1, 1], B[:, 2, 2], B[:, 0, 1], B[:, 1, 2], B[:, 0, 2]], 1)
    assert relmax(b.cpu().numpy().reshape(-1, 6), ref6) < 1e-12
    # the follower load makes the tangent non-symmetric
    w = syn.random_field(P.n_dofs, 1.0, seed=93)
    w[P.fixed] = 0.0
    v2 = v.copy()
    v2[P.fixed] = 0.0
    yw, yv = torch.empty_like(y), torch.empty_like(y)
    nl.nle_jv(ctx, _t(w), yw, nl.NLE_FP64)
    nl.nle_jv(ctx, _t(v2), yv, nl.NLE_FP64)
    asym = abs(float(v2 @ yw.cpu().numpy()) - float(w @ yv.cpu().numpy()))
    assert asym > 1e-9 * np.linalg.norm(v2) * np.linalg.norm(yw.cpu().numpy())
    with pytest.raises(nl.NleError) as e:
        nl.nle_energy(ctx, _t(u))
    assert e.value.status == nl.NLE_E_UNSUPPORTED


SOLVES = [
    ("nk", "fp64", {"ksp": "gmres", "orth": "mgs"}),
    ("ink", "mixed", {"ksp": "gmres", "orth": "cgs2"}),
    ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10, "ksp": "gmres", "h0_refresh": 10}),
]


@pytest.mark.parametrize("method,prec,kw", SOLVES)
def test_follower_cook_solves_match_oracle(method, prec, kw):
    mesh, P, ctx = _setup(8, 8, 1, 5.0, be=64, tau=2.0)
    scales = [0.5, 1.0]
    ustar = newton.solve_schedule(P, scales)[0]
    Pd = fem.cook_problem(mesh, mu=MU, lam=5.0 * MU, tau=2.0)
    udead = newton.solve_schedule(Pd, scales)[0]
    assert relnorm(ustar, udead) > 1e-3  # the follower load changes the answer
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    opts = problems.make_opts(method, prec, **dict(kw))
    tight = prec == "fp64"
    if tight:
        opts.snes_rtol = 1e-11
    reps = problems.solve_schedule(ctx, u, method, opts, scales)
    assert problems.schedule_ok(reps, scales), [(r["load_scale"], r["status_name"]) for r in reps]
    assert relnorm(u.cpu().numpy(), ustar) <= (1e-8 if tight else 1e-6)
