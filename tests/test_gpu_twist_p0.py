"""GPU parity of the paper's own twist statement (Sec. 4 "Twist test"): the
polyconvex law M5 (alpha_p = beta_p = alpha_s = beta_s = 9000) on the
inf-sup stable pair quadratic displacement / one pressure per element
(P2-P0), and the lower block-triangular Schur preconditioners of App. B
(lumped pressure mass, or SIMPLE), against the FP64 oracle (oracle/mixed.py,
oracle/precond.py).

Tolerances: kernels and preconditioner applications FP64 <= 1e-12
(max-norm relative to the largest entry); FP32 Jacobian action entry by
entry against 64 eps32 (|K||v|)_i; rotation-schedule solves against the
oracle's exact-Newton roots, <= 1e-8 (FP64 at a 1e-10 stopping rule) and
<= 1e-6 (mixed), displacement and pressure separately.
"""

import math

import numpy as np
import pytest

import synthetic as syn
from oracle import mixed, newton, precond
from tests.gpu_common import assert_fp32_entrywise, relmax, relnorm, row_magnitude

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402


def _t(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _setup(n, theta):
    mesh = syn.twist_p2_mesh(n)
    P = mixed.twist_problem_p0(mesh, theta)
    ctx = nl.Context(0)
    problems.setup_twist_p0(ctx, mesh)
    dofs, vals = syn.twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], theta)
    nl.nle_set_dirichlet(ctx, dofs, vals)
    return mesh, P, ctx


def _state(P, seed, amp=0.03):
    rng = np.random.default_rng(seed)
    A = amp * rng.standard_normal((3, 3))
    u = (P.X @ A.T).reshape(-1) + 0.002 * rng.standard_normal(3 * P.n_u)
    p = 2000.0 * rng.standard_normal(P.n_p)
    return P.lift(np.concatenate([u, p]))


@pytest.mark.parametrize("n", [1, 3])
def test_p0_m5_kernels_parity(n):
    mesh, P, ctx = _setup(n, math.radians(20))
    x = _state(P, seed=80 + n)
    assert ctx.n_dofs == P.n_dofs == 3 * P.n_u + P.conn.shape[0]
    r = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    rn = nl.nle_residual(ctx, _t(x), r)
    ref = P.residual(x)
    assert relmax(r.cpu().numpy(), ref) < 1e-12
    assert abs(rn - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    pi = nl.nle_energy(ctx, _t(x))
    assert abs(pi - P.energy(x)) <= 1e-11 * max(1.0, abs(P.energy(x)))
    K = P.stiffness(x)
    v = syn.random_field(P.n_dofs, 1.0, seed=90 + n)
    nl.nle_linearize(ctx, _t(x), nl.NLE_FP32)
    y = torch.empty_like(r)
    nl.nle_jv(ctx, _t(v), y, nl.NLE_FP64)
    assert relmax(y.cpu().numpy(), K @ v) < 1e-12
    y32 = torch.empty(P.n_dofs, dtype=torch.float32, device="cuda")
    nl.nle_jv(ctx, _t(v, torch.float32), y32, nl.NLE_FP32)
    assert_fp32_entrywise(y32.cpu().numpy(), K @ v, row_magnitude(K, v))
    d = torch.empty_like(r)
    nl.nle_diag(ctx, d)
    nu = 3 * P.n_u
    dh = d.cpu().numpy()
    assert relmax(dh[:nu], K.diagonal()[:nu]) < 1e-12
    assert relmax(dh[nu:], P.pressure_mass_lumped() / P.mu_eff) < 1e-14


def test_simple_diagonal_and_schur_applications_parity():
    mesh, P, ctx = _setup(3, math.radians(15))
    x = _state(P, seed=85)
    K = P.stiffness(x)
    nu = 3 * P.n_u
    nl.nle_linearize(ctx, _t(x), nl.NLE_FP32)
    s = torch.empty(P.conn.shape[0], dtype=torch.float64, device="cuda")
    nl.nle_simple_diag(ctx, s)
    s_ref = precond.simple_schur_diagonal(K, nu)
    assert relmax(s.cpu().numpy(), s_ref) < 1e-12
    dA = K.diagonal()[:nu]
    b = syn.random_field(P.n_dofs, 1.0, seed=86)
    mass = P.pressure_mass_lumped() / P.mu_eff
    for schur, sd in ((nl.NLE_SCHUR_LOWER_SIMPLE, s_ref), (nl.NLE_SCHUR_LOWER_MASS, mass)):
        ref = precond.schur_lower_apply(K, nu, b, lambda ru: ru / dA, sd)
        y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
        nl.nle_schur_apply(ctx, nl.NLE_PC_JACOBI, schur, _t(b), y)
        assert relmax(y.cpu().numpy(), ref) < 1e-12, schur
        y32 = torch.empty(P.n_dofs, dtype=torch.float32, device="cuda")
        nl.nle_schur_apply(ctx, nl.NLE_PC_JACOBI, schur, _t(b, torch.float32), y32, nl.NLE_FP32)
        assert relnorm(y32.double().cpu().numpy(), ref) < 1e-5, schur
    # refusals: in place, SIMPLE on the linear-pressure pair, no pressure field
    with pytest.raises(nl.NleError):
        nl.nle_schur_apply(ctx, nl.NLE_PC_JACOBI, nl.NLE_SCHUR_LOWER_MASS, y, y)
    m1 = syn.twist_p2_mesh(1)
    ctx1 = nl.Context(0)
    problems.setup_twist(ctx1, m1, 1.0)
    z = torch.zeros(ctx1.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_linearize(ctx1, z, nl.NLE_FP64)
    with pytest.raises(nl.NleError) as e:
        nl.nle_schur_apply(ctx1, nl.NLE_PC_JACOBI, nl.NLE_SCHUR_LOWER_SIMPLE, z, z.clone())
    assert e.value.status == nl.NLE_E_UNSUPPORTED
    with pytest.raises(nl.NleError) as e:  # the lower forms need GMRES
        nl.nle_solve_nk(ctx1, z, problems.make_opts("nk", ksp="minres",
                                                    schur=nl.NLE_SCHUR_LOWER_MASS))
    assert e.value.status == nl.NLE_E_UNSUPPORTED


ANGLES = [math.radians(10 * s) for s in range(1, 10)]

SOLVES = [
    ("nk", "fp64", {"ksp": "gmres", "schur": nl.NLE_SCHUR_LOWER_SIMPLE, "snes_rtol": 1e-10,
                    "ksp_atol": 1e-14}),
    ("ink", "mixed", {"ksp": "gmres", "schur": nl.NLE_SCHUR_LOWER_SIMPLE}),
    ("ink", "mixed", {"ksp": "gmres", "schur": nl.NLE_SCHUR_LOWER_MASS}),
    ("ink", "mixed", {"ksp": "minres"}),
    ("ink", "fp64", {"ksp": "gmres", "schur": nl.NLE_SCHUR_LOWER_SIMPLE, "pc": "amg",
                     "snes_rtol": 1e-10}),
]


@pytest.mark.parametrize("n", [2, 6])
@pytest.mark.parametrize("method,prec,kw", SOLVES)
def test_p0_twist_schedule_matches_oracle(method, prec, kw, n):
    mesh = syn.twist_p2_mesh(n)
    P = mixed.twist_problem_p0(mesh, 0.0)
    if n == 6:  # stored by tests/golden/make_golden.py
        import os

        xs = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                  "twist6_p0.npy"))
    else:
        xs = np.zeros(P.n_dofs)
        for th in ANGLES:
            mixed.set_twist_angle(P, mesh, th)
            xs, _ = newton.newton_exact(P, xs, 1.0)
    ctx = nl.Context(0)
    problems.setup_twist_p0(ctx, mesh)
    opts = problems.make_opts(method, prec, **dict(kw))
    x = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_twist(
        ctx, x, method, opts, ANGLES,
        lambda th: syn.twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], th))
    assert problems.twist_ok(reps, ANGLES), [(r["theta"], r["status_name"]) for r in reps]
    xh = x.cpu().numpy()
    nu = 3 * P.n_u
    tol = 1e-8 if prec == "fp64" else 1e-6
    assert relnorm(xh[:nu], xs[:nu]) <= tol
    assert relnorm(xh[nu:], xs[nu:]) <= tol * 10
