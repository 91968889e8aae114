"""GPU parity of the aggregation multigrid preconditioner (NLE_PC_AMG; the
AMG of Sec. 4 and App. A with the construction fixed in oracle/amg.py)
against the FP64 oracle: the hierarchy's level sizes, one V-cycle applied to
seeded vectors on Cook (symmetric tangent), the follower-traction Cook and the
cardiac shell (nonsymmetric), the shell with an implicit step's inertia and
dashpots, the quadratic Cook mesh and the twist's field split, GMRES iteration counts of an NK
solve against the oracle's loop with the same cycle, and solves (NK, iNK
mixed, BFGS-preonly with the cycle as H0, a heartbeat step) against the
oracle's roots.

Tolerances.  The FP64 cycle differs from the oracle's by rounding in the
Galerkin products and in the coarsest solve (a dense inverse on the GPU
side, an LU solve in the oracle), amplified by the coarsest operator's
condition number: 1e-10 relative max-norm.  The FP32 cycle rounds every
level's operator and the coarsest inverse to FP32: 1e-3 relative 2-norm.
Solutions: <= 1e-8 (FP64 at a 1e-11 stopping rule), <= 1e-6 (mixed).
"""

import numpy as np
import pytest

import synthetic as syn
from oracle import amg, fem, newton, solvers
from tests.gpu_common import MU, relmax, relnorm, smooth_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402

C = syn.CARDIAC


def _t(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _cook(nx, ny, nz, ratio=5.0, be=512, tau=1.0):
    mesh = syn.cook_mesh(nx, ny, nz)
    P = fem.cook_problem(mesh, mu=MU, lam=ratio * MU, tau=tau)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, ratio * MU, tau, block_size=be)
    return mesh, P, ctx


def _cycle_parity(mesh, P, ctx, u, s, seed):
    nl.nle_set_load_scale(ctx, s)
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    K = P.stiffness(u, load_scale=s)
    H = amg.setup(K, mesh.X, mesh.conn, P.fixed)
    b = syn.random_field(P.n_dofs, 1.0, seed=seed)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, _t(b), y, nl.NLE_FP64)
    assert nl.nle_amg_levels(ctx) == [A.shape[0] for A in H.A]
    ref = amg.vcycle(H, b)
    assert relmax(y.cpu().numpy(), ref) < 1e-10
    y32 = torch.empty(P.n_dofs, dtype=torch.float32, device="cuda")
    nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, _t(b, torch.float32), y32, nl.NLE_FP32)
    assert relnorm(y32.double().cpu().numpy(), ref) < 1e-3
    # the same cycle twice: bitwise repeatable
    y2 = torch.empty_like(y)
    nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, _t(b), y2, nl.NLE_FP64)
    assert torch.equal(y, y2)
    return H


@pytest.mark.parametrize("grid,be", [((16, 16, 2), 512), ((24, 20, 3), 128)])
def test_cycle_parity_cook(grid, be):
    mesh, P, ctx = _cook(*grid, be=be, tau=4.0)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=81, amp=0.03))
    H = _cycle_parity(mesh, P, ctx, u, 0.8, seed=82)
    assert H.n_levels >= 2


def test_cycle_parity_cardiac():
    mesh = syn.shell_mesh(2, 8, 16)
    P = fem.cardiac_problem(mesh, C, gamma=0.03)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=128)
    nl.nle_set_active_tension(ctx, 0.03)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=83, amp=0.02))
    _cycle_parity(mesh, P, ctx, u, 0.7, seed=84)


def test_cycle_parity_p2_cook():
    # quadratic displacement tetrahedra: the node graph takes all ten nodes
    from oracle import p2
    mesh = syn.cook_p2_mesh(8, 6, 2)
    P = p2.cook_p2_problem(mesh, mu=MU, lam=5.0 * MU, tau=2.0)
    ctx = nl.Context(0)
    problems.setup_cook_p2(ctx, mesh, MU, 5.0 * MU, 2.0)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=87, amp=0.03))
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    K = P.stiffness(u)
    H = amg.setup(K, mesh.X, mesh.conn, P.fixed)
    assert H.n_levels >= 2
    b = syn.random_field(P.n_dofs, 1.0, seed=88)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, _t(b), y, nl.NLE_FP64)
    assert nl.nle_amg_levels(ctx) == [A.shape[0] for A in H.A]
    assert relmax(y.cpu().numpy(), amg.vcycle(H, b)) < 1e-10
    # and a solve with CG and the cycle against the oracle root
    ustar, _ = newton.newton_exact(P, np.zeros(P.n_dofs), 1.0)
    z = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    st, rep = nl.nle_solve_nk(ctx, z, problems.make_opts(
        "nk", ksp="cg", pc="amg", snes_rtol=1e-11, ksp_atol=1e-15))
    assert st == nl.NLE_OK, rep
    assert relnorm(z.cpu().numpy(), ustar) <= 1e-8


def test_field_split_cycle_parity_twist():
    # displacement-pressure mesh: the cycle on the displacement block of the
    # tangent, the pressure entries scaled by the inverse lumped mass over mu
    from oracle import mixed
    mesh = syn.twist_p2_mesh(3)
    P = mixed.twist_problem(mesh, 1.0, 0.1)
    ctx = nl.Context(0)
    problems.setup_twist(ctx, mesh, 1.0)
    dofs, vals = syn.twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], 0.1)
    nl.nle_set_dirichlet(ctx, dofs, vals)
    rng = np.random.default_rng(89)
    x = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    nl.nle_linearize(ctx, _t(x), nl.NLE_FP32)
    nu = 3 * P.n_u
    K = P.stiffness(x).tocsr()
    H = amg.setup(K[:nu, :nu], mesh.X, mesh.conn, P.fixed[:nu])
    assert H.n_levels >= 2
    v = syn.random_field(P.n_dofs, 1.0, seed=90)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, _t(v), y, nl.NLE_FP64)
    assert nl.nle_amg_levels(ctx) == [A.shape[0] for A in H.A]
    ref = np.concatenate([amg.vcycle(H, v[:nu]), v[nu:] / (P.pressure_mass_lumped() / 1.0)])
    assert relmax(y.cpu().numpy()[:nu], ref[:nu]) < 1e-10
    assert relmax(y.cpu().numpy()[nu:], ref[nu:]) < 1e-12


def test_twist_schedule_with_field_split():
    import math
    from oracle import mixed
    mesh = syn.twist_p2_mesh(2)
    angles = [math.radians(10 * s) for s in range(1, 4)]
    P = mixed.twist_problem(mesh, 1.0, 0.0)
    xs = np.zeros(P.n_dofs)
    for th in angles:
        mixed.set_twist_angle(P, mesh, th)
        xs, _ = newton.newton_exact(P, xs, 1.0)
    ctx = nl.Context(0)
    problems.setup_twist(ctx, mesh, 1.0)
    opts = problems.make_opts("nk", "fp64", ksp="gmres", pc="amg", restart=1000,
                              snes_rtol=1e-10, ksp_atol=1e-14)
    x = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_twist(
        ctx, x, "nk", opts, angles,
        lambda th: syn.twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], th))
    assert problems.twist_ok(reps, angles), [(r["theta"], r["status_name"]) for r in reps]
    xh = x.cpu().numpy()
    nu = 3 * P.n_u
    assert relnorm(xh[:nu], xs[:nu]) <= 1e-8
    assert relnorm(xh[nu:], xs[nu:]) <= 1e-8


def test_cycle_parity_follower_cook():
    # the follower traction makes the tangent nonsymmetric
    mesh = syn.cook_mesh(16, 12, 2)
    P = fem.cook_problem(mesh, mu=MU, lam=5.0 * MU, tau=4.0, follower=True)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, 5.0 * MU, 4.0, block_size=256, follower=True)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=91, amp=0.03))
    H = _cycle_parity(mesh, P, ctx, u, 0.9, seed=92)
    assert H.n_levels >= 2


def test_cycle_parity_with_inertia_and_dashpots():
    # an implicit heartbeat step: lumped-mass inertia and epicardial dashpots
    # enter the tangent the hierarchy is built from
    mesh = syn.shell_mesh(2, 8, 16)
    P = fem.cardiac_problem(mesh, C, gamma=0.03)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=128)
    nl.nle_set_active_tension(ctx, 0.03)
    rho, dt, beta, gamma = 1e-7, C["dt"], 0.25, 0.5
    c, cv = 1.0 / (beta * dt * dt), gamma / (beta * dt)
    ut = P.lift(smooth_state(mesh, P.n_dofs, seed=93, amp=0.02))
    vt = syn.random_field(P.n_dofs, 0.05, seed=94)
    vt[P.fixed] = 0.0
    P.set_inertia(rho, c, ut)
    P.set_robin_damping(2e-5, 2e-6)
    P.set_step_velocity(cv, vt)
    nl.nle_set_inertia(ctx, rho, c, _t(ut))
    nl.nle_set_robin_damping(ctx, 2e-5, 2e-6)
    nl.nle_set_step_velocity(ctx, cv, _t(vt))
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=95, amp=0.02))
    _cycle_parity(mesh, P, ctx, u, 0.5, seed=96)


def test_one_level_hierarchy_is_the_exact_solve():
    mesh, P, ctx = _cook(4, 4, 1)  # 150 unknowns: below the coarsening threshold
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=85, amp=0.03))
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP64)
    b = syn.random_field(P.n_dofs, 1.0, seed=86)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, _t(b), y, nl.NLE_FP64)
    assert nl.nle_amg_levels(ctx) == [P.n_dofs]
    K = P.stiffness(u)
    assert relmax(y.cpu().numpy(), np.linalg.solve(K.toarray(), b)) < 1e-10


def test_nk_gmres_counts_follow_oracle_loop():
    mesh, P, ctx = _cook(16, 16, 2, tau=2.0)

    def lin(u):
        K = P.stiffness(u)
        H = amg.setup(K, mesh.X, mesh.conn, P.fixed)
        return (lambda v: K @ v), (lambda v: amg.vcycle(H, v))

    ref = solvers.newton_krylov(lambda u: P.residual(u), lin, np.zeros(P.n_dofs), inexact=False)
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    st, rep = nl.nle_solve_nk(ctx, u, problems.make_opts("nk", ksp="gmres", pc="amg"))
    assert st == nl.NLE_OK, rep
    assert abs(rep["nit"] - ref["nit"]) <= 1
    assert all(abs(a - b) <= 2 for a, b in zip(rep["lit_hist"], ref["lits"])), (
        rep["lit_hist"], ref["lits"])
    # far fewer Krylov iterations than with point Jacobi
    u2 = torch.zeros_like(u)
    st, rep2 = nl.nle_solve_nk(ctx, u2, problems.make_opts("nk", ksp="gmres"))
    assert st == nl.NLE_OK
    assert 3 * rep["lit_total"] < rep2["lit_total"], (rep["lit_total"], rep2["lit_total"])


def test_nk_cg_counts_follow_oracle_loop():
    # the cycle is symmetric for the symmetric dead-load tangent: CG with it
    mesh, P, ctx = _cook(16, 16, 2, tau=2.0)

    def lin(u):
        K = P.stiffness(u)
        H = amg.setup(K, mesh.X, mesh.conn, P.fixed)
        return (lambda v: K @ v), (lambda v: amg.vcycle(H, v))

    ref = solvers.newton_krylov(lambda u: P.residual(u), lin, np.zeros(P.n_dofs), ksp="cg")
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    o = problems.make_opts("nk", ksp="cg", pc="amg")
    o.check_every = 4
    st, rep = nl.nle_solve_nk(ctx, u, o)
    assert st == nl.NLE_OK, rep
    assert abs(rep["nit"] - ref["nit"]) <= 1
    for a, b in zip(rep["lit_hist"], ref["lits"]):
        assert abs(a - b) <= max(2, 0.02 * b), (rep["lit_hist"], ref["lits"])


def test_nk_minres_counts_follow_oracle_loop():
    # MINRES with the cycle as its (symmetric positive definite) preconditioner
    mesh, P, ctx = _cook(16, 16, 2, tau=2.0)

    def lin(u):
        K = P.stiffness(u)
        H = amg.setup(K, mesh.X, mesh.conn, P.fixed)
        return (lambda v: K @ v), (lambda v: amg.vcycle(H, v))

    ref = solvers.newton_krylov(lambda u: P.residual(u), lin, np.zeros(P.n_dofs), ksp="minres")
    for prec in ("fp64", "mixed"):
        u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
        o = problems.make_opts("nk", prec, ksp="minres", pc="amg")
        o.check_every = 4
        st, rep = nl.nle_solve_nk(ctx, u, o)
        assert st == nl.NLE_OK, rep
        assert abs(rep["nit"] - ref["nit"]) <= 1
        if prec == "fp64":
            for a, b in zip(rep["lit_hist"], ref["lits"]):
                assert abs(a - b) <= max(2, 0.02 * b), (rep["lit_hist"], ref["lits"])


SOLVES = [
    ("nk", "fp64", {"snes_rtol": 1e-11, "ksp_atol": 1e-15}),
    ("nk", "fp64", {"snes_rtol": 1e-11, "ksp_atol": 1e-15, "ksp": "minres"}),
    ("ink", "mixed", {"ksp": "minres"}),
    ("nk", "fp64", {"snes_rtol": 1e-11, "ksp_atol": 1e-15, "ksp": "cg"}),
    ("ink", "mixed", {}),
    ("ink", "mixed", {"ksp": "cg"}),
    ("bfgs", "fp64", {"h0": "preonly", "qn_m": 20, "snes_rtol": 1e-11, "snes_max_it": 400}),
]


@pytest.mark.parametrize("method,prec,kw", SOLVES)
def test_cook_solves_match_oracle_root(method, prec, kw):
    mesh, P, ctx = _cook(16, 16, 2, tau=2.0)
    ustar, _ = newton.newton_exact(P, np.zeros(P.n_dofs), 1.0)
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    st, rep = problems.SOLVERS[method](ctx, u, problems.make_opts(
        method, prec, **{"ksp": "gmres", "pc": "amg", **kw}))
    assert st == nl.NLE_OK, rep
    err = relnorm(u.cpu().numpy(), ustar)
    assert err <= (1e-8 if prec == "fp64" else 1e-6), err


def test_heartbeat_steps_with_multigrid():
    mesh = syn.shell_mesh(2, 6, 12)
    steps = syn.heartbeat_schedule()[:3]
    P = fem.cardiac_problem(mesh, C)
    ustar = newton.solve_heartbeat(P, steps, C["gamma_max"])[0]
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=128)
    opts = problems.make_opts("ink", "mixed", ksp="gmres", pc="amg", restart=1000)
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_heartbeat(ctx, u, "ink", opts, steps, C["gamma_max"])
    assert problems.heartbeat_ok(reps, steps), [(r["t"], r["status_name"]) for r in reps]
    assert relnorm(u.cpu().numpy(), ustar) <= 1e-6


def test_multigrid_usage_errors():
    mesh, P, ctx = _cook(8, 8, 1)
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_linearize(ctx, u, nl.NLE_FP64)
    with pytest.raises(nl.NleError) as e:
        nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, u, u, nl.NLE_FP64)
    assert e.value.status == nl.NLE_E_INVAL
    # with a pressure field the field split runs with GMRES only
    mt = syn.twist_p2_mesh(2)
    ctx2 = nl.Context(0)
    problems.setup_twist(ctx2, mt, 1.0)
    z2 = torch.zeros(ctx2.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NleError) as e:
        nl.nle_solve_nk(ctx2, z2, problems.make_opts("nk", ksp="cg", pc="amg"))
    assert e.value.status == nl.NLE_E_UNSUPPORTED
    # a new Dirichlet set rebuilds the hierarchy
    y = torch.empty_like(u)
    nl.nle_pc_apply(ctx, nl.NLE_PC_AMG, torch.ones_like(u), y, nl.NLE_FP64)
    nl.nle_set_dirichlet(ctx, np.arange(6), np.zeros(6))
    assert nl.nle_amg_levels(ctx) == []
