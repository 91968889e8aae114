"""GPU parity of the implicit time step's inertia (row-sum lumped P1 mass,
Newmark's average-acceleration rule; the heartbeat of Sec. 4 as a dynamic
problem) against the FP64 oracle: residual, Jacobian action (FP64, FP32),
diagonal, nodal blocks and incremental potential with inertia on the Cook and
cardiac meshes; the Newmark predictor and corrector; and a few dynamic
heartbeat steps against the oracle's exact-Newton time stepping.

Tolerances: kernels FP64 <= 1e-12 (max-norm relative to the largest entry),
FP32 Jacobian action <= 1e-5 (2-norm); Newmark vectors <= 1e-14 (elementwise
arithmetic); trajectories <= 1e-8 (FP64 at a 1e-11 stopping rule) and
<= 1e-6 (mixed) relative 2-norm.
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

C = syn.CARDIAC
RHO = 1e-7  # moves the 5-step cardiac trajectory ~20% away from the quasi-static one
BETA, GAMMA = 0.25, 0.5
# epicardial dashpots: move the 5-step damped trajectory ~11% from the undamped one
C_PERP, C_PAR = 2e-5, 2e-6


def _t(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _cook(be):
    mesh = syn.cook_mesh(12, 10, 3)
    P = fem.cook_problem(mesh, mu=MU, lam=50.0 * MU, tau=4.0)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, 50.0 * MU, 4.0, block_size=be)
    return mesh, P, ctx


def _cardiac(be):
    mesh = syn.shell_mesh(2, 6, 12)
    P = fem.cardiac_problem(mesh, C, gamma=0.03)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=be)
    nl.nle_set_active_tension(ctx, 0.03)
    return mesh, P, ctx


def _check_kernels(mesh, P, ctx, u, s, rho, coef, energy):
    ut = P.lift(smooth_state(mesh, P.n_dofs, seed=71, amp=0.03))
    P.set_inertia(rho, coef, ut)
    nl.nle_set_inertia(ctx, rho, coef, _t(ut))
    nl.nle_set_load_scale(ctx, s)
    r = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    rn = nl.nle_residual(ctx, _t(u), r)
    ref = P.residual(u, s)
    assert relmax(r.cpu().numpy(), ref) < 1e-12
    assert abs(rn - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    K = P.stiffness(u, load_scale=s)
    v = syn.random_field(P.n_dofs, 1.0, seed=72)
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
    if energy:
        e = nl.nle_energy(ctx, _t(u))
        eref = P.energy(u, s)
        assert abs(e - eref) <= 1e-12 * abs(eref)
    # switching the term off restores the quasi-static operators
    P.set_inertia(0.0, 0.0, ut)
    nl.nle_set_inertia(ctx, 0.0, 0.0, None)
    nl.nle_residual(ctx, _t(u), r)
    assert relmax(r.cpu().numpy(), P.residual(u, s)) < 1e-12


@pytest.mark.parametrize("be", [64, 512])
def test_inertia_kernels_cook(be):
    mesh, P, ctx = _cook(be)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=70, amp=0.05))
    # c m comparable with the stiffness: the inertia term is not a rounding-level change
    _check_kernels(mesh, P, ctx, u, 0.7, 2e-3, 1.0 / (BETA * 0.05 ** 2), energy=True)


def test_inertia_kernels_cardiac():
    mesh, P, ctx = _cardiac(128)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=73, amp=0.02))
    _check_kernels(mesh, P, ctx, u, 0.6, RHO, 1.0 / (BETA * C["dt"] ** 2), energy=False)


def test_newmark_vectors():
    mesh, P, ctx = _cook(512)
    rng = np.random.default_rng(74)
    u, v, a, un = (rng.standard_normal(P.n_dofs) for _ in range(4))
    dt = 0.013
    ut = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    vt = torch.empty_like(ut)
    nl.nle_newmark_predict(ctx, dt, BETA, _t(u), _t(v), _t(a), ut, gamma=GAMMA, v_tilde=vt)
    ut_ref = newton.newmark_predict(u, v, a, dt, BETA)
    assert relmax(ut.cpu().numpy(), ut_ref) < 1e-14
    assert relmax(vt.cpu().numpy(), v + dt * (1.0 - GAMMA) * a) < 1e-14
    vd, ad = _t(v), _t(a)
    nl.nle_newmark_correct(ctx, dt, BETA, GAMMA, _t(un), ut, vd, ad)
    v_ref, a_ref = newton.newmark_correct(un, ut.cpu().numpy(), v, a, dt, BETA, GAMMA)
    assert relmax(vd.cpu().numpy(), v_ref) < 1e-14
    assert relmax(ad.cpu().numpy(), a_ref) < 1e-14


def test_inertia_usage_errors():
    mesh, P, ctx = _cook(512)
    z = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    for rho, coef in ((-1.0, 1.0), (1.0, -1.0), (float("nan"), 1.0), (1.0, float("inf"))):
        with pytest.raises(nl.NleError) as e:
            nl.nle_set_inertia(ctx, rho, coef, z)
        assert e.value.status == nl.NLE_E_INVAL
    with pytest.raises(nl.NleError) as e:
        nl.nle_set_inertia(ctx, 1.0, 1.0, None)
    assert e.value.status == nl.NLE_E_INVAL
    for dt, beta in ((0.0, 0.25), (0.1, 0.0)):
        with pytest.raises(nl.NleError) as e:
            nl.nle_newmark_predict(ctx, dt, beta, z, z, z, z)
        assert e.value.status == nl.NLE_E_INVAL
    m2 = syn.cook_p2_mesh(3, 3, 1)
    ctx2 = nl.Context(0)
    problems.setup_cook_p2(ctx2, m2, MU, 5.0 * MU)
    z2 = torch.zeros(ctx2.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NleError) as e:
        nl.nle_set_inertia(ctx2, 1.0, 1.0, z2)
    assert e.value.status == nl.NLE_E_UNSUPPORTED
    # a new mesh drops the inertia term
    nl.nle_set_inertia(ctx, 1e-3, 1e3, z)
    problems.setup_cook(ctx, mesh, MU, 50.0 * MU, 4.0, block_size=512)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=75, amp=0.05))
    r = torch.empty_like(z)
    nl.nle_residual(ctx, _t(u), r)
    assert relmax(r.cpu().numpy(), P.residual(u, 1.0)) < 1e-12


def test_dashpot_kernels_cardiac():
    mesh, P, ctx = _cardiac(128)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=76, amp=0.02))
    ut = P.lift(smooth_state(mesh, P.n_dofs, seed=77, amp=0.02))
    vt = syn.random_field(P.n_dofs, 0.05, seed=78)
    vt[P.fixed] = 0.0
    c, cv = 1.0 / (BETA * C["dt"] ** 2), GAMMA / (BETA * C["dt"])
    P.set_inertia(RHO, c, ut)
    P.set_robin_damping(C_PERP, C_PAR)
    P.set_step_velocity(cv, vt)
    nl.nle_set_inertia(ctx, RHO, c, _t(ut))
    nl.nle_set_robin_damping(ctx, C_PERP, C_PAR)
    nl.nle_set_step_velocity(ctx, cv, _t(vt))
    s = 0.6
    nl.nle_set_load_scale(ctx, s)
    r = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_residual(ctx, _t(u), r)
    ref = P.residual(u, s)
    assert relmax(r.cpu().numpy(), ref) < 1e-12
    # the dashpots change the residual well above rounding
    P.set_robin_damping(0.0, 0.0)
    assert relmax(P.residual(u, s), ref) > 1e-6
    P.set_robin_damping(C_PERP, C_PAR)
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    K = P.stiffness(u, load_scale=s)
    v = syn.random_field(P.n_dofs, 1.0, seed=79)
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
    with pytest.raises(nl.NleError) as e:
        nl.nle_set_robin_damping(ctx, -1.0, 0.0)
    assert e.value.status == nl.NLE_E_INVAL
    with pytest.raises(nl.NleError) as e:
        nl.nle_set_step_velocity(ctx, 1.0, None)
    assert e.value.status == nl.NLE_E_INVAL


N_STEPS = 5

DYN = [
    ("ink", "mixed", {}),
    ("nk", "fp64", {"snes_rtol": 1e-11, "ksp_atol": 1e-15}),
    ("bfgs", "fp64", {"h0": "ksp", "qn_m": 20, "h0_refresh": 20, "snes_rtol": 1e-11,
                      "ksp_atol": 1e-15, "pc": "bjacobi3"}),
]


@pytest.mark.parametrize("method,prec,kw", DYN)
def test_dynamic_heartbeat_matches_oracle(method, prec, kw):
    mesh = syn.shell_mesh(2, 6, 12)
    steps = syn.heartbeat_schedule()[:N_STEPS]
    P = fem.cardiac_problem(mesh, C)
    u_ref, v_ref, a_ref, _ = newton.solve_heartbeat_dynamic(P, steps, C["gamma_max"], RHO,
                                                            C["dt"], rtol=1e-13)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=128)
    opts = problems.make_opts(method, prec, ksp="gmres", restart=1000, **dict(kw))
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps, v, a = problems.solve_heartbeat_dynamic(ctx, u, method, opts, steps, C["gamma_max"],
                                                  RHO, C["dt"], BETA, GAMMA)
    assert problems.heartbeat_ok(reps, steps), [(r["t"], r["status_name"]) for r in reps]
    tol = 1e-8 if prec == "fp64" else 1e-6
    for got, ref in ((u, u_ref), (v, v_ref), (a, a_ref)):
        err = relnorm(got.cpu().numpy(), ref)
        assert err <= tol, err
    # the inertia is off again: the residual is the quasi-static one
    r = torch.empty_like(u)
    nl.nle_set_load_scale(ctx, steps[-1][1])
    nl.nle_residual(ctx, u, r)
    fem.set_active_tension(P, C["gamma_max"] * steps[-1][1])
    # the quasi-static residual of a dynamic state is the inertia force that
    # the step left, a difference of much larger element forces: rounding
    # sits near 1e-11 of it, while a leftover inertia term would be O(1)
    assert relmax(r.cpu().numpy(), P.residual(u.cpu().numpy(), steps[-1][1])) < 1e-9


@pytest.mark.parametrize("method,prec,kw", DYN[:2])
def test_damped_dynamic_heartbeat_matches_oracle(method, prec, kw):
    mesh = syn.shell_mesh(2, 6, 12)
    steps = syn.heartbeat_schedule()[:N_STEPS]
    P = fem.cardiac_problem(mesh, C)
    P.set_robin_damping(C_PERP, C_PAR)
    u_ref, v_ref, a_ref, _ = newton.solve_heartbeat_dynamic(P, steps, C["gamma_max"], RHO,
                                                            C["dt"], rtol=1e-13)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=128)
    nl.nle_set_robin_damping(ctx, C_PERP, C_PAR)
    opts = problems.make_opts(method, prec, ksp="gmres", restart=1000, **dict(kw))
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps, v, a = problems.solve_heartbeat_dynamic(ctx, u, method, opts, steps, C["gamma_max"],
                                                  RHO, C["dt"], BETA, GAMMA)
    assert problems.heartbeat_ok(reps, steps), [(r["t"], r["status_name"]) for r in reps]
    tol = 1e-8 if prec == "fp64" else 1e-6
    for got, ref in ((u, u_ref), (v, v_ref), (a, a_ref)):
        err = relnorm(got.cpu().numpy(), ref)
        assert err <= tol, err
