"""GPU parity of the cardiac-like workload (Sec. 4, "Heartbeat test", with the
substitute law M4): element kernels with per-element fibres and active
tension, the follower endocardial pressure and the epicardial springs against
the FP64 oracle, and quasi-static heartbeat solves (NK / iNK with GMRES,
inexact BFGS) against the oracle's exact-Newton roots.

Tolerances: kernels FP64 <= 1e-12 (max-norm relative to the largest entry),
FP32 Jacobian action <= 1e-5 (2-norm); solutions <= 1e-6 (mixed) and
<= 1e-8 (FP64 at a 1e-10 stopping rule) relative 2-norm.
"""

import numpy as np
import pytest

import synthetic as syn
from oracle import fem, newton
from tests.gpu_common import assert_fp32_entrywise, relmax, relnorm, row_magnitude, smooth_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402

C = syn.CARDIAC
GRIDS = [((2, 6, 12), 512), ((2, 6, 12), 64), ((3, 8, 20), 200)]


def _setup(grid, be, gamma=0.0):
    mesh = syn.shell_mesh(*grid)
    P = fem.cardiac_problem(mesh, C, gamma=gamma)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=be)
    nl.nle_set_active_tension(ctx, gamma)
    return mesh, P, ctx


def _t(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


@pytest.mark.parametrize("grid,be", GRIDS)
def test_cardiac_residual_parity(grid, be):
    mesh, P, ctx = _setup(grid, be, gamma=0.04)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=41))
    for s in (0.0, 0.6, 1.0):
        nl.nle_set_load_scale(ctx, s)
        r = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
        rn = nl.nle_residual(ctx, _t(u), r)
        ref = P.residual(u, s)
        assert relmax(r.cpu().numpy(), ref) < 1e-12, s
        assert abs(rn - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("grid,be", GRIDS)
def test_cardiac_jacobian_action_and_diagonal_parity(grid, be):
    mesh, P, ctx = _setup(grid, be, gamma=0.03)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=42))
    v = syn.random_field(P.n_dofs, 1.0, seed=43)
    s = 0.8
    nl.nle_set_load_scale(ctx, s)
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    nl.nle_set_load_scale(ctx, 0.1)  # the Jacobian keeps the linearization's pressure
    ref = P.jv(u, v, load_scale=s)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_jv(ctx, _t(v), y, nl.NLE_FP64)
    assert relmax(y.cpu().numpy(), ref) < 1e-12
    y32 = torch.empty(P.n_dofs, dtype=torch.float32, device="cuda")
    nl.nle_jv(ctx, _t(v, torch.float32), y32, nl.NLE_FP32)
    assert relnorm(y32.double().cpu().numpy(), ref) < 1e-5
    assert_fp32_entrywise(y32.cpu().numpy(), ref,
                          row_magnitude(P.stiffness(u, load_scale=s), v, P, u),
                          dir_dofs=P.ddofs, v=v)
    d = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_diag(ctx, d)
    assert relmax(d.cpu().numpy(), P.diagonal(u, load_scale=s)) < 1e-12
    # the follower pressure makes the tangent non-symmetric
    w = syn.random_field(P.n_dofs, 1.0, seed=44)
    w[P.fixed] = 0.0
    v2 = v.copy()
    v2[P.fixed] = 0.0
    yw = torch.empty_like(y)
    yv = torch.empty_like(y)
    nl.nle_jv(ctx, _t(w), yw, nl.NLE_FP64)
    nl.nle_jv(ctx, _t(v2), yv, nl.NLE_FP64)
    a, b = float(v2 @ yw.cpu().numpy()), float(w @ yv.cpu().numpy())
    assert abs(a - b) > 1e-11 * abs(a)  # well above FP64 rounding of the dots
    assert abs(a - float(v2 @ (P.jv(u, w, load_scale=s)))) <= 1e-11 * abs(a)


def test_cardiac_potential_without_pressure():
    mesh, P, ctx = _setup((2, 6, 12), 64, gamma=0.05)
    nl.nle_set_pressure(ctx, np.zeros((0, 3), dtype=np.int32), 0.0)
    P.pressure_tri = None
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=45))
    pi = nl.nle_energy(ctx, _t(u))
    ref = P.energy(u)
    assert abs(pi - ref) <= 1e-12 * abs(ref)


def test_cardiac_usage_errors():
    mesh = syn.shell_mesh(2, 6, 12)
    ctx = nl.Context(0)
    nl.nle_upload_mesh(ctx, mesh.X, mesh.conn)
    nl.nle_set_material(ctx, nl.NLE_MAT_M4, [C["a"], C["b"], C["af"], C["bf"], C["kappa"]])
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    r = torch.empty_like(u)
    with pytest.raises(nl.NleError) as e:
        nl.nle_residual(ctx, u, r)  # fibres missing
    assert e.value.status == nl.NLE_E_STATE
    bad = mesh.elem_fibre * 2.0
    with pytest.raises(nl.NleError):
        nl.nle_set_fibres(ctx, bad)
    nl.nle_set_fibres(ctx, mesh.elem_fibre)
    nl.nle_set_pressure(ctx, mesh.faces["endo"], C["p_max"])
    with pytest.raises(nl.NleError) as e:
        nl.nle_energy(ctx, u)
    assert e.value.status == nl.NLE_E_UNSUPPORTED
    tri = mesh.faces["epi"].copy()
    tri[0, 0] = mesh.n_nodes
    with pytest.raises(nl.NleError):
        nl.nle_set_robin(ctx, tri, 1.0, 1.0)
    with pytest.raises(nl.NleError):
        nl.nle_set_material(ctx, nl.NLE_MAT_M4, [C["a"], C["b"], C["af"], C["bf"]])


N_STEPS = 5  # t = 0.02 .. 0.10 (activation rising to 0.71 of its peak)


def _oracle_root(mesh, steps):
    P = fem.cardiac_problem(mesh, C)
    return newton.solve_heartbeat(P, steps, C["gamma_max"])[0]


SOLVES = [
    ("ink", "mixed", {}),
    ("nk", "mixed", {}),
    # FP64 at a tighter stopping rule; the Krylov absolute tolerance is lowered
    # with it (App. A's 1e-10 would stop the linear solves above that rule)
    ("nk", "fp64", {"snes_rtol": 1e-10, "ksp_atol": 1e-14}),
    ("bfgs", "mixed", {"h0": "ksp", "qn_m": 10}),
]


@pytest.mark.parametrize("method,prec,kw", SOLVES)
def test_heartbeat_steps_match_oracle(method, prec, kw):
    mesh = syn.shell_mesh(2, 6, 12)
    steps = syn.heartbeat_schedule()[:N_STEPS]
    ustar = _oracle_root(mesh, steps)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh), block_size=128)
    # restart above the 756 dofs: full GMRES
    opts = problems.make_opts(method, prec, ksp="gmres", restart=1000, **dict(kw))
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_heartbeat(ctx, u, method, opts, steps, C["gamma_max"])
    assert problems.heartbeat_ok(reps, steps), [(r["t"], r["status_name"]) for r in reps]
    err = relnorm(u.cpu().numpy(), ustar)
    assert err <= (1e-8 if prec == "fp64" else 1e-6), err


def test_full_heartbeat_returns_to_rest():
    # all 20 steps with mixed iNK: at the last step the activation and the
    # pressure vanish and the oracle's root is the reference state
    mesh = syn.shell_mesh(2, 6, 12)
    steps = syn.heartbeat_schedule()
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh))
    opts = problems.make_opts("ink", "mixed", ksp="gmres", restart=1000)
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_heartbeat(ctx, u, "ink", opts, steps[:10], C["gamma_max"])
    assert problems.heartbeat_ok(reps, steps[:10])
    peak = u.cpu().numpy().copy()  # t = 0.2, peak activation
    reps = problems.solve_heartbeat(ctx, u, "ink", opts, steps[10:], C["gamma_max"],
                                    start=steps[9])
    assert problems.heartbeat_ok(reps, steps)
    ustar = _oracle_root(mesh, steps[:10])
    assert relnorm(peak, ustar) <= 1e-6
    assert float(u.abs().max()) <= 1e-6 * float(np.abs(ustar).max())


@pytest.mark.parametrize("method,prec,kw", [
    ("ink", "fp64", {"ksp": "cg", "pc": "amg", "snes_rtol": 1e-10, "ksp_atol": 1e-14}),
    ("ink", "mixed", {"ksp": "minres"}),
])
def test_heartbeat_4x20x64_to_peak_matches_stored_oracle_root(method, prec, kw):
    # the 4x20x64 shell (30,720 tets), 10 time steps to the activation peak,
    # against the oracle's root stored by tests/golden/make_golden.py
    import os

    ustar = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                 "heart4x20x64_peak.npy"))
    mesh = syn.shell_mesh(4, 20, 64)
    steps = syn.heartbeat_schedule()[:10]
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, C, syn.shell_dirichlet(mesh))
    opts = problems.make_opts(method, prec, **dict(kw))
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_heartbeat(ctx, u, method, opts, steps, C["gamma_max"])
    assert problems.heartbeat_ok(reps, steps), [(r["t"], r["status_name"]) for r in reps]
    err = relnorm(u.cpu().numpy(), ustar)
    assert err <= (1e-8 if prec == "fp64" else 1e-6), err


@pytest.mark.parametrize("method,prec,kw", [
    ("ink", "fp64", {"ksp": "cg", "pc": "amg", "snes_rtol": 1e-10, "ksp_atol": 1e-14}),
    ("ink", "mixed", {"ksp": "cg", "pc": "amg"}),
    ("nk", "fp64", {"ksp": "minres", "pc": "amg", "snes_rtol": 1e-10, "ksp_atol": 1e-14}),
])
def test_heartbeat_strong_pressure_symmetric_krylov_reaches_oracle_root(method, prec, kw):
    # 50 times the endocardial pressure and twice the activation, 10 steps to
    # the peak: the follower pressure's nonsymmetric part grows with p (at the
    # oracle's root ||K - K^T||_F / ||K||_F is about 4e-6, 40 times that of
    # the nominal load), and the shell's largest displacement triples.  CG and
    # MINRES, which assume a symmetric tangent, still bring every Newton step
    # to the FP64 rule, and the solution is the oracle's exact-Newton root.
    import scipy.sparse.linalg as sla

    c = dict(C)
    c["p_max"] = 50.0 * C["p_max"]
    c["gamma_max"] = 2.0 * C["gamma_max"]
    mesh = syn.shell_mesh(2, 6, 12)
    steps = syn.heartbeat_schedule()[:10]
    P = fem.cardiac_problem(mesh, c)
    ustar = newton.solve_heartbeat(P, steps, c["gamma_max"])[0]
    K = P.stiffness(ustar, load_scale=steps[-1][1])
    assert sla.norm(K - K.T) > 1e-6 * sla.norm(K)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, c, syn.shell_dirichlet(mesh), block_size=128)
    opts = problems.make_opts(method, prec, **dict(kw))
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_heartbeat(ctx, u, method, opts, steps, c["gamma_max"])
    assert problems.heartbeat_ok(reps, steps), [(r["t"], r["status_name"]) for r in reps]
    err = relnorm(u.cpu().numpy(), ustar)
    assert err <= (1e-8 if prec == "fp64" else 1e-6), err


# ---- the paper's Guccione law (M6) with the fibre / sheet frame ------------------
GUC = (0.1, 5.0, 2.0, 2.0, 1.0, 1.0, 1.0, 100.0)  # C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B


def _guc(block_size=128, gamma=0.03):
    mesh = syn.shell_mesh(2, 6, 12)
    P = fem.guccione_problem(mesh, C, GUC, gamma=gamma)
    ctx = nl.Context(0)
    problems.setup_guccione(ctx, mesh, C, GUC, syn.shell_dirichlet(mesh), block_size=block_size)
    nl.nle_set_active_tension(ctx, gamma)
    return mesh, P, ctx


@pytest.mark.parametrize("be", [64, 512])
def test_guccione_kernels_parity(be):
    mesh, P, ctx = _guc(be)
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=111, amp=0.03))
    for s in (0.0, 0.7):
        nl.nle_set_load_scale(ctx, s)
        r = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
        rn = nl.nle_residual(ctx, _t(u), r)
        ref = P.residual(u, s)
        assert relmax(r.cpu().numpy(), ref) < 1e-12
        assert abs(rn - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)
    s = 0.7
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    K = P.stiffness(u, load_scale=s)
    v = syn.random_field(P.n_dofs, 1.0, seed=112)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_jv(ctx, _t(v), y, nl.NLE_FP64)
    assert relmax(y.cpu().numpy(), K @ v) < 1e-12
    y32 = torch.empty(P.n_dofs, dtype=torch.float32, device="cuda")
    nl.nle_jv(ctx, _t(v, torch.float32), y32, nl.NLE_FP32)
    assert_fp32_entrywise(y32.cpu().numpy(), K @ v, row_magnitude(K, v, P, u),
                          dir_dofs=P.ddofs, v=v)
    d = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_diag(ctx, d)
    assert relmax(d.cpu().numpy(), K.diagonal()) < 1e-12
    # the potential without the follower pressure (springs, law and activation)
    ctx2 = nl.Context(0)
    nl.nle_upload_mesh(ctx2, mesh.X, mesh.conn)
    nl.nle_set_material(ctx2, nl.NLE_MAT_M6, list(GUC))
    nl.nle_set_fibre_frame(ctx2, mesh.elem_fibre, mesh.elem_sheet)
    nl.nle_set_active_tension(ctx2, 0.03)
    P2 = fem.Problem(mesh.X, mesh.conn, "M6", P.params, np.zeros(P.n_dofs), np.zeros(0, np.int64),
                     np.zeros(0))
    e = nl.nle_energy(ctx2, _t(u))
    assert abs(e - P2.energy(u)) <= 1e-11 * abs(P2.energy(u))
    # refusals: no sheets, block Jacobi
    ctx3 = nl.Context(0)
    nl.nle_upload_mesh(ctx3, mesh.X, mesh.conn)
    nl.nle_set_material(ctx3, nl.NLE_MAT_M6, list(GUC))
    nl.nle_set_fibres(ctx3, mesh.elem_fibre)
    with pytest.raises(nl.NleError) as er:
        nl.nle_residual(ctx3, _t(u), r)
    assert er.value.status == nl.NLE_E_STATE
    with pytest.raises(nl.NleError):
        nl.nle_set_fibre_frame(ctx3, mesh.elem_fibre, mesh.elem_fibre)  # not orthogonal
    with pytest.raises(nl.NleError) as er:
        nl.nle_block_diag(ctx, torch.empty(6 * mesh.n_nodes, dtype=torch.float64, device="cuda"))
    assert er.value.status == nl.NLE_E_UNSUPPORTED


@pytest.mark.parametrize("method,prec,kw", [
    ("ink", "mixed", {"ksp": "gmres", "restart": 1000}),
    ("nk", "fp64", {"ksp": "gmres", "restart": 1000, "snes_rtol": 1e-10, "ksp_atol": 1e-14}),
    ("bfgs", "mixed", {"ksp": "gmres", "restart": 1000, "h0": "ksp", "qn_m": 10}),
])
def test_guccione_heartbeat_steps_match_oracle(method, prec, kw):
    mesh = syn.shell_mesh(2, 6, 12)
    steps = syn.heartbeat_schedule()[:N_STEPS]
    P = fem.guccione_problem(mesh, C, GUC)
    ustar = newton.solve_heartbeat(P, steps, C["gamma_max"])[0]
    ctx = nl.Context(0)
    problems.setup_guccione(ctx, mesh, C, GUC, syn.shell_dirichlet(mesh), block_size=128)
    opts = problems.make_opts(method, prec, **dict(kw))
    u = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    reps = problems.solve_heartbeat(ctx, u, method, opts, steps, C["gamma_max"])
    assert problems.heartbeat_ok(reps, steps), [(r["t"], r["status_name"]) for r in reps]
    err = relnorm(u.cpu().numpy(), ustar)
    assert err <= (1e-8 if prec == "fp64" else 1e-6), err
