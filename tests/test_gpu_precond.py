"""GPU parity of the Jacobi-type preconditioners (point and nodal 3x3 block)
against the oracle's definitions on the assembled tangent, and solves with
the block preconditioner against the oracle's exact-Newton root.

Tolerances: blocks and FP64 applications <= 1e-12 (max-norm relative to the
largest entry); FP32 application <= 1e-5 (2-norm); solutions <= 1e-8 (FP64
at a 1e-11 stopping rule) and <= 1e-6 (mixed).
"""

import numpy as np
import pytest

import synthetic as syn
from oracle import fem, materials, newton, precond
from tests.gpu_common import MU, assert_fp32_entrywise, relmax, relnorm, row_magnitude, smooth_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2203_05610_amd import nlelast as nl  # noqa: E402
from paper_2203_05610_amd import problems  # noqa: E402


def _t(x, dtype=torch.float64):
    return torch.tensor(np.asarray(x), dtype=dtype, device="cuda")


def _cook(nx, ny, nz, ratio, be, mat="M1", tau=1.0):
    mesh = syn.cook_mesh(nx, ny, nz)
    kind = materials.M1 if mat == "M1" else materials.M2
    P = fem.cook_problem(mesh, mu=MU, lam=ratio * MU, tau=tau, material=kind)
    ctx = nl.Context(0)
    problems.setup_cook(ctx, mesh, MU, ratio * MU, tau,
                        material=nl.NLE_MAT_M1 if mat == "M1" else nl.NLE_MAT_M2, block_size=be)
    return mesh, P, ctx


def _cardiac(be):
    mesh = syn.shell_mesh(2, 6, 12)
    P = fem.cardiac_problem(mesh, syn.CARDIAC, gamma=0.03)
    ctx = nl.Context(0)
    problems.setup_cardiac(ctx, mesh, syn.CARDIAC, syn.shell_dirichlet(mesh), block_size=be)
    nl.nle_set_active_tension(ctx, 0.03)
    return mesh, P, ctx


def _pack(B):
    return np.stack([B[:, 0, 0], B[:, 1, 1], B[:, 2, 2], B[:, 0, 1], B[:, 1, 2], B[:, 0, 2]], 1)


CASES = [("cook", (6, 5, 2, 50.0, 64, "M1")), ("cook", (7, 5, 2, 20.0, 128, "M2")),
         ("cook", (12, 10, 3, 5000.0, 512, "M1")), ("cardiac", (200,))]


def _make(kind, args):
    return _cook(*args) if kind == "cook" else _cardiac(*args)


@pytest.mark.parametrize("kind,args", CASES)
def test_block_diagonal_and_applications_match_oracle(kind, args):
    mesh, P, ctx = _make(kind, args)
    n_nodes = mesh.X.shape[0]
    u = P.lift(smooth_state(mesh, P.n_dofs, seed=81))
    s = 0.7
    nl.nle_set_load_scale(ctx, s)
    nl.nle_linearize(ctx, _t(u), nl.NLE_FP32)
    K = P.stiffness(u, load_scale=s)
    B = precond.node_blocks(K, n_nodes)
    b = torch.empty(6 * n_nodes, dtype=torch.float64, device="cuda")
    nl.nle_block_diag(ctx, b)
    assert relmax(b.cpu().numpy().reshape(-1, 6), _pack(B)) < 1e-12

    x = syn.random_field(P.n_dofs, 1.0, seed=82)
    y = torch.empty(P.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_pc_apply(ctx, nl.NLE_PC_BJACOBI3, _t(x), y)
    ref = precond.block_jacobi_apply(B, x)
    assert relmax(y.cpu().numpy(), ref) < 1e-12
    y32 = torch.empty(P.n_dofs, dtype=torch.float32, device="cuda")
    nl.nle_pc_apply(ctx, nl.NLE_PC_BJACOBI3, _t(x, torch.float32), y32, nl.NLE_FP32)
    assert relnorm(y32.double().cpu().numpy(), ref) < 1e-5
    # the applied 3x3 inverses, column by column (a block that is not
    # positive definite is applied as its diagonal)
    cols = [precond.block_jacobi_apply(B, np.tile(np.eye(3)[c], n_nodes)).reshape(-1, 3)
            for c in range(3)]
    Ainv = np.abs(np.stack(cols, axis=2))
    mag = np.einsum("nij,nj->ni", Ainv, np.abs(x).reshape(-1, 3)).reshape(-1)
    assert_fp32_entrywise(y32.cpu().numpy(), ref, mag, what="block Jacobi")
    nl.nle_pc_apply(ctx, nl.NLE_PC_JACOBI, _t(x), y)
    assert relmax(y.cpu().numpy(), precond.point_jacobi_apply(K, x)) < 1e-12
    nl.nle_pc_apply(ctx, nl.NLE_PC_NONE, _t(x), y)
    assert np.array_equal(y.cpu().numpy(), x)


def test_block_preconditioner_usage_errors():
    mesh, P, ctx = _cook(3, 3, 1, 5.0, 64)
    b = torch.empty(6 * mesh.X.shape[0], dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NleError) as e:
        nl.nle_block_diag(ctx, b)
    assert e.value.status == nl.NLE_E_STATE
    x = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    with pytest.raises(nl.NleError) as e:
        nl.nle_pc_apply(ctx, 7, x, torch.empty_like(x))
    assert e.value.status == nl.NLE_E_INVAL
    tw = syn.twist_p2_mesh(1)
    ctx2 = nl.Context(0)
    problems.setup_twist(ctx2, tw, 1.0)
    xm = torch.zeros(ctx2.n_dofs, dtype=torch.float64, device="cuda")
    nl.nle_linearize(ctx2, xm, nl.NLE_FP64)
    with pytest.raises(nl.NleError) as e:
        nl.nle_pc_apply(ctx2, nl.NLE_PC_BJACOBI3, xm, torch.empty_like(xm))
    assert e.value.status == nl.NLE_E_UNSUPPORTED
    with pytest.raises(nl.NleError) as e:
        nl.nle_solve_nk(ctx2, xm, problems.make_opts("nk", ksp="minres", pc="bjacobi3"))
    assert e.value.status == nl.NLE_E_UNSUPPORTED


METHODS = [
    ("nk", {"ksp": "cg"}),
    ("nk", {"ksp": "minres"}),
    ("nk", {"ksp": "gmres", "orth": "mgs"}),
    ("ink", {"ksp": "cg"}),
    ("ink", {"ksp": "gmres", "orth": "cgs2", "restart": 30}),
    ("bfgs", {"h0": "preonly", "qn_m": 10}),
    ("bfgs", {"h0": "ksp", "qn_m": 10, "ksp": "cg"}),
]

_ROOT = {}


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("method,kw", METHODS)
def test_block_jacobi_solves_match_oracle_root(method, kw, precision):
    mesh, P, ctx = _cook(8, 8, 1, 5.0, 64)
    if "c1" not in _ROOT:
        _ROOT["c1"] = newton.solve_schedule(P, [1.0])[0]
    ustar = _ROOT["c1"]
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    opts = problems.make_opts(method, precision, pc="bjacobi3", **dict(kw))
    tight = precision == "fp64"
    if tight:
        opts.snes_rtol = 1e-11
    if method == "bfgs" and kw.get("h0") == "preonly":
        opts.snes_max_it = 5000
    st, rep = problems.SOLVERS[method](ctx, u, opts)
    assert st == nl.NLE_OK, rep
    err = relnorm(u.cpu().numpy(), ustar)
    assert err <= (1e-8 if tight else 1e-6), (err, rep["nit"])


def test_block_jacobi_cg_iterations_follow_oracle_pcg():
    # first Newton step from u = 0: the same preconditioned CG on the
    # assembled tangent needs the same number of iterations (+-2)
    mesh, P, ctx = _cook(8, 8, 1, 50.0, 64)
    u0 = np.zeros(P.n_dofs)
    K = P.stiffness(u0)
    b = -P.residual(u0)
    B = precond.node_blocks(K, mesh.X.shape[0])
    _, its_ref = precond.pcg(K, b, lambda r: precond.block_jacobi_apply(B, r), rtol=1e-6)
    _, its_pt = precond.pcg(K, b, lambda r: precond.point_jacobi_apply(K, r), rtol=1e-6)
    u = torch.zeros(P.n_dofs, dtype=torch.float64, device="cuda")
    o = problems.make_opts("nk", ksp="cg", pc="bjacobi3")
    o.check_every = 2
    o.snes_max_it = 1
    st, rep = nl.nle_solve_nk(ctx, u, o)
    assert st in (nl.NLE_OK, nl.NLE_DIVERGED_MAXIT)
    assert abs(rep["lit_hist"][0] - its_ref) <= 2, (rep["lit_hist"][0], its_ref, its_pt)
