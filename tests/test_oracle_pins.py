"""Pins of the FP64 oracle against facts fixed by the paper and by mechanics.

Every check here compares the oracle with something other than itself:
closed forms, invariants (frame indifference, force / moment balance,
patch test), an independent textbook linear-elastic assembly, finite
differences, brute-force dense algebra, exact volumes and loads of the
synthetic geometry.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle import fem, linear, materials, newton, solvers

MU = 80.194


def _rand_F(rng, n, amp=0.3):
    F = np.eye(3) + amp * rng.standard_normal((n, 3, 3))
    d = np.linalg.det(F)
    F[d < 0, :, 0] *= -1.0  # keep det > 0
    return F


def _rot(axis, ang):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


LAWS = [(materials.M1, (MU, 5.0 * MU)), (materials.M2, (MU, 5.0 * MU, 0.25))]


# ------------------------------------------------------------ geometry / loads
def test_cook_volume_and_traction_resultant():
    m = syn.cook_mesh(8, 8, 1)
    G, V = fem.p1_geometry(m.X, m.conn)
    assert np.all(V > 0)
    assert abs(V.sum() - 14400.0) < 1e-9
    f = fem.dead_traction(m.X, m.faces["load"], (0.0, 2.5, 0.0)).reshape(-1, 3)
    # loaded face: x = 48, y in [44, 60], z in [0, 10] -> area 160
    assert np.allclose(f.sum(axis=0), [0.0, 160.0 * 2.5, 0.0], rtol=0, atol=1e-10)
    # gradients of the shape functions sum to zero (partition of unity)
    assert np.abs(G.sum(axis=1)).max() < 1e-12


def test_cube_and_shell_volumes():
    _, V = fem.p1_geometry(*(lambda m: (m.X, m.conn))(syn.cube_mesh(5)))
    assert abs(V.sum() - 1.0) < 1e-12
    sh = syn.shell_mesh(2, 10, 24)
    _, Vs = fem.p1_geometry(sh.X, sh.conn)
    assert np.all(Vs > 0)


def _face_counts(conn):
    f = np.concatenate([np.sort(conn[:, idx], axis=1) for idx in
                        ([1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2])])
    _, cnt = np.unique(f, axis=0, return_counts=True)
    return cnt


@pytest.mark.parametrize("grid", [(3, 2, 2), (4, 4, 1)])
def test_kuhn_mesh_is_conforming(grid):
    nx, ny, nz = grid
    m = syn.cook_mesh(nx, ny, nz)
    cnt = _face_counts(m.conn)
    assert set(np.unique(cnt)) <= {1, 2}
    n_boundary = 2 * 2 * (nx * ny + ny * nz + nx * nz)  # two triangles per boundary quad
    assert (cnt == 1).sum() == n_boundary


def test_shell_mesh_periodic_conforming():
    sh = syn.shell_mesh(2, 6, 12)
    cnt = _face_counts(sh.conn)
    assert set(np.unique(cnt)) <= {1, 2}
    # closed in phi: boundary = endo + epi + apex ring + base ring
    n_t, n_s, n_c = 2, 6, 12
    assert (cnt == 1).sum() == 2 * (2 * n_s * n_c) + 2 * (2 * n_t * n_c)
    assert sh.faces["endo"].shape[0] == 2 * n_s * n_c


# ------------------------------------------------------------ materials
@pytest.mark.parametrize("kind,params", LAWS)
def test_stress_free_reference(kind, params):
    P = materials.piola(kind, np.eye(3)[None], params)
    assert np.abs(P).max() < 1e-12 * MU


@pytest.mark.parametrize("kind,params", LAWS)
def test_piola_is_gradient_of_energy(kind, params):
    rng = np.random.default_rng(1)
    F = _rand_F(rng, 20)
    P = materials.piola(kind, F, params)
    h = 1e-30
    for k in range(3):
        for L in range(3):
            Fc = F.astype(complex)
            Fc[:, k, L] += 1j * h
            dpsi = materials.energy(kind, Fc, params).imag / h
            assert np.allclose(dpsi, P[:, k, L], rtol=1e-11, atol=1e-9 * MU)


def test_M1_cauchy_stress_textbook_form():
    # compressible neo-Hookean in spatial form: sigma = mu/J (b - I) + lam ln J / J I
    rng = np.random.default_rng(2)
    lam = 7.0 * MU
    F = _rand_F(rng, 30)
    P = materials.piola(materials.M1, F, (MU, lam))
    J = np.linalg.det(F)
    sigma = np.einsum("eij,ekj->eik", P, F) / J[:, None, None]
    b = np.einsum("eij,ekj->eik", F, F)
    ref = (MU / J)[:, None, None] * (b - np.eye(3)) + (lam * np.log(J) / J)[:, None, None] * np.eye(3)
    assert np.allclose(sigma, ref, rtol=1e-11, atol=1e-10 * MU)


def test_M2_split_special_cases():
    lam = 9.0 * MU
    kappa = lam + 2 * MU / 3
    # pure dilatation: the isochoric part vanishes, P = kappa (a^6 - 1) / (2 a) I
    for a in (0.9, 1.05, 1.3):
        P = materials.piola(materials.M2, a * np.eye(3)[None], (MU, lam, 0.25))[0]
        assert np.allclose(P, kappa * (a ** 6 - 1) / (2 * a) * np.eye(3), rtol=1e-12)
    # isochoric stretch diag(a, 1/a, 1): only the deviatoric part, mu (F - I1/3 F^-T)
    a = 1.4
    F = np.diag([a, 1 / a, 1.0])
    I1 = a * a + 1 / (a * a) + 1
    P = materials.piola(materials.M2, F[None], (MU, lam, 0.25))[0]
    ref = MU * (F - I1 / 3 * np.diag([1 / a, a, 1.0]))
    assert np.allclose(P, ref, rtol=1e-12, atol=1e-12 * MU)


@pytest.mark.parametrize("kind,params", LAWS)
def test_frame_indifference_of_stress(kind, params):
    rng = np.random.default_rng(3)
    F = _rand_F(rng, 10)
    Q = _rot([1.0, 2.0, -0.5], 0.7)
    P = materials.piola(kind, F, params)
    PQ = materials.piola(kind, np.einsum("ij,ejk->eik", Q, F), params)
    assert np.allclose(PQ, np.einsum("ij,ejk->eik", Q, P), rtol=1e-11, atol=1e-9 * MU)


# ------------------------------------------------------------ assembly
def _cook(nx=4, ny=4, nz=1, ratio=5.0, material=materials.M1):
    m = syn.cook_mesh(nx, ny, nz)
    return m, fem.cook_problem(m, mu=MU, lam=ratio * MU, material=material)


def test_residual_at_rest_is_minus_load():
    m, P = _cook()
    r = P.residual(np.zeros(P.n_dofs), 1.0)
    ref = -P.f_ext.copy()
    ref[P.fixed] = 0
    assert np.allclose(r, ref, atol=1e-12)
    assert np.abs(P.residual(np.zeros(P.n_dofs), 0.0)).max() == 0.0


@pytest.mark.parametrize("kind", [materials.M1, materials.M2])
def test_rigid_rotation_gives_zero_internal_force(kind):
    m, P = _cook(material=kind)
    Q = _rot([0.3, -1.0, 0.4], 0.9)
    u = (m.X @ Q.T - m.X).reshape(-1)
    f = P.internal_force(u)
    assert np.abs(f).max() < 1e-10 * MU


def test_patch_test_affine_field():
    m, P = _cook(6, 6, 2)
    H = 0.02 * np.random.default_rng(4).standard_normal((3, 3))
    u = (m.X @ H.T).reshape(-1)
    f = P.internal_force(u).reshape(-1, 3)
    # interior nodes (not on any boundary face) carry zero net force
    nx, ny, nz = 6, 6, 2
    idx = np.arange(m.n_nodes)
    i, j, k = idx % (nx + 1), (idx // (nx + 1)) % (ny + 1), idx // ((nx + 1) * (ny + 1))
    interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    assert interior.sum() > 0
    scale = np.abs(f).max()
    assert np.abs(f[interior]).max() < 1e-11 * scale


def test_force_and_moment_balance():
    m, P = _cook(5, 4, 2)
    u = syn.random_field(P.n_dofs, 0.05, seed=5)
    f = P.internal_force(u).reshape(-1, 3)
    x = m.X + u.reshape(-1, 3)
    scale = np.abs(f).max()
    assert np.abs(f.sum(axis=0)).max() < 1e-11 * scale * m.n_nodes
    mom = np.cross(x, f).sum(axis=0)
    assert np.abs(mom).max() < 1e-10 * scale * 60 * m.n_nodes


@pytest.mark.parametrize("kind", [materials.M1, materials.M2])
def test_tangent_matches_central_differences(kind):
    m, P = _cook(3, 3, 1, ratio=50.0, material=kind)
    u = P.lift(syn.random_field(P.n_dofs, 0.05, seed=6))
    v = syn.random_field(P.n_dofs, 1.0, seed=7)
    v[P.fixed] = 0
    Jv = P.jv(u, v)
    h = 1e-5
    fd = (P.residual(u + h * v) - P.residual(u - h * v)) / (2 * h)
    assert np.linalg.norm(fd - Jv) <= 1e-7 * np.linalg.norm(Jv)


def test_tangent_symmetric():
    m, P = _cook(3, 3, 1)
    u = P.lift(syn.random_field(P.n_dofs, 0.05, seed=8))
    K = P.stiffness(u)
    assert abs(K - K.T).max() <= 1e-12 * abs(K).max()


@pytest.mark.parametrize("kind,c_vol", [(materials.M1, None), (materials.M2, 0.25)])
def test_tangent_at_rest_is_linear_elasticity(kind, c_vol):
    m = syn.cook_mesh(3, 2, 1)
    lam = 12.0 * MU
    P = fem.cook_problem(m, mu=MU, lam=lam, material=kind, c_vol=c_vol)
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False)
    Klin = linear.stiffness_linear(m.X, m.conn, lam, MU)
    assert abs(K - Klin).max() <= 1e-11 * abs(Klin).max()


def test_printed_cook_law_has_fourfold_bulk_term():
    # with the literal coefficient (c_vol = 1) the small-strain tangent equals
    # linear elasticity with lambda' = 4 kappa - 2 mu / 3 (the reading's motivation)
    m = syn.cook_mesh(2, 2, 1)
    lam = 3.0 * MU
    kappa = lam + 2 * MU / 3
    P = fem.cook_problem(m, mu=MU, lam=lam, material=materials.M2, c_vol=1.0)
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False)
    Klin = linear.stiffness_linear(m.X, m.conn, 4 * kappa - 2 * MU / 3, MU)
    assert abs(K - Klin).max() <= 1e-11 * abs(Klin).max()


def test_small_load_linear_limit():
    m = syn.cook_mesh(4, 4, 1)
    lam = 5.0 * MU
    Klin = linear.stiffness_linear(m.X, m.conn, lam, MU)
    P = fem.cook_problem(m, mu=MU, lam=lam)
    free = P.free
    ulin = np.zeros(P.n_dofs)
    ulin[free] = spla.spsolve(Klin[free][:, free].tocsc(), P.f_ext[free])
    errs = []
    for tau in (1e-3, 1e-4):
        u, _ = newton.newton_exact(P, np.zeros(P.n_dofs), tau)
        errs.append(np.linalg.norm(u / tau - ulin) / np.linalg.norm(ulin))
    assert errs[0] < 1e-2
    assert errs[1] < 0.2 * errs[0]  # error is O(tau)


def test_exact_newton_converges_quadratically():
    m, P = _cook(8, 8, 1)  # the 384-tet Cook mesh
    u, h = newton.newton_exact(P, np.zeros(P.n_dofs), 1.0, rtol=1e-14)
    h = np.array(h) / h[0]
    assert h[-1] <= 1e-11
    # normalised quadratic contraction once in the asymptotic regime:
    # ||r_k+1|| / ||r_0|| <= 10 (||r_k|| / ||r_0||)^2 (a linear rate fails this)
    tail = [i for i in range(len(h) - 1) if h[i] < 1e-2]
    assert len(tail) >= 2
    for i in tail:
        assert h[i + 1] <= 10.0 * h[i] ** 2


# ------------------------------------------------------------ linear algebra
def _spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.linspace(1.0, cond, n)) @ Q.T


def test_two_loop_equals_dense_bfgs_update():
    n = 12
    A = _spd(n, 9)
    rng = np.random.default_rng(10)
    pairs = []
    for _ in range(5):
        s = rng.standard_normal(n)
        pairs.append((s, A @ s))
    H0 = np.diag(1.0 / np.diag(A))
    g = rng.standard_normal(n)
    z = solvers.two_loop(g, pairs, lambda q: H0 @ q)
    H = solvers.bfgs_inverse_dense(H0, pairs)
    assert np.allclose(z, H @ g, rtol=1e-12, atol=1e-12)
    s, y = pairs[-1]
    assert np.allclose(H @ y, s, rtol=1e-11)  # secant equation


def test_lbfgs_exact_initial_inverse_converges_in_one_step():
    n = 20
    A = _spd(n, 11)
    b = np.random.default_rng(12).standard_normal(n)
    Ainv = np.linalg.inv(A)
    res = solvers.lbfgs(lambda u: A @ u - b, lambda q: Ainv @ q, np.zeros(n), rtol=1e-12)
    assert res["converged"] and res["nit"] == 1


def _krylov_minimizer(A, Minv, b, k):
    """Brute force: argmin ||b - A M^-1 y|| over y in span{b, (A M^-1) b, ...}."""
    AM = A @ Minv
    basis = [b]
    for _ in range(k - 1):
        basis.append(AM @ basis[-1])
    Kb = np.array(basis).T
    c, *_ = np.linalg.lstsq(AM @ Kb, b, rcond=None)
    return Minv @ (Kb @ c)


@pytest.mark.parametrize("orth", ["mgs", "cgs2"])
def test_gmres_iterate_is_krylov_least_squares(orth):
    n = 9
    rng = np.random.default_rng(13)
    A = np.eye(n) * 3 + rng.standard_normal((n, n))  # nonsymmetric
    d = np.abs(np.diag(A)) + 1
    Minv = np.diag(1.0 / d)
    b = rng.standard_normal(n)
    for k in (1, 3, 5):
        x, its, _, _ = solvers.gmres(lambda v: A @ v, b, lambda v: v / d, rtol=0, atol=0,
                                     max_it=k, orth=orth)
        assert its == k
        ref = _krylov_minimizer(A, Minv, b, k)
        assert np.allclose(x, ref, rtol=1e-9, atol=1e-10)
    x, its, _, conv = solvers.gmres(lambda v: A @ v, b, lambda v: v / d, rtol=1e-14, atol=0,
                                    max_it=n)
    assert np.allclose(A @ x, b, atol=1e-10)


def test_gmres_restarted_and_cg_solve_spd():
    A = _spd(30, 14, cond=200)
    b = np.random.default_rng(15).standard_normal(30)
    d = np.diag(A)
    x1, _, _, c1 = solvers.gmres(lambda v: A @ v, b, lambda v: v / d, rtol=1e-12, atol=0,
                                 restart=7, max_it=3000)
    x2, k2, _, c2 = solvers.cg(lambda v: A @ v, b, lambda v: v / d, rtol=1e-12, atol=0)
    xs = np.linalg.solve(A, b)
    assert c1 and c2
    assert np.allclose(x1, xs, rtol=1e-9) and np.allclose(x2, xs, rtol=1e-9)


def _krylov_minimizer_anorm(A, Minv, b, k):
    """Brute force: argmin ||x - A^-1 b||_A over x in K_k(M^-1 A, M^-1 b).
    The normal equations of that A-norm problem are (K^T A K) c = K^T b."""
    MA = Minv @ A
    Kb = np.zeros((b.size, 0))
    w = Minv @ b
    for _ in range(k):  # an orthonormal basis of the same space, column by column
        for _ in range(2):
            w = w - Kb @ (Kb.T @ w)
        Kb = np.column_stack([Kb, w / np.linalg.norm(w)])
        w = MA @ Kb[:, -1]
    c = np.linalg.solve(Kb.T @ A @ Kb, Kb.T @ b)
    return Kb @ c


def test_cg_iterate_is_a_norm_krylov_minimizer():
    """Preconditioned CG's k-th iterate minimises the A-norm of the error over
    the k-dimensional Krylov space of M^-1 A and M^-1 b (the defining property
    of CG; a wrong beta, alpha or inner product breaks it after step 1 or 2)."""
    n = 12
    A = _spd(n, 31, cond=50)
    rng = np.random.default_rng(32)
    d = np.diag(A) * (1.0 + 0.5 * rng.random(n))  # not the exact diagonal
    Minv = np.diag(1.0 / d)
    b = rng.standard_normal(n)
    xs = np.linalg.solve(A, b)
    errs = []
    for k in (1, 2, 3, 5, 8):
        x, its, _, _ = solvers.cg(lambda v: A @ v, b, lambda v: v / d, rtol=0, atol=0, max_it=k)
        assert its == k
        ref = _krylov_minimizer_anorm(A, Minv, b, k)
        assert np.allclose(x, ref, rtol=1e-9, atol=1e-11), k
        e = x - xs
        errs.append(float(e @ A @ e))
    # the A-norm error never increases (nested spaces)
    assert all(errs[i + 1] <= errs[i] * (1 + 1e-12) for i in range(len(errs) - 1))
    # and at k = n the iterate is the exact solution
    x, its, _, _ = solvers.cg(lambda v: A @ v, b, lambda v: v / d, rtol=0, atol=0, max_it=n)
    assert np.allclose(x, xs, rtol=1e-8, atol=1e-10)


def _krylov_minimizer_weighted(A, Minv, b, k):
    """Brute force: argmin ||b - A x||_{M^-1} over x in K_k(M^-1 A, M^-1 b)."""
    MA = Minv @ A
    basis = [Minv @ b]
    for _ in range(k - 1):
        basis.append(MA @ basis[-1])
    Kb = np.array(basis).T
    L = np.linalg.cholesky(Minv)  # ||e||_{M^-1} = ||L^T e||
    c, *_ = np.linalg.lstsq(L.T @ A @ Kb, L.T @ b, rcond=None)
    return Kb @ c


def test_minres_iterate_is_weighted_krylov_minimizer_on_indefinite_matrix():
    n = 10
    rng = np.random.default_rng(21)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.concatenate([np.linspace(-5, -1, 4), np.linspace(1, 9, 6)])) @ Q.T
    d = np.abs(np.diag(A)) + 1.0  # SPD Jacobi-like preconditioner
    b = rng.standard_normal(n)
    for k in (1, 2, 4, 6):
        x, its, _, _ = solvers.minres(lambda v: A @ v, b, lambda v: v / d, rtol=0, atol=0, max_it=k)
        assert its == k
        assert np.allclose(x, _krylov_minimizer_weighted(A, np.diag(1 / d), b, k), rtol=1e-8,
                           atol=1e-10)
    x, its, hist, conv = solvers.minres(lambda v: A @ v, b, lambda v: v / d, rtol=1e-12, atol=0,
                                        max_it=200)
    assert conv and np.allclose(A @ x, b, atol=1e-10)
    # unpreconditioned MINRES on a symmetric matrix coincides with GMRES
    xm, *_ = solvers.minres(lambda v: A @ v, b, None, rtol=0, atol=0, max_it=5)
    xg, *_ = solvers.gmres(lambda v: A @ v, b, None, rtol=0, atol=0, max_it=5)
    assert np.allclose(xm, xg, rtol=1e-8, atol=1e-10)


def test_eisenstat_walker_closed_form():
    f = solvers.ew_forcing
    assert f(0, 1.0, 0.0, 0.0, 0.0) == 0.1
    # |1 - 1.5| / 2 = 0.25, clipped to eta_max = 0.1
    assert f(1, 1.0, 2.0, 1.5, 0.1) == 0.1
    # |1e-3 - 9e-4| / 1e-1 = 1e-3; safeguard 0.1^phi = 0.0241 < 0.1 is inactive
    assert abs(f(2, 1e-3, 1e-1, 9e-4, 0.1) - 1e-3) < 1e-15
    # safeguard active with a larger cap: 0.5^phi = 0.3258 > 0.1 wins over 1e-3
    assert abs(f(2, 1e-3, 1e-1, 9e-4, 0.5, rtolmax=0.9) - 0.5 ** 1.6180339887498949) < 1e-12
    # version 2: gamma (||r_k|| / ||r_k-1||)^alpha
    assert abs(f(3, 1e-2, 1e-1, 0.0, 0.01, version=2, rtolmax=0.9) - 0.1 ** 1.6180339887498949) < 1e-15


def test_inexact_newton_and_bfgs_reach_exact_root():
    m, P = _cook(4, 4, 1)
    ustar, _ = newton.newton_exact(P, np.zeros(P.n_dofs), 1.0)

    def lin(u):
        K = P.stiffness(u)
        d = K.diagonal()
        return (lambda v: K @ v), (lambda v: v / d)

    res = solvers.newton_krylov(lambda u: P.residual(u), lin, np.zeros(P.n_dofs), inexact=True,
                                rtol=1e-10, ksp_max_it=5000)
    assert res["converged"]
    assert np.linalg.norm(res["u"] - ustar) <= 1e-8 * np.linalg.norm(ustar)
    K0 = P.stiffness(np.zeros(P.n_dofs))
    lu = spla.splu(K0.tocsc())
    res = solvers.lbfgs(lambda u: P.residual(u), lu.solve, np.zeros(P.n_dofs), m=10, rtol=1e-10)
    assert res["converged"]
    assert np.linalg.norm(res["u"] - ustar) <= 1e-7 * np.linalg.norm(ustar)


def test_lbfgs_refresh_rebuilds_h0_and_drops_pairs():
    # on a quadratic g = A u - b with an exact relinearization (H0 = A^-1),
    # the first refreshed step lands on the root; without refresh and with a
    # poor H0 the same iteration count does not
    from oracle import solvers

    rng = np.random.default_rng(2)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.standard_normal(n)
    ustar = np.linalg.solve(A, b)
    res = lambda u: A @ u - b
    poor = lambda q: q / (4.0 * np.diag(A))
    exact = lambda u: (lambda q: np.linalg.solve(A, q))
    r = solvers.lbfgs(res, poor, np.zeros(n), m=3, max_it=3, refresh=2, relinearize=exact,
                      rtol=1e-14)
    assert np.linalg.norm(r["u"] - ustar) <= 1e-10 * np.linalg.norm(ustar)
    assert r["nit"] == 3
    r0 = solvers.lbfgs(res, poor, np.zeros(n), m=3, max_it=3, rtol=1e-14)
    assert np.linalg.norm(r0["u"] - ustar) > 1e-6 * np.linalg.norm(ustar)


def test_newton_lag_reuses_the_first_tangent_on_a_quadratic_residual():
    # r(u) = A u + 0.1 u^3 - b: with lag = 3 the second and third iterations
    # use the tangent at u0, exactly the chord iteration written out here
    from oracle import solvers

    rng = np.random.default_rng(4)
    n = 8
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    b = rng.standard_normal(n)
    res = lambda u: A @ u + 0.1 * u ** 3 - b
    jac = lambda u: A + np.diag(0.3 * u ** 2)
    calls = []

    def lin(u):
        calls.append(u.copy())
        K = jac(u)
        return (lambda v: K @ v), (lambda v: v)

    r = solvers.newton_krylov(res, lin, np.zeros(n), lag=3, max_it=4, ksp_rtol=1e-14,
                              ksp_atol=0.0, rtol=1e-30)
    assert len(calls) == 2  # iterations 0 and 3
    u = np.zeros(n)
    K0 = jac(u)
    for _ in range(3):
        u = u - np.linalg.solve(K0, res(u))
    u = u - np.linalg.solve(jac(u), res(u))
    assert np.linalg.norm(r["u"] - u) <= 1e-10 * np.linalg.norm(u)
