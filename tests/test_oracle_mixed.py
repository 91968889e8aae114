"""Pins of the oracle's mixed P2-P1 twist form (Sec. 4 "Twist test", law M3).

Compared with: closed-form integrals of monomials over a tetrahedron,
exact reproduction of quadratic fields, the patch test (constant pressure,
isochoric affine deformation), central differences, and the small-strain
limit assembled independently (Vandermonde-built quadratic basis, collapsed
Gauss rule) in oracle/linear.py.
"""

import math

import numpy as np
import pytest

import synthetic as syn
from oracle import linear, mixed, newton


def test_quadrature_is_exact_for_quadratics():
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]])
    lam = mixed.QUAD_BARY
    pts = lam @ X
    w = np.full(4, 1.0 / 24.0)  # V/4 with V = 1/6
    assert abs(w.sum() - 1 / 6) <= 1e-16
    assert abs(w @ pts[:, 0] - 1 / 24) <= 1e-16
    assert abs(w @ pts[:, 0] ** 2 - 1 / 60) <= 1e-16
    assert abs(w @ (pts[:, 0] * pts[:, 1]) - 1 / 120) <= 1e-16


def test_p2_gradients_reproduce_quadratic_fields():
    m = syn.twist_p2_mesh(2)
    rng = np.random.default_rng(51)
    A = rng.standard_normal((3, 10))

    def field(x):
        mono = np.stack([np.ones(len(x)), x[:, 0], x[:, 1], x[:, 2], x[:, 0] ** 2, x[:, 1] ** 2,
                         x[:, 2] ** 2, x[:, 0] * x[:, 1], x[:, 0] * x[:, 2], x[:, 1] * x[:, 2]], 1)
        return mono @ A.T

    def grad(x):
        z, o = np.zeros(len(x)), np.ones(len(x))
        dm = [np.stack([z, o, z, z, 2 * x[:, 0], z, z, x[:, 1], x[:, 2], z], 1),
              np.stack([z, z, o, z, z, 2 * x[:, 1], z, x[:, 0], z, x[:, 2]], 1),
              np.stack([z, z, z, o, z, z, 2 * x[:, 2], z, x[:, 0], x[:, 1]], 1)]
        return np.stack([d @ A.T for d in dm], axis=2)  # (pts, i, J)

    P = mixed.twist_problem(m, 1.0, 0.0)
    U = field(m.X)[P.conn]  # (e, 10, 3)
    for q in range(4):
        H = np.einsum("eai,eaJ->eiJ", U, P.gradN[q])
        xq = np.einsum("a,eai->ei", mixed.QUAD_BARY[q], m.X[P.conn[:, :4]])
        assert np.abs(H - grad(xq)).max() <= 1e-12
        assert np.abs(P.gradN[q].sum(axis=1)).max() <= 1e-12  # partition of unity


def test_rest_and_constant_pressure_patch():
    m = syn.twist_p2_mesh(2)
    P = mixed.MixedProblem(m.X, m.conn, m.pconn, m.n_pressure, 1.0, np.zeros(0, np.int64),
                           np.zeros(0))
    x = np.zeros(P.n_dofs)
    assert np.abs(P.residual(x)).max() == 0.0
    # constant pressure, no displacement: zero divergence-free stress field
    # except on the boundary, where R_u is the traction -p0 N integrated
    x[3 * P.n_u:] = 0.7
    r = P.residual(x)
    ru = r[: 3 * P.n_u].reshape(-1, 3)
    X = m.X
    interior = np.all((X > 1e-12) & (X < 1 - 1e-12), axis=1)
    assert np.abs(ru[interior]).max() <= 1e-14
    assert np.abs(r[3 * P.n_u:]).max() == 0.0
    # resultant of the boundary forces of a uniform pressure vanishes
    assert np.abs(ru.sum(0)).max() <= 1e-14


def test_isochoric_affine_patch():
    # simple shear (J = 1) with constant pressure: interior forces vanish
    m = syn.twist_p2_mesh(2)
    P = mixed.MixedProblem(m.X, m.conn, m.pconn, m.n_pressure, 1.3, np.zeros(0, np.int64),
                           np.zeros(0))
    Gm = np.zeros((3, 3))
    Gm[0, 1] = 0.3
    x = np.concatenate([(m.X @ Gm.T).reshape(-1), np.full(P.n_p, -0.4)])
    r = P.residual(x)
    ru = r[: 3 * P.n_u].reshape(-1, 3)
    interior = np.all((m.X > 1e-12) & (m.X < 1 - 1e-12), axis=1)
    assert np.abs(ru[interior]).max() <= 1e-13
    assert np.abs(r[3 * P.n_u:]).max() <= 1e-15


def test_mixed_tangent_central_differences_and_symmetry():
    m = syn.twist_p2_mesh(2)
    P = mixed.twist_problem(m, 1.0, math.radians(20))
    rng = np.random.default_rng(52)
    x = P.lift(np.concatenate([0.02 * rng.standard_normal(3 * P.n_u),
                               0.1 * rng.standard_normal(P.n_p)]))
    v = rng.standard_normal(P.n_dofs)
    v[P.fixed] = 0
    K = P.stiffness(x)
    h = 1e-6
    fd = (P.residual(x + h * v) - P.residual(x - h * v)) / (2 * h)
    assert np.linalg.norm(K @ v - fd) <= 1e-8 * np.linalg.norm(fd)
    assert abs(K - K.T).max() <= 1e-13 * abs(K).max()


def test_small_strain_blocks_match_independent_assembly():
    m = syn.twist_p2_mesh(1)
    mu = 1.7
    P = mixed.MixedProblem(m.X, m.conn, m.pconn, m.n_pressure, mu, np.zeros(0, np.int64),
                           np.zeros(0))
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False)
    nu = 3 * P.n_u
    Kuu = K[:nu, :nu]
    Kpu = K[nu:, :nu]
    Klin = linear.stiffness_linear_p2(m.X, m.conn, 0.0, mu)
    Bdiv = linear.divergence_p2p1(m.X, m.conn, m.pconn, P.n_p)
    assert abs(Kuu - Klin).max() <= 1e-12 * abs(Klin).max()
    assert abs(Kpu - Bdiv).max() <= 1e-12 * abs(Bdiv).max()
    assert abs(K[nu:, nu:]).max() == 0.0


def test_twist_exact_newton_converges_quadratically():
    m = syn.twist_p2_mesh(2)
    P = mixed.twist_problem(m, 1.0, 0.0)
    x = np.zeros(P.n_dofs)
    for s in range(1, 10):
        mixed.set_twist_angle(P, m, math.radians(10 * s))
        x, h = newton.newton_exact(P, x, 1.0)
        assert len(h) <= 7
        hh = np.array(h) / h[0]
        k = int(np.argmax(hh < 1e-4))
        assert hh[k + 1] <= 10 * hh[k] ** 2 or hh[k + 1] <= 1e-13
    assert P.min_jacobian(x) > 0.5


# ---- the paper's twist statement: law M5 on the P2-P0 pair (Sec. 4) -----------
M5 = mixed.TWIST_M5


def _rand_F(rng, n=5, amp=0.2):
    return np.eye(3) + amp * rng.standard_normal((n, 3, 3))


def test_m5_stress_free_reference_and_printed_balance():
    F = np.eye(3)[None]
    assert np.abs(mixed.m5_piola(F, np.zeros(1), M5)).max() <= 1e-10
    # any other constants leave a stress at rest unless 2 a_p + 4 b_p = 4 b_s + 2 a_s
    assert np.abs(mixed.m5_piola(F, np.zeros(1), (1.0, 2.0, 3.0, 4.0))).max() > 1.0
    assert abs(mixed.m5_energy(F, np.zeros(1), M5)[0]) <= 1e-9


def test_m5_piola_is_gradient_of_energy():
    rng = np.random.default_rng(61)
    F = _rand_F(rng)
    p = rng.standard_normal(5) * 100.0
    prm = (1.3, 0.7, 2.1, 0.4)  # generic constants: each term checked on its own
    P = mixed.m5_piola(F, p, prm)
    h = 1e-30
    for i in range(3):
        for j in range(3):
            Fc = F.astype(np.complex128)
            Fc[:, i, j] += 1j * h
            d = mixed.m5_energy(Fc, p, prm).imag / h
            assert np.allclose(P[:, i, j], d, rtol=1e-12, atol=1e-12)


def test_m5_frame_indifference():
    rng = np.random.default_rng(62)
    F = _rand_F(rng)
    p = rng.standard_normal(5)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    P = mixed.m5_piola(F, p, M5)
    PQ = mixed.m5_piola(Q[None] @ F, p, M5)
    assert np.allclose(PQ, Q[None] @ P, rtol=1e-12, atol=1e-9)
    # the energy is invariant too
    assert np.allclose(mixed.m5_energy(Q[None] @ F, p, M5), mixed.m5_energy(F, p, M5),
                       rtol=1e-12, atol=1e-9)


def test_p2p0_tangent_at_rest_is_linear_elasticity_and_divergence():
    # at rest (u = 0, p = 0) the displacement block is small-strain elasticity
    # with mu = 2 (a_p + b_p), lambda = 4 b_p, and the pressure rows are
    # -int div v on each element; both assembled independently in linear.py
    m = syn.twist_p2_mesh(2)
    P = mixed.twist_problem_p0(m, 0.0)
    P.ddofs = np.zeros(0, np.int64)
    P.dvals = np.zeros(0)
    P.__post_init__()
    K = P.stiffness(np.zeros(P.n_dofs))
    nu = 3 * P.n_u
    ap, bp = M5[0], M5[1]
    Klin = linear.stiffness_linear_p2(m.X, m.conn, 4.0 * bp, 2.0 * (ap + bp))
    assert abs(K[:nu, :nu] - Klin).max() <= 1e-9 * abs(Klin).max()
    Bref = linear.divergence_p2p0(m.X, m.conn)
    assert abs(K[nu:, :nu] - Bref).max() <= 1e-12 * abs(Bref).max()
    assert abs(K[:nu, nu:] - Bref.T).max() <= 1e-12 * abs(Bref).max()
    assert abs(K[nu:, nu:]).max() == 0.0
    # lumped P0 pressure mass = element volumes; mu_eff of the law
    assert np.allclose(P.pressure_mass_lumped(), P.V)
    assert P.mu_eff == 2.0 * (ap + bp)


def test_p2p0_twist_newton_reaches_incompressible_root():
    # exact Newton on one twist step: quadratic convergence and, at the root,
    # int_e (J - 1) = 0 on every element (the P0 constraint) to rounding
    m = syn.twist_p2_mesh(2)
    P = mixed.twist_problem_p0(m, math.radians(20))
    x, hist = newton.newton_exact(P, np.zeros(P.n_dofs), 1.0)
    assert hist[-1] <= 1e-10 * hist[0]
    nu = 3 * P.n_u
    r = P.residual(x)
    assert np.abs(r[nu:]).max() <= 1e-12 * max(1.0, np.abs(x[:nu]).max())
    assert np.abs(x[nu:]).max() > 1.0  # a nonzero pressure holds the constraint


def _saddle(n_u=9, n_p=3, seed=71):
    """A saddle-point matrix [[A, B^T], [B, 0]] with diagonal A and pressure
    rows of disjoint supports, where SIMPLE's diag(A) is A itself and
    B diag(A)^-1 B^T is diagonal: the Schur complement is exact."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    A = np.diag(1.0 + rng.random(n_u))
    B = np.zeros((n_p, n_u))
    for b in range(n_p):
        B[b, 3 * b: 3 * b + 3] = rng.standard_normal(3)
    K = np.block([[A, B.T], [B, np.zeros((n_p, n_p))]])
    return sp.csr_matrix(K), np.diag(A)


def test_schur_lower_with_exact_schur_converges_in_two_gmres_steps():
    # App. B: with the exact Schur complement the lower block-triangular
    # preconditioner leaves (M P^-1 - I)^2 = 0, so GMRES needs two steps; the
    # block-diagonal form leaves three distinct eigenvalues, three steps
    from oracle import precond, solvers

    K, dA = _saddle()
    n_u = dA.size
    s = precond.simple_schur_diagonal(K, n_u)
    b = np.random.default_rng(72).standard_normal(K.shape[0])
    low = lambda r: precond.schur_lower_apply(K, n_u, r, lambda ru: ru / dA, s)  # noqa: E731
    x, its, _, ok = solvers.gmres(lambda v: K @ v, b, low, rtol=1e-12, atol=0.0, max_it=20)
    assert ok and its == 2
    diag = lambda r: np.concatenate([r[:n_u] / dA, -r[n_u:] / s])  # noqa: E731
    x2, its2, _, ok2 = solvers.gmres(lambda v: K @ v, b, diag, rtol=1e-12, atol=0.0, max_it=20)
    assert ok2 and its2 == 3
    assert np.allclose(K @ x, b, atol=1e-10) and np.allclose(K @ x2, b, atol=1e-10)


def test_simple_schur_diagonal_of_p0_is_elementwise():
    # with one pressure per element each pressure row lives on its element, so
    # the SIMPLE diagonal is sum over the element's free dofs of B_ei^2 / A_ii
    m = syn.twist_p2_mesh(2)
    P = mixed.twist_problem_p0(m, math.radians(10))
    x = P.lift(np.zeros(P.n_dofs))
    K = P.stiffness(x)
    nu = 3 * P.n_u
    s = mixed_simple = None  # noqa: F841
    from oracle import precond

    s = precond.simple_schur_diagonal(K, nu)
    dA = K.diagonal()[:nu]
    Kd = K.toarray()
    for e in (0, 5, P.conn.shape[0] - 1):
        dofs = P.edofs[e, :30]
        free = P.free[dofs]
        ref = np.sum(Kd[nu + e, dofs[free]] ** 2 / dA[dofs[free]])
        assert abs(s[e] - ref) <= 1e-12 * ref
