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
