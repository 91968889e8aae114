"""Pins of the oracle's quadratic-displacement Cook problem (law M1): checked
against an independent small-strain P2 assembly (its own basis and quadrature),
the exact traction resultant, an affine patch test, central differences and the
gradient of the potential."""

import numpy as np

import synthetic as syn
from oracle import linear, p2

MU, LAM = 80.194, 400.9


def _problem(tau=1.0):
    m = syn.cook_p2_mesh(3, 2, 1)
    return m, p2.cook_p2_problem(m, mu=MU, lam=LAM, tau=tau)


def test_tangent_at_rest_matches_independent_p2_assembly():
    m, P = _problem()
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False).toarray()
    Kl = linear.stiffness_linear_p2(m.X, m.conn, LAM, MU).toarray()
    assert np.abs(K - Kl).max() <= 1e-10 * np.abs(Kl).max()


def test_traction_goes_to_midpoints_with_the_exact_resultant():
    m, P = _problem(tau=2.5)
    f = P.f_ext.reshape(-1, 3)
    area = 16.0 * 10.0  # the x = 48 side: y in [44, 60], thickness 10
    assert np.allclose(f.sum(0), [0.0, 2.5 * area, 0.0], rtol=1e-14)
    n_vert = int(np.asarray(m.conn)[:, :4].max()) + 1
    assert np.all(f[:n_vert] == 0.0)


def test_affine_patch_test():
    m, P = _problem()
    rng = np.random.default_rng(3)
    A = 0.05 * rng.standard_normal((3, 3))
    u = (m.X @ A.T + np.array([0.1, -0.2, 0.3])).reshape(-1)
    re = P.element_residual(u[P.edofs])
    r = np.zeros(P.n_dofs)
    np.add.at(r, P.edofs.reshape(-1), re.reshape(-1))
    X = m.X
    inner = ~((np.isclose(X[:, 2], 0) | np.isclose(X[:, 2], 10))
              | np.isclose(X[:, 0], 0) | np.isclose(X[:, 0], 48)
              | np.isclose(X[:, 1], 44 / 48 * X[:, 0]) | np.isclose(X[:, 1], 44 + X[:, 0] / 3))
    assert inner.sum() > 0
    rr = r.reshape(-1, 3)
    assert np.abs(rr[inner]).max() <= 1e-10 * np.abs(rr).max()


def test_tangent_and_residual_consistency():
    m, P = _problem()
    rng = np.random.default_rng(5)
    u = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    K = P.stiffness(u, dirichlet=False)
    v = rng.standard_normal(P.n_dofs)
    h = 1e-6

    def rfree(x):
        re = P.element_residual(x[P.edofs])
        r = np.zeros(P.n_dofs)
        np.add.at(r, P.edofs.reshape(-1), re.reshape(-1))
        return r

    fd = (rfree(u + h * v) - rfree(u - h * v)) / (2 * h)
    assert np.abs(K @ v - fd).max() <= 1e-6 * np.abs(fd).max()
    # the residual is the gradient of the potential (free dofs)
    w = rng.standard_normal(P.n_dofs)
    w[P.fixed] = 0.0
    d = (P.energy(u + h * w, 0.7) - P.energy(u - h * w, 0.7)) / (2 * h)
    assert abs(d - P.residual(u, 0.7) @ w) <= 1e-6 * abs(d)
