"""Pins of the oracle's quadratic-displacement elements with the other
compressible laws (M2, the cardiac-like M4 and Guccione's M6): the tangent at
rest against the independent small-strain P2 assembly with each law's
small-strain Lame constants, the element forces of an affine state against
the closed form (the integrals of the quadratic shape-function gradients),
and central differences of the residual and of the potential."""

import numpy as np

import synthetic as syn
from oracle import linear, materials, p2

MU, LAM = 80.194, 400.9
M4C = dict(a=0.1, b=5.0, af=0.2, bf=5.0, kappa=100.0)
GUC = (0.1, 5.0, 2.0, 2.0, 1.0, 1.0, 1.0, 100.0)  # C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B (MPa)


def _frames(ne, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((ne, 3))
    f /= np.linalg.norm(f, axis=1)[:, None]
    s = rng.standard_normal((ne, 3))
    s -= (s * f).sum(1)[:, None] * f
    s /= np.linalg.norm(s, axis=1)[:, None]
    return f, s


def _problem(m, law, params):
    n = m.X.shape[0]
    return p2.P2Problem(m.X, m.conn, law, params, np.zeros(3 * n), np.zeros(0, dtype=np.int64),
                        np.zeros(0))


def test_tangents_at_rest_match_the_small_strain_p2_assembly():
    # M2 with c_vol = 1/4 is Lame (lambda, mu) at small strain; M4 without
    # active tension has mu = a and bulk modulus kappa (with exactly unit,
    # axis-aligned fibres I4 = 1 exactly at rest, where the fibre exponential
    # has zero stress and tangent); M6 with equal b's has Q = b E:E, so
    # mu = C b / 2 and the volumetric term B/2 (J - 1) ln J gives lambda = B
    m = syn.cook_p2_mesh(3, 2, 1)
    ne = m.conn.shape[0]
    f, s = _frames(ne, 1)
    fax = np.eye(3)[np.random.default_rng(4).integers(0, 3, ne)]
    b = 4.0
    cases = [
        (materials.M2, (MU, LAM, 0.25), LAM, MU),
        (materials.M4, (M4C["a"], M4C["b"], M4C["af"], M4C["bf"], M4C["kappa"], 0.0, fax),
         M4C["kappa"] - 2.0 * M4C["a"] / 3.0, M4C["a"]),
        (materials.M6, (2.0, b, b, b, b, b, b, 30.0, 0.0, f, s), 30.0, 2.0 * b / 2.0),
    ]
    for law, params, lam, mu in cases:
        P = _problem(m, law, params)
        K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False).toarray()
        Kl = linear.stiffness_linear_p2(m.X, m.conn, lam, mu).toarray()
        assert np.abs(K - Kl).max() <= 1e-9 * np.abs(Kl).max(), law


def test_affine_state_element_forces_follow_the_closed_form():
    # F constant: the element's forces are V P(F_e) (g_a + g_b) at the edge
    # midpoint of edge (a, b) and zero at the vertices (the gradient of a
    # quadratic vertex function integrates to zero), with P_e of each
    # element's own fibre (and sheet)
    m = syn.cook_p2_mesh(2, 2, 1)
    ne = m.conn.shape[0]
    f, s = _frames(ne, 2)
    rng = np.random.default_rng(3)
    A = 0.05 * rng.standard_normal((3, 3))
    F = np.eye(3) + A
    u = (m.X @ A.T).reshape(-1)
    for law, params in [
        (materials.M2, (MU, LAM, 0.25)),
        (materials.M4, (M4C["a"], M4C["b"], M4C["af"], M4C["bf"], M4C["kappa"], 0.03, f)),
        (materials.M6, GUC + (0.03, f, s)),
    ]:
        P = _problem(m, law, params)
        re = P.element_residual(u[P.edofs]).reshape(ne, 10, 3)
        Pe = materials.piola(law, np.broadcast_to(F, (ne, 3, 3)), params)
        g = P.G  # (n_e, 4, 3): gradients of the barycentric coordinates
        assert np.abs(re[:, :4]).max() <= 1e-12 * np.abs(re).max(), law
        for k, (a, b) in enumerate(p2.EDGES):
            ref = P.V[:, None] * np.einsum("eiJ,eJ->ei", Pe, g[:, a] + g[:, b])
            assert np.abs(re[:, 4 + k] - ref).max() <= 1e-12 * np.abs(ref).max(), (law, k)


def test_tangent_residual_and_potential_consistency():
    mesh = syn.p2_from_p1(syn.shell_mesh(2, 4, 8))
    P4 = p2.shell_p2_problem(mesh, dict(syn.CARDIAC), gamma=0.03)
    P6 = p2.shell_p2_problem(mesh, dict(syn.CARDIAC), gamma=0.03, law=GUC)
    rng = np.random.default_rng(5)
    for P in (P4, P6):
        u = P.lift(0.05 * rng.standard_normal(P.n_dofs))
        K = P.stiffness(u, dirichlet=False)
        v = rng.standard_normal(P.n_dofs)
        h = 1e-6

        def rfree(x):
            re = P.element_residual(x[P.edofs])
            r = np.zeros(P.n_dofs)
            np.add.at(r, P.edofs.reshape(-1), re.reshape(-1))
            return r

        fd = (rfree(u + h * v) - rfree(u - h * v)) / (2 * h)
        assert np.abs(K @ v - fd).max() <= 1e-6 * np.abs(fd).max(), P.material
        w = rng.standard_normal(P.n_dofs)
        w[P.fixed] = 0.0
        d = (P.energy(u + h * w) - P.energy(u - h * w)) / (2 * h)
        assert abs(d - P.residual(u) @ w) <= 1e-6 * abs(d), P.material
