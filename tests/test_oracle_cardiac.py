"""Pins of the oracle's cardiac-like parts: law M4 (isotropic and fibre
exponentials, volumetric penalty, active stress of Sec. 4 "Heartbeat test"),
the follower endocardial pressure and the elastic Robin springs.

Each check compares with something other than the formula under test:
complex-step derivatives of the energy, invariance under rotations, the
linear-elastic limit from the independent textbook assembly, the gradient of
an enclosed volume, vanishing resultants of a uniform pressure on a closed
surface, an independent quadrature rule, and central differences.
"""

import math

import numpy as np
import pytest

import synthetic as syn
from oracle import fem, linear, materials, newton

A, B, AF, BF, KAPPA = 0.1, 5.0, 0.2, 5.0, 100.0


def _unit(rng, n):
    f = rng.standard_normal((n, 3))
    return f / np.linalg.norm(f, axis=1)[:, None]


def _rot(axis, ang):
    a = np.asarray(axis, float)
    a /= np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * K + (1 - math.cos(ang)) * K @ K


def _params(gamma, fib):
    return (A, B, AF, BF, KAPPA, gamma, fib)


# ------------------------------------------------------------------- law M4
def test_m4_piola_is_gradient_of_energy():
    rng = np.random.default_rng(11)
    n = 64
    F = np.eye(3) + 0.15 * rng.standard_normal((n, 3, 3))
    fib = _unit(rng, n)
    pr = _params(0.03, fib)
    I4 = np.einsum("eij,ej->ei", F, fib)
    I4 = (I4 ** 2).sum(1)
    assert (I4 > 1).any() and (I4 < 1).any()  # both branches of the fibre term
    P = materials.piola(materials.M4, F, pr)
    h = 1e-30
    for k in range(3):
        for L in range(3):
            Fc = F.astype(complex)
            Fc[:, k, L] += 1j * h
            d = materials.energy(materials.M4, Fc, pr).imag / h
            assert np.abs(d - P[:, k, L]).max() <= 1e-12 * np.abs(P).max()


def test_m4_stress_at_identity_is_the_active_prestress():
    rng = np.random.default_rng(12)
    fib = _unit(rng, 5)
    F = np.broadcast_to(np.eye(3), (5, 3, 3)).copy()
    P0 = materials.piola(materials.M4, F, _params(0.0, fib))
    assert np.abs(P0).max() <= 1e-15
    g = 0.06
    P = materials.piola(materials.M4, F, _params(g, fib))
    assert np.allclose(P, g * np.einsum("ei,ej->eij", fib, fib), rtol=0, atol=1e-15)


def test_m4_frame_indifference_and_transverse_isotropy():
    rng = np.random.default_rng(13)
    n = 32
    F = np.eye(3) + 0.2 * rng.standard_normal((n, 3, 3))
    fib = _unit(rng, n)
    pr = _params(0.04, fib)
    Q = _rot([0.3, -1.0, 0.5], 1.1)
    P = materials.piola(materials.M4, F, pr)
    PQ = materials.piola(materials.M4, np.einsum("ij,ejk->eik", Q, F), pr)
    assert np.abs(PQ - np.einsum("ij,ejk->eik", Q, P)).max() <= 1e-13 * np.abs(P).max()
    # rotating the reference frame together with the fibre leaves Psi unchanged
    R = _rot([1.0, 0.2, -0.7], 0.8)
    psi = materials.energy(materials.M4, F, pr)
    psiR = materials.energy(materials.M4, np.einsum("eij,kj->eik", F, R),
                            _params(0.04, fib @ R.T))
    assert np.abs(psiR - psi).max() <= 1e-13 * np.abs(psi).max()


def test_m4_fibre_term_is_tension_only():
    # uniaxial isochoric stretch along the fibre: the fibre exponential adds
    # stress above I4 = 1 and nothing below
    f = np.array([[1.0, 0.0, 0.0]])
    for lam in (0.9, 1.1):
        F = np.diag([lam, lam ** -0.5, lam ** -0.5])[None]
        with_f = materials.piola(materials.M4, F, (A, B, AF, BF, KAPPA, 0.0, f))
        no_f = materials.piola(materials.M4, F, (A, B, 0.0, BF, KAPPA, 0.0, f))
        d = with_f - no_f
        if lam < 1:
            assert np.abs(d).max() == 0.0
        else:
            assert d[0, 0, 0] > 0 and np.abs(d[0, 1:, :]).max() == 0.0


def test_m4_tangent_at_rest_is_linear_elasticity():
    # gamma = 0 and exactly unit, axis-aligned fibres (I4 = 1 exactly at rest,
    # the fibre exponential has zero stress and zero tangent there): the law
    # linearises to Lame mu = a, lambda = kappa - 2a/3
    m = syn.cook_mesh(3, 2, 1)
    rng = np.random.default_rng(14)
    fib = np.eye(3)[rng.integers(0, 3, m.n_elems)]
    P = fem.Problem(m.X, m.conn, materials.M4, _params(0.0, fib), np.zeros(m.n_dofs),
                    np.zeros(0, dtype=np.int64), np.zeros(0))
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False)
    Klin = linear.stiffness_linear(m.X, m.conn, KAPPA - 2 * A / 3, A)
    assert abs(K - Klin).max() <= 1e-11 * abs(Klin).max()


# ------------------------------------------------------- follower pressure
def _closed_cube(n=2):
    m = syn.cube_mesh(n)
    X = m.X
    tris = [syn.boundary_faces(X, m.conn, np.isclose(X[:, d], v))
            for d in range(3) for v in (0.0, 1.0)]
    return m, np.concatenate(tris)


def _enclosed_volume(x, tri):
    return np.einsum("fi,fi->", x[tri[:, 0]], np.cross(x[tri[:, 1]], x[tri[:, 2]])) / 6.0


def test_pressure_on_closed_surface_is_gradient_of_enclosed_volume():
    m, tri = _closed_cube(2)
    assert abs(_enclosed_volume(m.X, tri) - 1.0) <= 1e-14  # outward, closed
    u = syn.random_field(m.n_dofs, 0.05, seed=21)
    p = 0.7
    f = fem.follower_pressure(m.X, u, tri, p)
    x = m.X + u.reshape(-1, 3)
    grad = np.zeros(m.n_dofs)
    h = 1e-30
    for d in range(m.n_dofs):
        xc = x.astype(complex)
        xc.reshape(-1)[d] += 1j * h
        grad[d] = _enclosed_volume(xc, tri).imag / h
    assert np.abs(f - p * grad).max() <= 1e-13 * np.abs(f).max()
    # uniform pressure on a closed surface: zero net force and moment
    F = f.reshape(-1, 3)
    assert np.abs(F.sum(0)).max() <= 1e-13 * np.abs(F).max()
    assert np.abs(np.cross(x, F).sum(0)).max() <= 1e-13 * np.abs(F).max()


def test_pressure_jacobian_central_differences_and_closed_symmetry():
    m = syn.shell_mesh(2, 6, 12)
    tri = m.faces["endo"]
    u = syn.random_field(m.n_dofs, 0.1, seed=22)
    v = syn.random_field(m.n_dofs, 1.0, seed=23)
    p = 0.002
    K = fem.follower_pressure_jacobian(m.X, u, tri, p)
    h = 1e-5
    fd = (fem.follower_pressure(m.X, u + h * v, tri, p)
          - fem.follower_pressure(m.X, u - h * v, tri, p)) / (2 * h)
    assert np.linalg.norm(K @ v - fd) <= 1e-9 * np.linalg.norm(fd)
    assert abs(K - K.T).max() > 1e-3 * abs(K).max()  # open surface: not symmetric
    mc, trc = _closed_cube(2)
    Kc = fem.follower_pressure_jacobian(mc.X, syn.random_field(mc.n_dofs, 0.05, seed=24), trc, p)
    assert abs(Kc - Kc.T).max() <= 1e-14 * abs(Kc).max()  # closed: conservative


# ------------------------------------------------------------ Robin springs
def test_robin_matrix_equals_midpoint_quadrature():
    m = syn.shell_mesh(2, 6, 12)
    tri = m.faces["epi"]
    kp, kt = 2e-4, 2e-5
    R = fem.robin_matrix(m.X, tri, kp, kt)
    u = syn.random_field(m.n_dofs, 1.0, seed=25).reshape(-1, 3)
    w = syn.random_field(m.n_dofs, 1.0, seed=26).reshape(-1, 3)
    # edge-midpoint rule, exact for quadratics on a triangle: weights A/3
    X = m.X
    tot = 0.0
    for a, b, c in tri:
        nrm = np.cross(X[b] - X[a], X[c] - X[a])
        area = 0.5 * np.linalg.norm(nrm)
        N = nrm / (2 * area)
        for (i, j) in ((a, b), (b, c), (c, a)):
            uq, wq = 0.5 * (u[i] + u[j]), 0.5 * (w[i] + w[j])
            Ku = kt * uq + (kp - kt) * np.dot(N, uq) * N
            tot += area / 3.0 * np.dot(Ku, wq)
    assert abs(w.reshape(-1) @ (R @ u.reshape(-1)) - tot) <= 1e-13 * abs(tot)
    assert abs(R - R.T).max() <= 1e-14 * abs(R).max()


# ------------------------------------------------------------ whole problem
def test_cardiac_residual_jacobian_central_differences():
    m = syn.shell_mesh(2, 6, 12)
    P = fem.cardiac_problem(m, syn.CARDIAC, gamma=0.03)
    u = P.lift(syn.random_field(P.n_dofs, 0.02, seed=27))
    v = syn.random_field(P.n_dofs, 1.0, seed=28)
    v[P.fixed] = 0
    s = 0.7
    Jv = P.jv(u, v, load_scale=s)
    h = 1e-6
    fd = (P.residual(u + h * v, s) - P.residual(u - h * v, s)) / (2 * h)
    assert np.linalg.norm(fd - Jv) <= 1e-7 * np.linalg.norm(Jv)


def test_cardiac_potential_without_pressure_matches_residual():
    # springs + M4 (with active tension) are conservative: r = grad Pi
    m = syn.shell_mesh(2, 6, 12)
    P = fem.cardiac_problem(m, syn.CARDIAC, gamma=0.03)
    P.pressure_tri = None
    u = P.lift(syn.random_field(P.n_dofs, 0.02, seed=29))
    v = syn.random_field(P.n_dofs, 1.0, seed=30)
    v[P.fixed] = 0
    h = 1e-6
    dpi = (P.energy(u + h * v) - P.energy(u - h * v)) / (2 * h)
    assert abs(dpi - P.residual(u) @ v) <= 1e-7 * abs(dpi)


def test_heartbeat_oracle_converges_and_returns_to_rest():
    m = syn.shell_mesh(2, 6, 12)
    P = fem.cardiac_problem(m, syn.CARDIAC)
    sched = syn.heartbeat_schedule()
    u, hists = newton.solve_heartbeat(P, sched, syn.CARDIAC["gamma_max"])
    assert all(len(h) <= 8 for h in hists)
    # the last step has (numerically) no activation and no pressure: rest
    assert sched[-1][1] < 1e-12
    assert np.abs(u).max() <= 1e-9


# ---- the paper's Guccione law (M6, Sec. 4 "Heartbeat test") ---------------------
def _frame(rng, n):
    f = rng.standard_normal((n, 3))
    f /= np.linalg.norm(f, axis=1)[:, None]
    s = rng.standard_normal((n, 3))
    s -= np.einsum("ni,ni->n", s, f)[:, None] * f
    s /= np.linalg.norm(s, axis=1)[:, None]
    return f, s


G6 = (0.9, 18.0, 3.5, 2.5, 1.6, 1.2, 0.8, 50.0)  # C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B


def _g6(f, s, gamma=0.0, law=G6):
    return tuple(law) + (gamma, f, s)


def test_m6_stress_free_and_active_stress_at_rest():
    rng = np.random.default_rng(101)
    f, s = _frame(rng, 4)
    I = np.broadcast_to(np.eye(3), (4, 3, 3))
    assert np.abs(materials.piola("M6", I, _g6(f, s))).max() <= 1e-14
    # at F = I the active stress is gamma f (x) f
    P = materials.piola("M6", I, _g6(f, s, gamma=0.3))
    assert np.allclose(P, 0.3 * np.einsum("ni,nj->nij", f, f), atol=1e-14)


def test_m6_piola_is_gradient_of_energy():
    rng = np.random.default_rng(102)
    f, s = _frame(rng, 6)
    F = np.eye(3) + 0.15 * rng.standard_normal((6, 3, 3))
    prm = _g6(f, s, gamma=0.2)
    P = materials.piola("M6", F, prm)
    h = 1e-30
    for i in range(3):
        for j in range(3):
            Fc = F.astype(np.complex128)
            Fc[:, i, j] += 1j * h
            d = materials.energy("M6", Fc, prm).imag / h
            assert np.allclose(P[:, i, j], d, rtol=1e-12, atol=1e-12)


def test_m6_frame_indifference_and_material_frame_rotation():
    rng = np.random.default_rng(103)
    f, s = _frame(rng, 5)
    F = np.eye(3) + 0.2 * rng.standard_normal((5, 3, 3))
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    prm = _g6(f, s, gamma=0.1)
    # spatial rotation: P(QF) = Q P(F)
    assert np.allclose(materials.piola("M6", Q[None] @ F, prm), Q[None] @ materials.piola("M6", F, prm),
                       atol=1e-10)
    # rotating the body and its fibre frame together: Psi(F Q^T; Q f, Q s) = Psi(F; f, s)
    prm_r = _g6(f @ Q.T, s @ Q.T, gamma=0.1)
    assert np.allclose(materials.energy("M6", F @ Q.T[None], prm_r), materials.energy("M6", F, prm),
                       rtol=1e-12)


def test_m6_isotropic_small_strain_limit_is_linear_elasticity():
    # all b equal: Q = b |E|^2, and at small strain Psi = C b/2 |eps|^2 + B/2 (tr eps)^2,
    # i.e. mu = C b / 2, lambda = B; the tangent at rest of a mesh equals the
    # independent B-matrix assembly
    m = syn.cook_mesh(3, 3, 1)
    rng = np.random.default_rng(104)
    f, s = _frame(rng, m.n_elems)
    b = 4.0
    law = (0.8, b, b, b, b, b, b, 30.0)
    P = fem.Problem(m.X, m.conn, "M6", _g6(f, s, law=law), np.zeros(m.n_dofs), np.zeros(0, np.int64),
                    np.zeros(0))
    K = P.stiffness(np.zeros(m.n_dofs))
    Klin = linear.stiffness_linear(m.X, m.conn, 30.0, 0.8 * b / 2.0)
    assert abs(K - Klin).max() <= 1e-10 * abs(Klin).max()


def test_m6_anisotropy_fibre_stretch_is_stiffer():
    # uniaxial stretch along the fibre costs more than across it (b_ff > b_ss)
    rng = np.random.default_rng(105)
    f, s = _frame(rng, 1)
    n = np.cross(f[0], s[0])
    eps = 0.05
    Ff = np.eye(3) + eps * np.outer(f[0], f[0])
    Fs = np.eye(3) + eps * np.outer(s[0], s[0])
    Fn = np.eye(3) + eps * np.outer(n, n)
    law = (0.9, 18.0, 3.5, 2.5, 1.6, 1.2, 0.8, 0.0)
    e = [materials.energy("M6", F[None], _g6(f, s, law=law))[0] for F in (Ff, Fs, Fn)]
    assert e[0] > e[1] > e[2] > 0.0


GUC = (0.1, 5.0, 2.0, 2.0, 1.0, 1.0, 1.0, 100.0)  # C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B (MPa)


def test_guccione_heartbeat_steps_converge_quadratically():
    # three activation steps of the shell with the paper's law: exact Newton
    # converges quadratically in each (the tangent is the exact derivative)
    m = syn.shell_mesh(2, 6, 12)
    assert np.abs(np.einsum("ei,ei->e", m.elem_fibre, m.elem_sheet)).max() <= 1e-12
    C = syn.CARDIAC
    P = fem.guccione_problem(m, C, GUC)
    u, hists = newton.solve_heartbeat(P, syn.heartbeat_schedule()[:3], C["gamma_max"])
    for h in hists:
        r = np.array(h) / h[0]
        assert r[-1] <= 1e-10 and len(r) <= 8
        # the last step squares the relative residual (up to a constant): the
        # quadratic rate of Newton with the exact tangent
        assert r[-1] <= 50.0 * r[-2] ** 2, r
    assert np.abs(u).max() > 0.0
