"""Pins of the oracle's implicit dynamics (lumped mass, Newmark's average
acceleration rule): the lumped mass equals density times volume; the
residual with inertia is the gradient of the incremental potential; and a
small-amplitude free vibration follows the linear average-acceleration
recursion written out with the independent small-strain stiffness (which
conserves the energy exactly)."""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle import fem, linear, newton

MU, LAM = 80.194, 400.9


def test_lumped_mass_total():
    m = syn.cook_mesh(3, 3, 1)
    P = fem.cook_problem(m, mu=MU, lam=LAM)
    M = P.lumped_mass(1.3e-3).reshape(-1, 3)
    assert np.allclose(M.sum(0), 1.3e-3 * 14400.0, rtol=1e-13)


def test_inertia_residual_is_gradient_of_incremental_potential():
    m = syn.cook_mesh(3, 3, 1)
    P = fem.cook_problem(m, mu=MU, lam=LAM)
    rng = np.random.default_rng(4)
    ut = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    P.set_inertia(1e-3, 2.5e3, ut)
    u = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    w = rng.standard_normal(P.n_dofs)
    w[P.fixed] = 0.0
    h = 1e-6
    d = (P.energy(u + h * w, 0.6) - P.energy(u - h * w, 0.6)) / (2 * h)
    assert abs(d - P.residual(u, 0.6) @ w) <= 1e-7 * abs(d)
    K = P.stiffness(u, dirichlet=False)
    fd = (P.residual(u + h * w, 0.6) - P.residual(u - h * w, 0.6)) / (2 * h)
    fd[P.fixed] = 0.0
    Kw = K @ w
    Kw[P.fixed] = 0.0
    assert np.abs(Kw - fd).max() <= 1e-6 * np.abs(fd).max()


def test_small_amplitude_vibration_follows_linear_newmark():
    # at strains ~1e-7 the nonlinear step is the linear one: compare with
    # M u'' + K0 u = 0 stepped by the average-acceleration rule written out
    # with the independent small-strain stiffness K0, and check that this
    # linear trajectory keeps its energy (the rule conserves it exactly)
    m = syn.cook_mesh(4, 4, 1)
    P = fem.cook_problem(m, mu=MU, lam=LAM, tau=0.0)
    rho, dt, beta, gamma = 1e-3, 2e-3, 0.25, 0.5
    rng = np.random.default_rng(6)
    v0 = 1e-5 * rng.standard_normal(P.n_dofs)
    v0[P.fixed] = 0.0
    M = P.lumped_mass(rho)
    free = P.free
    K0 = linear.stiffness_linear(m.X, m.conn, LAM, MU).tocsc()[free][:, free]
    Mf = M[free]
    c = 1.0 / (beta * dt * dt)
    A = (K0 + sp.diags(c * Mf)).tocsc()
    ul, vl, al = np.zeros(free.sum()), v0[free].copy(), np.zeros(free.sum())
    e_lin0 = 0.5 * float(np.sum(Mf * vl * vl))
    u, v, a = np.zeros(P.n_dofs), v0.copy(), np.zeros(P.n_dofs)
    for _ in range(10):
        ut = newton.newmark_predict(u, v, a, dt, beta)
        P.set_inertia(rho, c, ut)
        u, _ = newton.newton_exact(P, u, 1.0, rtol=1e-14)
        v, a = newton.newmark_correct(u, ut, v, a, dt, beta, gamma)
        utl = ul + dt * vl + dt * dt * (0.5 - beta) * al
        ul = spla.spsolve(A, c * Mf * utl)
        anew = c * (ul - utl)
        vl = vl + dt * ((1 - gamma) * al + gamma * anew)
        al = anew
    P.set_inertia(0.0, 0.0, u)
    assert np.linalg.norm(u[free] - ul) <= 1e-5 * np.linalg.norm(ul)
    assert np.linalg.norm(v[free] - vl) <= 1e-5 * np.linalg.norm(vl)
    e_lin = 0.5 * float(np.sum(Mf * vl * vl)) + 0.5 * float(ul @ (K0 @ ul))
    assert abs(e_lin - e_lin0) <= 1e-10 * e_lin0


def test_damped_vibration_follows_linear_newmark_and_dissipates():
    # dashpots on the x = 48 face: at strains ~1e-7 the nonlinear implicit
    # steps equal the linear recursion written out with the independent
    # small-strain stiffness K0 and the face damping matrix C, which loses
    # energy at exactly the rate the trapezoidal rule implies,
    # E_{n+1} - E_n = -(dt/4) (v_n + v_{n+1})^T C (v_n + v_{n+1})
    m = syn.cook_mesh(4, 4, 1)
    base = fem.cook_problem(m, mu=MU, lam=LAM, tau=0.0)
    P = fem.Problem(base.X, base.conn, base.material, base.params, base.f_ext, base.ddofs,
                    base.dvals, robin_tri=m.faces["load"], k_perp=0.0, k_par=0.0)
    c_perp, c_par = 40.0, 10.0
    P.set_robin_damping(c_perp, c_par)
    rho, dt, beta, gamma = 1e-3, 2e-3, 0.25, 0.5
    c, cv = 1.0 / (beta * dt * dt), gamma / (beta * dt)
    rng = np.random.default_rng(7)
    v0 = 1e-5 * rng.standard_normal(P.n_dofs)
    v0[P.fixed] = 0.0
    M = P.lumped_mass(rho)
    free = P.free
    K0 = linear.stiffness_linear(m.X, m.conn, LAM, MU).tocsc()[free][:, free]
    C = fem.robin_matrix(m.X, m.faces["load"], c_perp, c_par).tocsc()[free][:, free]
    Mf = M[free]
    a0 = np.zeros(P.n_dofs)
    a0[free] = -(C @ v0[free]) / Mf  # consistent start at u = 0
    A = (K0 + sp.diags(c * Mf) + cv * C).tocsc()
    ul, vl, al = np.zeros(free.sum()), v0[free].copy(), a0[free].copy()
    u, v, a = np.zeros(P.n_dofs), v0.copy(), a0.copy()
    energy = lambda uu, vv: 0.5 * float(np.sum(Mf * vv * vv)) + 0.5 * float(uu @ (K0 @ uu))
    e_prev, lost = energy(ul, vl), 0.0
    for _ in range(10):
        ut = newton.newmark_predict(u, v, a, dt, beta)
        P.set_inertia(rho, c, ut)
        P.set_step_velocity(cv, v + dt * (1.0 - gamma) * a)
        u, _ = newton.newton_exact(P, u, 1.0, rtol=1e-14)
        v, a = newton.newmark_correct(u, ut, v, a, dt, beta, gamma)
        utl = ul + dt * vl + dt * dt * (0.5 - beta) * al
        vtl = vl + dt * (1.0 - gamma) * al
        vold = vl
        ul = spla.spsolve(A, c * Mf * utl + C @ (cv * utl - vtl))
        anew = c * (ul - utl)
        vl = vl + dt * ((1 - gamma) * al + gamma * anew)
        al = anew
        vb = vold + vl
        d = -0.25 * dt * float(vb @ (C @ vb))
        e_new = energy(ul, vl)
        assert abs((e_new - e_prev) - d) <= 1e-9 * e_prev
        lost -= d
        e_prev = e_new
    assert lost > 1e-3 * energy(np.zeros_like(ul), v0[free])  # the dashpots matter
    assert np.linalg.norm(u[free] - ul) <= 1e-5 * np.linalg.norm(ul)
    assert np.linalg.norm(v[free] - vl) <= 1e-5 * np.linalg.norm(vl)


def test_dashpot_force_is_the_spring_force_of_the_step_velocity():
    # with the dashpot coefficients equal to spring coefficients, the dashpot
    # force at velocity v~ + cv (u - u~) equals that spring matrix applied to
    # the velocity; the dashpot tangent is cv times it, symmetric and
    # positive semidefinite (one zero mode per off-face dof)
    C = syn.CARDIAC
    mesh = syn.shell_mesh(2, 6, 12)
    P = fem.cardiac_problem(mesh, C)
    rng = np.random.default_rng(11)
    ut = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    vt = 0.1 * rng.standard_normal(P.n_dofs)
    u = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    cv = 37.0
    P.set_inertia(1e-7, 2.5e3, ut)
    r0 = P.residual(u, 0.4)
    P.set_robin_damping(3.0 * C["k_perp"], 5.0 * C["k_par"])
    P.set_step_velocity(cv, vt)
    r1 = P.residual(u, 0.4)
    Rc = fem.robin_matrix(mesh.X, mesh.faces["epi"], 3.0 * C["k_perp"], 5.0 * C["k_par"])
    expect = Rc @ (vt + cv * (u - ut))
    expect[P.fixed] = 0.0
    assert np.abs((r1 - r0) - expect).max() <= 1e-12 * np.abs(expect).max()
    K1 = P.stiffness(u, load_scale=0.4).toarray()
    P.set_robin_damping(0.0, 0.0)
    K0 = P.stiffness(u, load_scale=0.4).toarray()
    free = P.free
    # the difference of two tangents carries their rounding (~1e-16 of |K|)
    tol = 1e-13 * np.abs(K0).max()
    D = (K1 - K0)[np.ix_(free, free)]
    Dref = cv * Rc.toarray()[np.ix_(free, free)]
    assert np.abs(D - Dref).max() <= tol
    assert np.abs(Dref - Dref.T).max() <= 1e-14 * np.abs(Dref).max()
    assert np.linalg.eigvalsh(Dref).min() >= -1e-12 * np.abs(Dref).max()
