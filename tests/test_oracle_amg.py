"""Pins of the oracle's aggregation multigrid (oracle/amg.py) against what
the definition and the mathematics fix: the aggregation's structure (roots
with their whole neighbourhood, members within distance two of the root,
roots three apart), orthonormal tentative prolongators whose range holds
every rigid motion, Galerkin coarse operators that annihilate the coarse
rigid modes of a floating body, a one-level hierarchy that is the exact
solve, a symmetric positive definite cycle for a symmetric positive definite
tangent with a convergent error propagator, the power-iteration estimate
against the spectrum, and fewer Krylov iterations than point Jacobi."""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synthetic as syn
from oracle import amg, fem

MU = 80.194


def _cook(nx, ny, nz, ratio=5.0, dirichlet=True):
    mesh = syn.cook_mesh(nx, ny, nz)
    P = fem.cook_problem(mesh, mu=MU, lam=ratio * MU, tau=1.0)
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=dirichlet)
    fixed = P.fixed if dirichlet else np.zeros(P.n_dofs, dtype=bool)
    return mesh, P, K, fixed


def test_start_vector_is_the_golden_ratio_sequence():
    # 2654435761 / 2^32 is the fractional part of the golden ratio to 2e-9
    x = amg.start_vector(3)
    assert x[0] == -0.5
    assert abs(x[1] - ((np.sqrt(5.0) - 1.0) / 2.0 - 0.5)) < 2.5e-9
    assert abs(x[2] - ((2.0 * (np.sqrt(5.0) - 1.0) / 2.0) % 1.0 - 0.5)) < 5e-9


def test_aggregation_structure():
    mesh = syn.cook_mesh(8, 6, 2)
    adj = amg.node_graph(mesh.conn, mesh.n_nodes)
    agg, n_agg = amg.aggregate(adj)
    assert agg.min() == 0 and set(agg.tolist()) == set(range(n_agg))
    roots = []
    for a in range(n_agg):
        mem = set(np.flatnonzero(agg == a).tolist())
        # a root: a member whose closed neighbourhood lies in the aggregate
        cand = [v for v in sorted(mem) if set(adj[v]) <= mem]
        assert cand, a
        r = cand[0]
        roots.append(r)
        ring1 = set(adj[r])
        ring2 = set(w for v in ring1 for w in adj[v])
        assert mem <= {r} | ring1 | ring2
    # roots' neighbourhoods are disjoint (pass 1): distinct roots are >= 3 apart
    for i, r in enumerate(roots):
        n1 = {r} | set(adj[r])
        for s in roots[i + 1:]:
            assert not (n1 & ({s} | set(adj[s])))


def test_prolongator_orthonormal_and_spans_rigid_motions():
    mesh, P, K, fixed = _cook(8, 6, 2)
    H = amg.setup(K, mesh.X, mesh.conn, fixed)
    P0 = H.P[0].toarray()
    assert np.abs(P0.T @ P0 - np.eye(P0.shape[1])).max() < 1e-12
    rng = np.random.default_rng(3)
    for _ in range(3):
        t, w = rng.standard_normal(3), rng.standard_normal(3)
        u = (t[None, :] + np.cross(w[None, :], mesh.X)).reshape(-1)
        u[fixed] = 0.0
        assert np.linalg.norm(P0 @ (P0.T @ u) - u) <= 1e-12 * np.linalg.norm(u)
    # Dirichlet rows are zero
    assert np.abs(P0[fixed]).max() == 0.0


def test_galerkin_operators_annihilate_coarse_rigid_modes():
    # a floating body at rest: K annihilates rigid motions, hence every
    # coarse operator annihilates their coarse representation
    mesh, P, K, fixed = _cook(20, 16, 3, dirichlet=False)
    H = amg.setup(K, mesh.X, mesh.conn, fixed)
    assert H.n_levels >= 3
    rng = np.random.default_rng(4)
    t, w = rng.standard_normal(3), rng.standard_normal(3)
    u = (t[None, :] + np.cross(w[None, :], mesh.X)).reshape(-1)
    assert np.linalg.norm(K @ u) <= 1e-10 * abs(K).max() * np.linalg.norm(u)
    v = u
    for lev in range(H.n_levels - 1):
        v = H.P[lev].T @ v  # P is orthonormal and spans v: this is its coordinates
        assert np.linalg.norm(H.P[lev] @ v - (u if lev == 0 else vprev)) <= 1e-10 * np.linalg.norm(v)
        A = H.A[lev + 1]
        assert np.linalg.norm(A @ v) <= 1e-9 * abs(A).max() * np.linalg.norm(v)
        vprev = v


def test_one_level_is_the_exact_solve(monkeypatch):
    mesh, P, K, fixed = _cook(4, 4, 1)
    monkeypatch.setattr(amg, "N_COARSE", 10 ** 6)
    H = amg.setup(K, mesh.X, mesh.conn, fixed)
    assert H.n_levels == 1
    b = np.random.default_rng(5).standard_normal(P.n_dofs)
    x = amg.vcycle(H, b)
    assert np.linalg.norm(K @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_cycle_is_spd_and_convergent_for_an_spd_tangent():
    mesh, P, K, fixed = _cook(8, 8, 1)
    H = amg.setup(K, mesh.X, mesh.conn, fixed)
    assert H.n_levels == 2
    n = P.n_dofs
    M = np.column_stack([amg.vcycle(H, e) for e in np.eye(n)])
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    # error propagation I - M K has spectral radius < 1
    Kd = K.toarray()
    rho = np.abs(np.linalg.eigvals(np.eye(n) - M @ Kd)).max()
    assert rho < 1.0, rho


def test_power_iteration_brackets_the_spectral_radius():
    mesh, P, K, fixed = _cook(8, 8, 1)
    D = K.diagonal()
    lam = np.abs(np.linalg.eigvals(np.diag(1.0 / D) @ K.toarray())).max()
    est = amg.spectral_radius(K, D)
    assert 0.8 * lam <= est <= lam * (1.0 + 1e-12), (est, lam)
    # a diagonal matrix with one dominant entry: the estimate converges to it
    A = sp.diags(np.r_[np.ones(20), 10.0])
    assert abs(amg.spectral_radius(A, np.ones(21)) - 10.0) < 1e-9


def test_fewer_iterations_than_point_jacobi():
    mesh, P, K, fixed = _cook(16, 16, 2)
    b = -P.residual(np.zeros(P.n_dofs), 1.0)
    H = amg.setup(K, mesh.X, mesh.conn, fixed)
    x, it = amg.gmres_amg(K, H, b, 1e-8, max_it=800)
    assert np.linalg.norm(b - K @ x) <= 1.01e-8 * np.linalg.norm(b)
    # point-Jacobi GMRES with the same (true residual) stopping rule
    cnt = [0]
    Mj = spla.LinearOperator(K.shape, matvec=lambda v: v / K.diagonal())
    spla.gmres(K, b, M=Mj, rtol=1e-8, restart=3000, maxiter=1,
               callback=lambda r: cnt.__setitem__(0, cnt[0] + 1), callback_type="pr_norm")
    assert 3 * it < cnt[0], (it, cnt[0])


def test_chebyshev_smoother_follows_the_chebyshev_polynomial():
    # on A = diag(lambda), D = I, the error after k steps from x = 0 is
    # T_k((theta - lambda) / delta) / T_k(theta / delta) times the exact solution
    rng = np.random.default_rng(9)
    rho = 3.7
    hi = amg.CHEB_SAFETY * rho
    lo = hi / amg.CHEB_RATIO
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    lam = np.r_[rng.uniform(lo, hi, 40), 0.5 * lo, 0.9 * lo]
    A = sp.diags(lam)
    xs = rng.standard_normal(lam.size)
    b = lam * xs
    for k in (1, 2, 3):
        x = amg.chebyshev(A, np.ones(lam.size), b, np.zeros(lam.size), rho, degree=k)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(k)
        factor = Tk((theta - lam) / delta) / Tk(theta / delta)
        assert np.allclose(xs - x, factor * xs, rtol=1e-10, atol=1e-12), k
        # inside the interval the error shrinks by at least 1 / T_k(theta / delta)
        inside = (lam >= lo) & (lam <= hi)
        assert np.all(np.abs(factor[inside]) <= 1.0 / abs(Tk(theta / delta)) + 1e-12)


def test_quadratic_mesh_hierarchy_keeps_rigid_motions():
    # quadratic elements: the node graph joins all ten nodes of an element; the
    # prolongator still spans every rigid motion and the Galerkin operators of a
    # floating body annihilate them (quadratic fields contain the rigid motions)
    from oracle import p2
    m = syn.cook_p2_mesh(6, 4, 1)
    P = p2.cook_p2_problem(m, mu=MU, lam=5.0 * MU)
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False).tocsr()
    adj = amg.node_graph(np.asarray(m.conn), m.X.shape[0])
    conn = np.asarray(m.conn)
    for e in (0, conn.shape[0] // 2, conn.shape[0] - 1):
        for a in conn[e]:
            assert set(conn[e].tolist()) - {a} <= set(adj[a])
    fixed = np.zeros(P.n_dofs, dtype=bool)
    H = amg.setup(K, m.X, conn, fixed)
    assert H.n_levels >= 2
    P0 = H.P[0].toarray()
    rng = np.random.default_rng(12)
    t, w = rng.standard_normal(3), rng.standard_normal(3)
    u = (t[None, :] + np.cross(w[None, :], m.X)).reshape(-1)
    assert np.linalg.norm(K @ u) <= 1e-10 * abs(K).max() * np.linalg.norm(u)
    assert np.linalg.norm(P0 @ (P0.T @ u) - u) <= 1e-12 * np.linalg.norm(u)
    vc = P0.T @ u
    assert np.linalg.norm(H.A[1] @ vc) <= 1e-9 * abs(H.A[1]).max() * np.linalg.norm(vc)


def test_pressure_block_of_the_field_split_is_the_lumped_mass():
    # the field split scales pressures by the lumped P1 pressure mass: row sums
    # of the consistent mass, integral of phi_i phi_j = V (1 + delta_ij) / 20 on
    # a tetrahedron, whose total is the domain's volume (the unit cube)
    from oracle import mixed
    m = syn.twist_p2_mesh(2)
    P = mixed.twist_problem(m, 1.0, 0.0)
    ml = P.pressure_mass_lumped()
    assert abs(ml.sum() - 1.0) < 1e-13 and ml.min() > 0.0
    pconn = np.asarray(m.pconn)
    Xv = np.zeros((P.n_p, 3))
    # pressure nodes sit at the elements' vertices (the first four displacement nodes)
    Xv[pconn.reshape(-1)] = m.X[np.asarray(m.conn)[:, :4].reshape(-1)]
    Mc = np.zeros((P.n_p, P.n_p))
    for e in range(pconn.shape[0]):
        x = Xv[pconn[e]]
        V = abs(np.linalg.det(np.column_stack([x[1] - x[0], x[2] - x[0], x[3] - x[0]]))) / 6.0
        Mc[np.ix_(pconn[e], pconn[e])] += V * (np.ones((4, 4)) + np.eye(4)) / 20.0
    assert np.allclose(Mc.sum(1), ml, rtol=1e-13, atol=0.0)


# ---------------------------------------------------- smoothed aggregation
def test_smoothed_prolongator_reproduces_rigid_motions_on_a_floating_body():
    # A annihilates the rigid motions, so one Jacobi step leaves them alone:
    # P_s (coarse coordinates of a rigid motion) = the rigid motion
    mesh, P, K, fixed = _cook(12, 10, 2, dirichlet=False)
    Ht = amg.setup(K, mesh.X, mesh.conn, fixed)
    Hs = amg.setup(K, mesh.X, mesh.conn, fixed, smooth=True)
    rng = np.random.default_rng(6)
    t, w = rng.standard_normal(3), rng.standard_normal(3)
    u = (t[None, :] + np.cross(w[None, :], mesh.X)).reshape(-1)
    c = Ht.P[0].T @ u  # coordinates in the tentative (orthonormal) basis
    assert np.linalg.norm(Ht.P[0] @ c - u) <= 1e-10 * np.linalg.norm(u)
    assert np.linalg.norm(Hs.P[0] @ c - u) <= 1e-9 * np.linalg.norm(u)
    # and the Galerkin operator annihilates them
    A1 = Hs.A[1]
    assert np.linalg.norm(A1 @ c) <= 1e-9 * abs(A1).max() * np.linalg.norm(c)
    assert abs(A1 - A1.T).max() <= 1e-12 * abs(A1).max()


def test_smoothing_lowers_every_prolongator_columns_energy():
    # |1 - omega lambda| <= 1 on the spectrum of D^-1 A (omega rho = 4/3 with
    # rho the power estimate, which falls short of the true radius by a few
    # percent at most), so no column's A-energy rises, and the total drops
    mesh, P, K, fixed = _cook(10, 8, 2)
    Ht = amg.setup(K, mesh.X, mesh.conn, fixed)
    Hs = amg.setup(K, mesh.X, mesh.conn, fixed, smooth=True)
    Pt, Ps = Ht.P[0], Hs.P[0]
    et = np.asarray((Pt.multiply(K @ Pt)).sum(axis=0)).ravel()
    es = np.asarray((Ps.multiply(K @ Ps)).sum(axis=0)).ravel()
    keep = et > 1e-12 * et.max()
    assert np.all(es[keep] <= et[keep] * (1.0 + 1e-12))
    assert es.sum() < 0.7 * et.sum(), (es.sum(), et.sum())
    # the smoothed columns reach one node ring beyond their aggregates
    assert Ps.nnz > 1.5 * Pt.nnz


def test_smoothed_cycle_is_spd_and_needs_fewer_iterations():
    mesh, P, K, fixed = _cook(8, 8, 1)
    Hs = amg.setup(K, mesh.X, mesh.conn, fixed, smooth=True)
    n = P.n_dofs
    M = np.column_stack([amg.vcycle(Hs, e) for e in np.eye(n)])
    assert np.abs(M - M.T).max() <= 1e-12 * np.abs(M).max()
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    mesh, P, K, fixed = _cook(16, 16, 2, ratio=500.0)
    b = -P.residual(np.zeros(P.n_dofs), 1.0)
    its = []
    for smooth in (False, True):
        H = amg.setup(K, mesh.X, mesh.conn, fixed, smooth=smooth)
        x, it = amg.gmres_amg(K, H, b, 1e-8, max_it=800)
        assert np.linalg.norm(b - K @ x) <= 1.01e-8 * np.linalg.norm(b)
        its.append(it)
    assert its[1] < its[0], its
