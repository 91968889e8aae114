"""Pins of the oracle's surface loads on 6-node faces (the quadratic
heartbeat): a flat face sends the whole load to its edge midpoints (the
quadratic vertex functions integrate to zero), the pressure on a closed
surface is p times the gradient of the enclosed volume (zero net force and
moment), its Jacobian against central differences, and the face mass of the
springs against its exact integrals."""

import numpy as np

import synthetic as syn
from oracle import p2


def _cube_p2(n=2):
    m1 = syn.cube_mesh(n)
    m = syn.p2_from_p1(m1)
    X = m1.X
    tris = [syn.boundary_faces(X, m1.conn, np.isclose(X[:, d], v)) for d in range(3)
            for v in (0.0, 1.0)]
    tri = np.concatenate(tris)
    return m, p2.tri6_nodes(np.asarray(m.conn), tri)


def test_flat_faces_load_only_their_midpoints():
    m, t6 = _cube_p2(2)
    f = p2.p2_follower_pressure(m.X, np.zeros(3 * m.X.shape[0]), t6[:4], 0.7).reshape(-1, 3)
    assert np.abs(f[t6[:4, :3].reshape(-1)]).max() <= 1e-15
    # each face: p a / 3 at each midpoint, a its area vector
    a2 = np.cross(m.X[t6[0, 1]] - m.X[t6[0, 0]], m.X[t6[0, 2]] - m.X[t6[0, 0]])
    total = 0.7 * 0.5 * np.linalg.norm(a2) * 4
    assert abs(np.linalg.norm(f.sum(0)) - total) <= 1e-12 * total


def test_closed_surface_pressure_is_p_grad_volume_and_balanced():
    m, t6 = _cube_p2(2)
    rng = np.random.default_rng(3)
    u = 0.05 * rng.standard_normal(3 * m.X.shape[0])
    f = p2.p2_follower_pressure(m.X, u, t6, 1.3)
    F = f.reshape(-1, 3)
    x = m.X + u.reshape(-1, 3)
    assert np.abs(F.sum(0)).max() <= 1e-12 * np.abs(F).max()
    assert np.abs(np.cross(x, F).sum(0)).max() <= 1e-12 * np.abs(F).max()

    def volume(uu):
        # V = 1/3 int x . n dA over the quadratic faces (divergence theorem),
        # with n dA = (x_xi x x_eta) dxi deta, by the same exact rule
        xx = m.X + uu.reshape(-1, 3)
        pts, wts = p2._gauss_triangle(4)
        v = 0.0
        for nodes in t6:
            xf = xx[nodes]
            for (a, b), w in zip(pts, wts):
                N, dN = p2._tri6_shapes(a, b)
                v += w * (N @ xf) @ np.cross(dN[:, 0] @ xf, dN[:, 1] @ xf) / 3.0
        return v

    h = 1e-6
    for j in rng.choice(f.size, 6, replace=False):
        e = np.zeros_like(u)
        e[j] = h
        d = (volume(u + e) - volume(u - e)) / (2 * h)
        assert abs(1.3 * d - f[j]) <= 1e-6 * np.abs(f).max(), j


def test_pressure_jacobian_matches_central_differences():
    m, t6 = _cube_p2(1)
    rng = np.random.default_rng(4)
    u = 0.05 * rng.standard_normal(3 * m.X.shape[0])
    K = p2.p2_follower_pressure_jacobian(m.X, u, t6, 0.9)
    v = rng.standard_normal(u.size)
    h = 1e-6
    fd = (p2.p2_follower_pressure(m.X, u + h * v, t6, 0.9)
          - p2.p2_follower_pressure(m.X, u - h * v, t6, 0.9)) / (2 * h)
    assert np.abs(K @ v - fd).max() <= 1e-7 * np.abs(fd).max()


def test_spring_face_mass_against_exact_integrals():
    # on a flat 6-node triangle: int N_a N_b dA = A/180 (6, -1, 0, -4 pattern):
    # vertex-vertex 6 (same) / -1, vertex-midpoint 0 (adjacent edge) / -4
    # (opposite edge), midpoint-midpoint 32 (same) / 16
    X = np.array([[0.0, 0, 0], [2.0, 0, 0], [0.0, 1.5, 0], [1.0, 0, 0], [1.0, 0.75, 0],
                  [0.0, 0.75, 0]])
    t6 = np.array([[0, 1, 2, 3, 4, 5]])
    R = p2.p2_robin_matrix(X, t6, 1.0, 1.0).toarray()  # K = I: R = M (x) I
    M = R[::3, ::3]
    A = 0.5 * 2.0 * 1.5
    ref = np.array([[6, -1, -1, 0, -4, 0],
                    [-1, 6, -1, 0, 0, -4],
                    [-1, -1, 6, -4, 0, 0],
                    [0, 0, -4, 32, 16, 16],
                    [-4, 0, 0, 16, 32, 16],
                    [0, -4, 0, 16, 16, 32]]) * A / 180.0
    assert np.abs(M - ref).max() <= 1e-14 * np.abs(ref).max()
    # normal springs: K = k_perp N (x) N + k_par (I - N (x) N), N = e_z here
    R2 = p2.p2_robin_matrix(X, t6, 3.0, 0.5).toarray()
    assert np.allclose(R2[2::3, 2::3], 3.0 * ref) and np.allclose(R2[0::3, 0::3], 0.5 * ref)


def test_shell_with_loads_consistent_and_reduces_to_p1_faces_at_rest():
    # residual = gradient of the potential for the springs' part, tangent
    # against central differences with the pressure, and at u = 0 the
    # pressure's nodal forces sum to the same resultant as on the P1 faces
    from oracle import fem

    m1 = syn.shell_mesh(2, 4, 8)
    mesh = syn.p2_from_p1(m1)
    C = dict(syn.CARDIAC)
    P = p2.shell_p2_problem(mesh, C, gamma=0.02, loads=True)
    rng = np.random.default_rng(8)
    u = P.lift(0.02 * rng.standard_normal(P.n_dofs))
    K = P.stiffness(u, dirichlet=False, load_scale=0.6)
    v = rng.standard_normal(P.n_dofs)
    h = 1e-6

    def rfree(x):
        re = P.element_residual(x[P.edofs])
        r = np.zeros(P.n_dofs)
        np.add.at(r, P.edofs.reshape(-1), re.reshape(-1))
        return r + P.surface_force(x, 0.6)

    fd = (rfree(u + h * v) - rfree(u - h * v)) / (2 * h)
    assert np.abs(K @ v - fd).max() <= 1e-6 * np.abs(fd).max()
    fp2 = p2.p2_follower_pressure(mesh.X, np.zeros(P.n_dofs), P.pressure_tri6, 1.0)
    fp1 = fem.follower_pressure(m1.X, np.zeros(3 * m1.n_nodes), np.asarray(m1.faces["endo"]), 1.0)
    assert np.allclose(fp2.reshape(-1, 3).sum(0), fp1.reshape(-1, 3).sum(0), rtol=1e-12,
                       atol=1e-12 * np.abs(fp1).sum())
