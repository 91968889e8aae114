"""Pins of the oracle's Jacobi-type preconditioners (point and nodal block).

Checks against what the mathematics fixes, not the extraction code itself:
the blocks at u = 0 equal those of the independent textbook small-strain
assembly, and for one tetrahedron they equal the closed form
V [mu (g.g) I + (mu + lambda) g g^T]; the follower-pressure part of a node's
own block is skew-symmetric (so the symmetric part of the cardiac block is
the strain-energy and spring part); Dirichlet dofs give identity rows and
columns; and block Jacobi equals point Jacobi when every block is diagonal.
"""

import numpy as np
import scipy.sparse as sp

import synthetic as syn
from oracle import fem, linear, precond

MU, LAM = 80.194, 400.9


def test_blocks_at_rest_match_textbook_assembly():
    mesh = syn.cook_mesh(3, 3, 1)
    P = fem.cook_problem(mesh, mu=MU, lam=LAM)
    K = P.stiffness(np.zeros(P.n_dofs), dirichlet=False)
    Kl = linear.stiffness_linear(mesh.X, mesh.conn, LAM, MU)
    B = precond.node_blocks(K, mesh.X.shape[0])
    Bl = precond.node_blocks(Kl, mesh.X.shape[0])
    assert np.abs(B - Bl).max() <= 1e-12 * np.abs(Bl).max()


def test_single_tet_block_closed_form():
    X = np.array([[0.0, 0.0, 0.0], [1.2, 0.1, 0.0], [0.2, 0.9, 0.1], [0.1, 0.3, 1.1]])
    conn = np.array([[0, 1, 2, 3]])
    M = np.concatenate([np.ones((4, 1)), X], axis=1)
    C = np.linalg.inv(M)
    g = C[1:, :].T  # (4, 3) shape-function gradients
    V = np.linalg.det(M) / 6.0
    Kl = linear.stiffness_linear(X, conn, LAM, MU)
    B = precond.node_blocks(Kl, 4)
    for a in range(4):
        ref = V * (MU * (g[a] @ g[a]) * np.eye(3) + (MU + LAM) * np.outer(g[a], g[a]))
        assert np.abs(B[a] - ref).max() <= 1e-12 * np.abs(ref).max()


def test_pressure_self_block_is_skew():
    mesh = syn.shell_mesh(2, 6, 12)
    C = syn.CARDIAC
    P = fem.cardiac_problem(mesh, C, gamma=0.02)
    rng = np.random.default_rng(5)
    u = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    tri = np.asarray(P.pressure_tri)
    Kp = fem.follower_pressure_jacobian(P.X, u, tri, 1.7).tocsr()
    nodes = np.unique(tri)
    blks = np.array([Kp[3 * k:3 * k + 3, 3 * k:3 * k + 3].toarray() for k in nodes])
    scale = np.abs(blks).max()
    # (inside a closed fan of faces the self blocks cancel to rounding level,
    # so the check is relative to the largest block)
    assert np.abs(blks + blks.transpose(0, 2, 1)).max() < 1e-12 * scale
    # and it is not zero: the symmetric part really drops something
    assert scale > 0


def test_dirichlet_identity_and_point_limit():
    mesh = syn.cook_mesh(3, 3, 1)
    P = fem.cook_problem(mesh, mu=MU, lam=LAM)
    rng = np.random.default_rng(3)
    u = P.lift(0.01 * rng.standard_normal(P.n_dofs))
    K = P.stiffness(u)
    B = precond.node_blocks(K, mesh.X.shape[0])
    fixed = P.fixed.reshape(-1, 3)
    for k in np.flatnonzero(fixed.all(axis=1)):
        assert np.array_equal(B[k], np.eye(3))
    # a block-diagonal matrix with diagonal blocks: block Jacobi = point Jacobi
    d = 1.0 + rng.random(P.n_dofs)
    D = sp.diags(d).tocsr()
    x = rng.standard_normal(P.n_dofs)
    zb = precond.block_jacobi_apply(precond.node_blocks(D, mesh.X.shape[0]), x)
    assert np.abs(zb - x / d).max() <= 1e-15 * np.abs(x / d).max()


def test_pcg_with_block_jacobi_solves_the_system():
    mesh = syn.cook_mesh(4, 4, 1)
    P = fem.cook_problem(mesh, mu=MU, lam=LAM)
    rng = np.random.default_rng(9)
    u = P.lift(0.005 * rng.standard_normal(P.n_dofs))
    K = P.stiffness(u)
    b = rng.standard_normal(P.n_dofs)
    b[P.fixed] = 0.0
    B = precond.node_blocks(K, mesh.X.shape[0])
    x, its = precond.pcg(K, b, lambda r: precond.block_jacobi_apply(B, r), rtol=1e-12)
    xd = sp.linalg.spsolve(K.tocsc(), b)
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    xp, itp = precond.pcg(K, b, lambda r: precond.point_jacobi_apply(K, r), rtol=1e-12)
    assert np.linalg.norm(xp - xd) <= 1e-9 * np.linalg.norm(xd)
    assert its < 400 and itp < 400


def test_indefinite_block_falls_back_to_its_diagonal():
    # an indefinite block (eigenvalues 3, -1, 2) next to an SPD one
    Bi = np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 0.0], [0.0, 0.0, 2.0]])
    Bs = np.array([[4.0, 1.0, 0.0], [1.0, 3.0, 0.5], [0.0, 0.5, 2.0]])
    x = np.array([1.0, -2.0, 0.5, 0.3, 0.7, -1.1])
    z = precond.block_jacobi_apply(np.stack([Bi, Bs]), x)
    assert np.allclose(z[:3], x[:3] / np.diag(Bi), rtol=1e-15)
    assert np.allclose(Bs @ z[3:], x[3:], rtol=1e-14)
