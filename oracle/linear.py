"""Textbook small-strain linear elasticity on P1 tetrahedra (independent pin).

Standard displacement-based finite elements: Voigt strain
eps = (e11, e22, e33, 2e23, 2e13, 2e12) = B u_e, isotropic constitutive
matrix D(lambda, mu), element stiffness V B^T D B.  None of the nonlinear
code (materials, complex-step tangent, residual assembly) is used, so the
nonlinear tangent at u = 0 can be checked against this one.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def voigt_D(lam: float, mu: float) -> np.ndarray:
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2.0 * mu
    D[3:, 3:] = mu * np.eye(3)
    return D


def _tet_gradients(Xe: np.ndarray):
    """Gradients of the four linear shape functions by solving the 4x4 system
    [1 x y z] c = e_a (the classic coefficient approach), and the volume."""
    M = np.concatenate([np.ones((4, 1)), Xe], axis=1)
    C = np.linalg.inv(M)  # column a: coefficients of N_a
    vol = abs(np.linalg.det(M)) / 6.0
    return C[1:, :].T, vol  # (4, 3)


def stiffness_linear(X: np.ndarray, conn: np.ndarray, lam: float, mu: float) -> sp.csr_matrix:
    D = voigt_D(lam, mu)
    n = X.shape[0]
    rows, cols, vals = [], [], []
    for e in range(conn.shape[0]):
        c = conn[e, :4]
        g, vol = _tet_gradients(X[c])
        B = np.zeros((6, 12))
        for a in range(4):
            gx, gy, gz = g[a]
            B[0, 3 * a + 0] = gx
            B[1, 3 * a + 1] = gy
            B[2, 3 * a + 2] = gz
            B[3, 3 * a + 1] = gz
            B[3, 3 * a + 2] = gy
            B[4, 3 * a + 0] = gz
            B[4, 3 * a + 2] = gx
            B[5, 3 * a + 0] = gy
            B[5, 3 * a + 1] = gx
        Ke = vol * B.T @ D @ B
        dofs = (3 * c[:, None] + np.arange(3)[None, :]).reshape(-1)
        rows.append(np.repeat(dofs, 12))
        cols.append(np.tile(dofs, 12))
        vals.append(Ke.reshape(-1))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * n, 3 * n)).tocsr()


# ---- quadratic displacement / linear pressure (independent of mixed.py) ----
def _duffy_rule(n: int = 3):
    """Points and weights on the unit tetrahedron {x, y, z >= 0, x+y+z <= 1}
    from an n^3 Gauss-Legendre rule on the cube mapped by the collapsed
    (Duffy) coordinates z = c, y = b (1 - c), x = a (1 - b)(1 - c), Jacobian
    (1 - b)(1 - c)^2.  n = 3 integrates every quadratic exactly."""
    t, w = np.polynomial.legendre.leggauss(n)
    t = 0.5 * (t + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            for k in range(n):
                a, b, c = t[i], t[j], t[k]
                pts.append((a * (1 - b) * (1 - c), b * (1 - c), c))
                wts.append(w[i] * w[j] * w[k] * (1 - b) * (1 - c) ** 2)
    return np.array(pts), np.array(wts)


def _quadratic_basis_gradients(Xn: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Gradients at pts of the Lagrange basis through the ten nodes Xn, built
    from monomials 1, x, y, z, x^2, y^2, z^2, xy, xz, yz (Vandermonde solve).
    Returns (n_pts, 10, 3)."""
    def mono(x):
        return np.array([1, x[0], x[1], x[2], x[0] ** 2, x[1] ** 2, x[2] ** 2,
                         x[0] * x[1], x[0] * x[2], x[1] * x[2]])

    def dmono(x):
        z = np.zeros(10)
        gx, gy, gz = z.copy(), z.copy(), z.copy()
        gx[1], gy[2], gz[3] = 1, 1, 1
        gx[4], gy[5], gz[6] = 2 * x[0], 2 * x[1], 2 * x[2]
        gx[7], gy[7] = x[1], x[0]
        gx[8], gz[8] = x[2], x[0]
        gy[9], gz[9] = x[2], x[1]
        return np.stack([gx, gy, gz], axis=1)  # (10 monomials, 3)

    Vd = np.array([mono(x) for x in Xn])  # rows: nodes
    C = np.linalg.inv(Vd)                 # column a: coefficients of basis a
    return np.array([C.T @ dmono(x) for x in pts])


def stiffness_linear_p2(X: np.ndarray, conn10: np.ndarray, lam: float, mu: float) -> sp.csr_matrix:
    """Small-strain elasticity with quadratic tetrahedra (B^T D B, exact rule)."""
    D = voigt_D(lam, mu)
    ref, wref = _duffy_rule(3)
    n = X.shape[0]
    rows, cols, vals = [], [], []
    for e in range(conn10.shape[0]):
        c = conn10[e]
        Xe = X[c]
        J = np.stack([Xe[1] - Xe[0], Xe[2] - Xe[0], Xe[3] - Xe[0]], axis=1)
        det = abs(np.linalg.det(J))
        pts = Xe[0][None, :] + ref @ J.T
        g = _quadratic_basis_gradients(Xe, pts)
        Ke = np.zeros((30, 30))
        for q in range(pts.shape[0]):
            B = np.zeros((6, 30))
            for a in range(10):
                gx, gy, gz = g[q, a]
                B[0, 3 * a] = gx
                B[1, 3 * a + 1] = gy
                B[2, 3 * a + 2] = gz
                B[3, 3 * a + 1], B[3, 3 * a + 2] = gz, gy
                B[4, 3 * a], B[4, 3 * a + 2] = gz, gx
                B[5, 3 * a], B[5, 3 * a + 1] = gy, gx
            Ke += wref[q] * det * B.T @ D @ B
        dofs = (3 * c[:, None] + np.arange(3)[None, :]).reshape(-1)
        rows.append(np.repeat(dofs, 30))
        cols.append(np.tile(dofs, 30))
        vals.append(Ke.reshape(-1))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(3 * n, 3 * n)).tocsr()


def divergence_p2p1(X: np.ndarray, conn10: np.ndarray, pconn: np.ndarray, n_p: int) -> sp.csr_matrix:
    """B[b, (a, i)] = -int q_b d(N_a)/dx_i (linear pressure hat q_b, quadratic
    displacement basis N_a), exact rule; shape (n_p, 3 n_u)."""
    ref, wref = _duffy_rule(3)
    rows, cols, vals = [], [], []
    for e in range(conn10.shape[0]):
        c = conn10[e]
        Xe = X[c]
        J = np.stack([Xe[1] - Xe[0], Xe[2] - Xe[0], Xe[3] - Xe[0]], axis=1)
        det = abs(np.linalg.det(J))
        pts = Xe[0][None, :] + ref @ J.T
        g = _quadratic_basis_gradients(Xe, pts)
        M = np.concatenate([np.ones((4, 1)), Xe[:4]], axis=1)
        Cq = np.linalg.inv(M)  # column b: coefficients of the linear hat of vertex b
        Be = np.zeros((4, 30))
        for q in range(pts.shape[0]):
            hat = np.concatenate([[1.0], pts[q]]) @ Cq
            for b in range(4):
                Be[b] -= wref[q] * det * hat[b] * g[q].reshape(-1)
        rows.append(np.repeat(pconn[e], 30))
        cols.append(np.tile((3 * c[:, None] + np.arange(3)[None, :]).reshape(-1), 4))
        vals.append(Be.reshape(-1))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n_p, 3 * X.shape[0])).tocsr()


def divergence_p2p0(X: np.ndarray, conn10: np.ndarray) -> sp.csr_matrix:
    """B[e, (a, i)] = -int_e d(N_a)/dx_i (pressure constant on element e,
    quadratic displacement basis N_a), exact rule; shape (n_e, 3 n_u)."""
    ref, wref = _duffy_rule(3)
    rows, cols, vals = [], [], []
    for e in range(conn10.shape[0]):
        c = conn10[e]
        Xe = X[c]
        J = np.stack([Xe[1] - Xe[0], Xe[2] - Xe[0], Xe[3] - Xe[0]], axis=1)
        det = abs(np.linalg.det(J))
        pts = Xe[0][None, :] + ref @ J.T
        g = _quadratic_basis_gradients(Xe, pts)
        Be = -np.einsum("q,qai->ai", wref * det, g).reshape(-1)
        rows.append(np.full(30, e))
        cols.append((3 * c[:, None] + np.arange(3)[None, :]).reshape(-1))
        vals.append(Be)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(conn10.shape[0], 3 * X.shape[0])).tocsr()
