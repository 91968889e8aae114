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
