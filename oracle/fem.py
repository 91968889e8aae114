"""P1 tetrahedral finite elements for quasi-static hyperelasticity (FP64).

Paper, Sec. 2 (eq. "momentum strong", quasi-static: inertia dropped) and
Sec. 3 (eq. "minimization"): the discrete problem is the stationarity of

    Pi(u) = sum_e V_e Psi(F_e) - s * f_ext . u

over displacements u with prescribed values on the Dirichlet dofs.  Its
gradient is the residual used by every solver here,

    r(u) = f_int(u) - s * f_ext,   f_int[a] = sum_e V_e P(F_e) grad N_a,

set to zero on Dirichlet dofs (which hold their prescribed values; strong
imposition, rows and columns of the tangent replaced by the identity).
This is the paper's R(d) = f - div P up to its overall sign (same root).

A P1 tetrahedron has a constant deformation gradient, so the one-point
rule is exact.  Vectors interleave components per node: dof = 3 a + i.
Dead tractions are per unit reference area; on a linear triangle the
consistent nodal load is t * A / 3 per vertex (exact).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import scipy.sparse as sp

from . import materials


def p1_geometry(X: np.ndarray, conn: np.ndarray):
    """Shape-function gradients G[e, a, :] = grad N_a and volumes V[e].

    With D = [X1 - X0, X2 - X0, X3 - X0] (columns), the barycentric
    coordinates are xi = D^-1 (x - X0), so grad N_a (a = 1, 2, 3) is row
    a-1 of D^-1 and grad N_0 = -(grad N_1 + grad N_2 + grad N_3).
    V = det(D) / 6, required positive (positively oriented elements).
    """
    X = np.asarray(X, dtype=np.float64)
    c = np.asarray(conn)[:, :4]
    x0 = X[c[:, 0]]
    D = np.stack([X[c[:, 1]] - x0, X[c[:, 2]] - x0, X[c[:, 3]] - x0], axis=-1)
    detD = np.linalg.det(D)
    Dinv = np.linalg.inv(D)
    G = np.empty((c.shape[0], 4, 3))
    G[:, 1:, :] = Dinv
    G[:, 0, :] = -Dinv.sum(axis=1)
    return G, detD / 6.0


def deformation_gradient(u: np.ndarray, conn: np.ndarray, G: np.ndarray) -> np.ndarray:
    """F_e = I + sum_a u_a (outer) grad N_a, shape (n_e, 3, 3)."""
    U = np.asarray(u).reshape(-1, 3)[conn[:, :4]]  # (e, a, i)
    return np.eye(3) + np.einsum("eai,eaJ->eiJ", U, G)


def scatter_nodal(n_nodes: int, conn: np.ndarray, fe: np.ndarray) -> np.ndarray:
    """Sum element nodal vectors fe[e, a, i] into a dof vector (3 n_nodes)."""
    out = np.zeros((n_nodes, 3))
    idx = conn[:, :4].reshape(-1)
    for i in range(3):
        out[:, i] = np.bincount(idx, weights=fe[:, :, i].reshape(-1), minlength=n_nodes)
    return out.reshape(-1)


def dead_traction(X: np.ndarray, tri: np.ndarray, t: Sequence[float]) -> np.ndarray:
    """Consistent nodal forces of a constant traction t per reference area."""
    X = np.asarray(X, dtype=np.float64)
    xa = X[tri[:, 0]]
    area = 0.5 * np.linalg.norm(np.cross(X[tri[:, 1]] - xa, X[tri[:, 2]] - xa), axis=1)
    fe = (area / 3.0)[:, None, None] * np.asarray(t, dtype=np.float64)[None, None, :]
    fe = np.broadcast_to(fe, (tri.shape[0], 3, 3))
    out = np.zeros((X.shape[0], 3))
    for i in range(3):
        out[:, i] = np.bincount(tri.reshape(-1), weights=fe[:, :, i].reshape(-1),
                                minlength=X.shape[0])
    return out.reshape(-1)


@dataclass
class Problem:
    """A P1 quasi-static problem: mesh, law, loads and Dirichlet data.

    f_ext is the reference (unit load-scale) external force vector; the
    residual subtracts load_scale * f_ext.  Dirichlet dofs hold `dvals`.
    """

    X: np.ndarray
    conn: np.ndarray
    material: str
    params: tuple
    f_ext: np.ndarray
    ddofs: np.ndarray
    dvals: np.ndarray

    def __post_init__(self):
        self.conn = np.asarray(self.conn)[:, :4].astype(np.int64)
        self.G, self.V = p1_geometry(self.X, self.conn)
        if np.any(self.V <= 0):
            raise ValueError("non-positive element volume")
        self.n_nodes = self.X.shape[0]
        self.n_dofs = 3 * self.n_nodes
        self.fixed = np.zeros(self.n_dofs, dtype=bool)
        self.fixed[np.asarray(self.ddofs, dtype=np.int64)] = True
        self.free = ~self.fixed

    # -- evaluation -------------------------------------------------------
    def lift(self, u: np.ndarray) -> np.ndarray:
        u = np.array(u, dtype=np.float64, copy=True)
        u[self.ddofs] = self.dvals
        return u

    def internal_force(self, u: np.ndarray) -> np.ndarray:
        F = deformation_gradient(u, self.conn, self.G)
        P = materials.piola(self.material, F, self.params)
        fe = self.V[:, None, None] * np.einsum("eiJ,eaJ->eai", P, self.G)
        return scatter_nodal(self.n_nodes, self.conn, fe)

    def residual(self, u: np.ndarray, load_scale: float = 1.0) -> np.ndarray:
        r = self.internal_force(u) - load_scale * self.f_ext
        r[self.fixed] = 0.0
        return r

    def min_jacobian(self, u: np.ndarray) -> float:
        return float(materials.det(deformation_gradient(u, self.conn, self.G)).min())

    def energy(self, u: np.ndarray, load_scale: float = 1.0) -> float:
        F = deformation_gradient(u, self.conn, self.G)
        psi = materials.energy(self.material, F, self.params)
        return float(np.sum(self.V * psi) - load_scale * np.dot(self.f_ext, u))

    # -- tangent ----------------------------------------------------------
    def element_stiffness(self, u: np.ndarray) -> np.ndarray:
        """K_e[(a,i),(b,k)] = V sum_{J,L} A_iJkL gradN_aJ gradN_bL, (n_e,12,12)."""
        F = deformation_gradient(u, self.conn, self.G)
        A = materials.tangent(self.material, F, self.params)
        Ke = np.einsum("e,eiJkL,eaJ,ebL->eaibk", self.V, A, self.G, self.G, optimize=True)
        return Ke.reshape(-1, 12, 12)

    def stiffness(self, u: np.ndarray, dirichlet: bool = True) -> sp.csr_matrix:
        """Assembled tangent dr/du (CSR); identity rows/cols on Dirichlet dofs."""
        Ke = self.element_stiffness(u)
        dofs = (3 * self.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        rows = np.repeat(dofs, 12, axis=1).reshape(-1)
        cols = np.tile(dofs, (1, 12)).reshape(-1)
        K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(self.n_dofs, self.n_dofs)).tocsr()
        if dirichlet:
            Dfree = sp.diags(self.free.astype(np.float64))
            K = (Dfree @ K @ Dfree + sp.diags(self.fixed.astype(np.float64))).tocsr()
        return K

    def jv(self, u: np.ndarray, v: np.ndarray) -> np.ndarray:
        """Jacobian action J(u) v with identity rows/cols on Dirichlet dofs."""
        return self.stiffness(u) @ v

    def diagonal(self, u: np.ndarray) -> np.ndarray:
        """Diagonal of the tangent (1 on Dirichlet dofs)."""
        return self.stiffness(u).diagonal()


def cook_problem(mesh, mu: float = 80.194, lam: float = 400.9, tau: float = 1.0,
                 material: str = materials.M1, c_vol: Optional[float] = None) -> Problem:
    """Cook's membrane: clamp x = 0, dead shear traction (0, tau, 0) on x = 48.

    f_ext is for traction tau; the residual's load_scale multiplies it.
    """
    params = (mu, lam) if material == materials.M1 else (mu, lam, 0.25 if c_vol is None else c_vol)
    f_ext = dead_traction(mesh.X, mesh.faces["load"], (0.0, tau, 0.0))
    ddofs = mesh.dirichlet_dofs("clamp")
    return Problem(mesh.X, mesh.conn, material, params, f_ext, ddofs, np.zeros(ddofs.size))
