"""Mixed displacement / pressure form of the twist test (FP64).

Paper, Sec. 4 ("Twist test"): an incompressible body with an inf-sup stable
pair of spaces and a pressure multiplier for det F = 1.  Here (the twist
workload's statement) the pair is quadratic displacement / linear pressure
(P2-P1) on tetrahedra and the law is incompressible neo-Hookean (M3):

    L(u, p) = sum_e int_e [ mu/2 (I1 - 3) - mu ln J - p (J - 1) ] dX

The residual is its gradient,
    R_u[a] = int P(F, p) grad N_a,      P = mu (F - F^-T) - p J F^-T,
    R_p[b] = - int (J - 1) lambda_b,
with N_a the ten quadratic shape functions (vertex a: lambda_a (2 lambda_a - 1),
edge (a, b): 4 lambda_a lambda_b, edges in the order (0,1), (1,2), (0,2), (0,3),
(1,3), (2,3)) and lambda_b the barycentric coordinates (linear pressure).
Integrals use the symmetric 4-point rule of degree 2: barycentric points
(alpha, beta, beta, beta) and permutations, alpha = (5 + 3 sqrt 5)/20,
beta = (5 - sqrt 5)/20, weight V/4 each.

Unknown vector: x = [u (3 per displacement node, interleaved) | p (one per
pressure node)].  Dirichlet data act on displacement dofs only (strong, as
in fem.py).  The tangent is taken by complex-step differentiation of the
element residual, assembled as a sparse symmetric indefinite matrix.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import materials
from .fem import p1_geometry

EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))
_A = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
_B = (5.0 - math.sqrt(5.0)) / 20.0
QUAD_BARY = np.array([[_A, _B, _B, _B], [_B, _A, _B, _B], [_B, _B, _A, _B], [_B, _B, _B, _A]])


def p2_gradients(G: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Gradients of the ten quadratic shape functions at barycentric point lam.

    G[e, a, :] = grad lambda_a (a = 0..3), lam shape (4,).  Returns (e, 10, 3).
    """
    out = np.empty(G.shape[:1] + (10, 3))
    for a in range(4):
        out[:, a] = (4.0 * lam[a] - 1.0) * G[:, a]
    for k, (a, b) in enumerate(EDGES):
        out[:, 4 + k] = 4.0 * (lam[b] * G[:, a] + lam[a] * G[:, b])
    return out


def m3_piola(F, p, mu):
    """P = mu (F - F^-T) - p J F^-T (valid for complex input)."""
    J = materials.det(F)
    FiT = materials.inv_transpose(F)
    return mu * (F - FiT) - (p * J)[..., None, None] * FiT


@dataclass
class MixedProblem:
    X: np.ndarray          # (n_u, 3) displacement-node coordinates
    conn: np.ndarray       # (n_e, 10)
    pconn: np.ndarray      # (n_e, 4)
    n_p: int
    mu: float
    ddofs: np.ndarray      # constrained displacement dofs
    dvals: np.ndarray

    def __post_init__(self):
        self.conn = np.asarray(self.conn, dtype=np.int64)
        self.pconn = np.asarray(self.pconn, dtype=np.int64)
        self.G, self.V = p1_geometry(self.X, self.conn[:, :4])
        if np.any(self.V <= 0):
            raise ValueError("non-positive element volume")
        self.n_u = self.X.shape[0]
        self.n_dofs = 3 * self.n_u + self.n_p
        self.fixed = np.zeros(self.n_dofs, dtype=bool)
        self.fixed[np.asarray(self.ddofs, dtype=np.int64)] = True
        self.free = ~self.fixed
        self.gradN = [p2_gradients(self.G, QUAD_BARY[q]) for q in range(4)]
        # element dof map: 30 displacement dofs (node-major), then 4 pressures
        ud = (3 * self.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 30)
        self.edofs = np.concatenate([ud, 3 * self.n_u + self.pconn], axis=1)

    def split(self, x):
        return x[: 3 * self.n_u], x[3 * self.n_u:]

    def lift(self, x):
        x = np.array(x, dtype=np.float64, copy=True)
        x[self.ddofs] = self.dvals
        return x

    def element_residual(self, xe):
        """Element residual (n_e, 34) from element dofs xe (n_e, 34); complex-safe."""
        U = xe[:, :30].reshape(-1, 10, 3)
        P_nodes = xe[:, 30:]
        out = np.zeros(xe.shape, dtype=xe.dtype)
        for q in range(4):
            gN = self.gradN[q]
            F = np.eye(3) + np.einsum("eai,eaJ->eiJ", U, gN)
            pq = P_nodes @ QUAD_BARY[q]
            w = self.V / 4.0
            P = m3_piola(F, pq, self.mu)
            out[:, :30] += (w[:, None, None] * np.einsum("eiJ,eaJ->eai", P, gN)).reshape(-1, 30)
            J = materials.det(F)
            out[:, 30:] += -(w * (J - 1.0))[:, None] * QUAD_BARY[q][None, :]
        return out

    def residual(self, x, load_scale: float = 1.0):
        """Residual (no external loads in the twist test; load_scale unused)."""
        xe = x[self.edofs]
        re = self.element_residual(xe)
        r = np.zeros(self.n_dofs)
        np.add.at(r, self.edofs.reshape(-1), re.reshape(-1))
        r[self.fixed] = 0.0
        return r

    def min_jacobian(self, x):
        U = x[self.edofs][:, :30].reshape(-1, 10, 3)
        return float(min(materials.det(np.eye(3) + np.einsum("eai,eaJ->eiJ", U, g)).min()
                         for g in self.gradN))

    def energy(self, x):
        xe = x[self.edofs]
        U = xe[:, :30].reshape(-1, 10, 3)
        tot = 0.0
        for q in range(4):
            F = np.eye(3) + np.einsum("eai,eaJ->eiJ", U, self.gradN[q])
            J = materials.det(F)
            I1 = np.einsum("eij,eij->e", F, F)
            pq = xe[:, 30:] @ QUAD_BARY[q]
            L = 0.5 * self.mu * (I1 - 3.0) - self.mu * np.log(J) - pq * (J - 1.0)
            tot += float(np.sum(self.V / 4.0 * L))
        return tot

    def stiffness(self, x, dirichlet: bool = True, load_scale: float = 1.0,
                  h: float = 1e-30) -> sp.csr_matrix:
        xe = x[self.edofs].astype(np.complex128)
        ne = xe.shape[0]
        Ke = np.empty((ne, 34, 34))
        for j in range(34):
            xp = xe.copy()
            xp[:, j] += 1j * h
            Ke[:, :, j] = self.element_residual(xp).imag / h
        rows = np.repeat(self.edofs, 34, axis=1).reshape(-1)
        cols = np.tile(self.edofs, (1, 34)).reshape(-1)
        K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(self.n_dofs, self.n_dofs)).tocsr()
        if dirichlet:
            D = sp.diags(self.free.astype(np.float64))
            K = (D @ K @ D + sp.diags(self.fixed.astype(np.float64))).tocsr()
        return K

    def jv(self, x, v):
        return self.stiffness(x) @ v

    def pressure_mass_lumped(self):
        """Row sums of the P1 pressure mass matrix: V/4 per vertex and element."""
        m = np.zeros(self.n_p)
        np.add.at(m, self.pconn.reshape(-1), np.repeat(self.V / 4.0, 4))
        return m


def twist_problem(mesh, mu: float, theta: float) -> MixedProblem:
    """Twist test: bottom clamped, top x/y rotated by theta about x = y = 1/2."""
    from synthetic import twist_dirichlet

    dofs, vals = twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], theta)
    return MixedProblem(mesh.X, mesh.conn, mesh.pconn, mesh.n_pressure, mu, dofs, vals)


def set_twist_angle(problem: MixedProblem, mesh, theta: float) -> None:
    from synthetic import twist_dirichlet

    dofs, vals = twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], theta)
    assert np.array_equal(dofs, problem.ddofs)
    problem.dvals = vals
