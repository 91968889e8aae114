"""Quadratic (10-node) displacement tetrahedra for the compressible laws (FP64).

Test infrastructure: only the tests, the smoke check and the CPU baseline
timing use this package.

Half of the paper's result tables use second-order elements (Sec. 6, the Cook
and heartbeat tables).  Here: Cook's membrane with P2 displacements and law
M1, Pi(u) = sum_e int_e Psi(F) dX - s f_ext . u, integrated with the same
symmetric 4-point rule of degree 2 as the mixed form (exact for the
linearised stiffness of straight-sided P2 elements), residual r = dPi/du,
complex-step tangent, strong Dirichlet rows and columns as in fem.py.

A constant traction t on a flat 6-node triangle of area A gives the vertices
nothing and each edge midpoint t A / 3 (the integrals of the quadratic shape
functions over the triangle).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import materials
from .fem import p1_geometry
from .mixed import EDGES, QUAD_BARY, p2_gradients


def edge_midpoints(conn10: np.ndarray) -> dict:
    """(min vertex, max vertex) -> midpoint node, from the P2 connectivity."""
    out = {}
    for k, (a, b) in enumerate(EDGES):
        for e in range(conn10.shape[0]):
            va, vb = int(conn10[e, a]), int(conn10[e, b])
            out[(min(va, vb), max(va, vb))] = int(conn10[e, 4 + k])
    return out


def p2_traction(X: np.ndarray, conn10: np.ndarray, tri: np.ndarray, t) -> np.ndarray:
    """Consistent nodal forces of a constant traction t (per reference area) on
    the flat 6-node triangles whose vertices are tri (midpoints from conn10)."""
    mid = edge_midpoints(conn10)
    f = np.zeros(3 * X.shape[0])
    tt = np.asarray(t, dtype=np.float64)
    for v in np.asarray(tri):
        area = 0.5 * np.linalg.norm(np.cross(X[v[1]] - X[v[0]], X[v[2]] - X[v[0]]))
        for a, b in ((0, 1), (1, 2), (0, 2)):
            m = mid[(min(v[a], v[b]), max(v[a], v[b]))]
            f[3 * m:3 * m + 3] += tt * area / 3.0
    return f


@dataclass
class P2Problem:
    X: np.ndarray
    conn: np.ndarray        # (n_e, 10)
    material: str
    params: tuple
    f_ext: np.ndarray
    ddofs: np.ndarray
    dvals: np.ndarray

    def __post_init__(self):
        self.conn = np.asarray(self.conn, dtype=np.int64)
        self.G, self.V = p1_geometry(self.X, self.conn[:, :4])
        if np.any(self.V <= 0):
            raise ValueError("non-positive element volume")
        self.n_nodes = self.X.shape[0]
        self.n_dofs = 3 * self.n_nodes
        self.fixed = np.zeros(self.n_dofs, dtype=bool)
        self.fixed[np.asarray(self.ddofs, dtype=np.int64)] = True
        self.free = ~self.fixed
        self.gradN = [p2_gradients(self.G, QUAD_BARY[q]) for q in range(4)]
        self.edofs = (3 * self.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 30)

    def lift(self, u):
        u = np.array(u, dtype=np.float64, copy=True)
        u[self.ddofs] = self.dvals
        return u

    def _F(self, U, q):
        return np.eye(3) + np.einsum("eai,eaJ->eiJ", U, self.gradN[q])

    def element_residual(self, ue):
        """(n_e, 30) element residuals from element dofs (n_e, 30); complex-safe."""
        U = ue.reshape(-1, 10, 3)
        out = np.zeros(ue.shape, dtype=ue.dtype)
        for q in range(4):
            P = materials.piola(self.material, self._F(U, q), self.params)
            w = self.V / 4.0
            out += (w[:, None, None] * np.einsum("eiJ,eaJ->eai", P, self.gradN[q])).reshape(-1, 30)
        return out

    def residual(self, u, load_scale: float = 1.0):
        re = self.element_residual(u[self.edofs])
        r = np.zeros(self.n_dofs)
        np.add.at(r, self.edofs.reshape(-1), re.reshape(-1))
        r -= load_scale * self.f_ext
        r[self.fixed] = 0.0
        return r

    def min_jacobian(self, u):
        U = u[self.edofs].reshape(-1, 10, 3)
        return float(min(materials.det(self._F(U, q)).min() for q in range(4)))

    def energy(self, u, load_scale: float = 1.0):
        U = u[self.edofs].reshape(-1, 10, 3)
        tot = 0.0
        for q in range(4):
            tot += float(np.sum(self.V / 4.0 * materials.energy(self.material, self._F(U, q),
                                                                 self.params)))
        return tot - load_scale * float(self.f_ext @ u)

    def stiffness(self, u, dirichlet: bool = True, load_scale: float = 1.0,
                  h: float = 1e-30) -> sp.csr_matrix:
        ue = u[self.edofs].astype(np.complex128)
        ne = ue.shape[0]
        Ke = np.empty((ne, 30, 30))
        for j in range(30):
            up = ue.copy()
            up[:, j] += 1j * h
            Ke[:, :, j] = self.element_residual(up).imag / h
        rows = np.repeat(self.edofs, 30, axis=1).reshape(-1)
        cols = np.tile(self.edofs, (1, 30)).reshape(-1)
        K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(self.n_dofs, self.n_dofs)).tocsr()
        if dirichlet:
            D = sp.diags(self.free.astype(np.float64))
            K = (D @ K @ D + sp.diags(self.fixed.astype(np.float64))).tocsr()
        return K

    def jv(self, u, v, load_scale: float = 1.0):
        return self.stiffness(u) @ v

    def diagonal(self, u, load_scale: float = 1.0):
        return self.stiffness(u).diagonal()


def cook_p2_problem(mesh2, mu: float = 80.194, lam: float = 400.9, tau: float = 1.0) -> P2Problem:
    """Cook's membrane with P2 displacements, law M1, dead shear traction
    (0, tau, 0) per reference area on x = 48, clamped on x = 0."""
    f = p2_traction(mesh2.X, mesh2.conn, mesh2.faces["load"], (0.0, tau, 0.0))
    dd = mesh2.dirichlet_dofs("clamp")
    return P2Problem(mesh2.X, mesh2.conn, materials.M1, (mu, lam), f, dd, np.zeros(dd.size))


def shell_p2_problem(mesh2, consts: dict, gamma: float = 0.0, law=None) -> P2Problem:
    """The ventricle shell with quadratic displacements: the cardiac-like law
    M4 (or, with law = (C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B), Guccione's
    law M6 with the mesh's sheets), the mesh's per-element fibres, active
    tension gamma, and the shell's constraints (base plane held in z at its
    vertices and edge midpoints, three circumferential pins).  No surface
    loads: the endocardial pressure and epicardial springs act on P1 faces
    only."""
    from synthetic import shell_dirichlet

    c = consts
    if law is None:
        material = materials.M4
        params = (c["a"], c["b"], c["af"], c["bf"], c["kappa"], gamma, mesh2.elem_fibre)
    else:
        material = materials.M6
        params = tuple(law) + (gamma, mesh2.elem_fibre, mesh2.elem_sheet)
    dd = shell_dirichlet(mesh2)
    return P2Problem(mesh2.X, mesh2.conn, material, params, np.zeros(3 * mesh2.X.shape[0]), dd,
                     np.zeros(dd.size))


def set_active_tension(problem: P2Problem, gamma: float) -> None:
    """Replace the active tension gamma of an M4 or M6 problem."""
    p = list(problem.params)
    p[8 if problem.material == materials.M6 else 5] = gamma
    problem.params = tuple(p)
