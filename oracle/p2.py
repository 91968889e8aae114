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
    # heartbeat surface loads on 6-node faces (node ids from tri6_nodes):
    # follower pressure (times the load scale) and elastic Robin springs
    pressure_tri6: np.ndarray = None
    pressure: float = 0.0
    robin_tri6: np.ndarray = None
    k_perp: float = 0.0
    k_par: float = 0.0

    def __post_init__(self):
        self.conn = np.asarray(self.conn, dtype=np.int64)
        self.R = (p2_robin_matrix(self.X, np.asarray(self.robin_tri6), self.k_perp, self.k_par)
                  if self.robin_tri6 is not None else None)
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

    def surface_force(self, u, load_scale: float = 1.0):
        """Residual part of the follower pressure and the springs."""
        out = np.zeros(self.n_dofs)
        if self.pressure_tri6 is not None:
            out += p2_follower_pressure(self.X, u, np.asarray(self.pressure_tri6),
                                        load_scale * self.pressure)
        if self.R is not None:
            out += self.R @ u
        return out

    def residual(self, u, load_scale: float = 1.0):
        re = self.element_residual(u[self.edofs])
        r = np.zeros(self.n_dofs)
        np.add.at(r, self.edofs.reshape(-1), re.reshape(-1))
        r -= load_scale * self.f_ext
        r += self.surface_force(u, load_scale)
        r[self.fixed] = 0.0
        return r

    def min_jacobian(self, u):
        U = u[self.edofs].reshape(-1, 10, 3)
        return float(min(materials.det(self._F(U, q)).min() for q in range(4)))

    def energy(self, u, load_scale: float = 1.0):
        """Strain energy, springs and dead loads (a follower pressure has no
        potential)."""
        U = u[self.edofs].reshape(-1, 10, 3)
        tot = 0.0
        for q in range(4):
            tot += float(np.sum(self.V / 4.0 * materials.energy(self.material, self._F(U, q),
                                                                 self.params)))
        if self.R is not None:
            tot += 0.5 * float(u @ (self.R @ u))
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
        if self.pressure_tri6 is not None:
            K = K + p2_follower_pressure_jacobian(self.X, u, np.asarray(self.pressure_tri6),
                                                  load_scale * self.pressure)
        if self.R is not None:
            K = K + self.R
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


def shell_p2_problem(mesh2, consts: dict, gamma: float = 0.0, law=None,
                     loads: bool = False) -> P2Problem:
    """The ventricle shell with quadratic displacements: the cardiac-like law
    M4 (or, with law = (C, b_ff, b_ss, b_nn, b_fs, b_fn, b_sn, B), Guccione's
    law M6 with the mesh's sheets), the mesh's per-element fibres, active
    tension gamma, and the shell's constraints (base plane held in z at its
    vertices and edge midpoints, three circumferential pins).  loads: the
    heartbeat's follower pressure p_max on the endocardium and springs on
    the epicardium, on the 6-node faces."""
    from synthetic import shell_dirichlet

    c = consts
    if law is None:
        material = materials.M4
        params = (c["a"], c["b"], c["af"], c["bf"], c["kappa"], gamma, mesh2.elem_fibre)
    else:
        material = materials.M6
        params = tuple(law) + (gamma, mesh2.elem_fibre, mesh2.elem_sheet)
    dd = shell_dirichlet(mesh2)
    kw = {}
    if loads:
        cn = np.asarray(mesh2.conn)
        kw = dict(pressure_tri6=tri6_nodes(cn, mesh2.faces["endo"]), pressure=c["p_max"],
                  robin_tri6=tri6_nodes(cn, mesh2.faces["epi"]), k_perp=c["k_perp"],
                  k_par=c["k_par"])
    return P2Problem(mesh2.X, mesh2.conn, material, params, np.zeros(3 * mesh2.X.shape[0]), dd,
                     np.zeros(dd.size), **kw)


def set_active_tension(problem: P2Problem, gamma: float) -> None:
    """Replace the active tension gamma of an M4 or M6 problem."""
    p = list(problem.params)
    p[8 if problem.material == materials.M6 else 5] = gamma
    problem.params = tuple(p)


# ---- surface loads on 6-node faces ------------------------------------------------
def _gauss_triangle(n: int = 4):
    """Collapsed (Duffy) Gauss-Legendre rule on the reference triangle
    {xi, eta >= 0, xi + eta <= 1}: xi = a, eta = b (1 - a) with n x n
    Gauss points on [0, 1]^2 and weights w_a w_b (1 - a); exact for
    polynomials of total degree <= 2 n - 2."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            pts.append((g[i], g[j] * (1.0 - g[i])))
            wts.append(w[i] * w[j] * (1.0 - g[i]))
    return np.array(pts), np.array(wts)


def _tri6_shapes(xi: float, eta: float):
    """Quadratic triangle shape functions and their (xi, eta) derivatives;
    nodes: vertices 0, 1, 2 (at (0,0), (1,0), (0,1)), then the midpoints of
    edges (0,1), (1,2), (0,2)."""
    L = np.array([1.0 - xi - eta, xi, eta])
    dL = np.array([[-1.0, -1.0], [1.0, 0.0], [0.0, 1.0]])
    N = np.empty(6)
    dN = np.empty((6, 2))
    for a in range(3):
        N[a] = L[a] * (2.0 * L[a] - 1.0)
        dN[a] = (4.0 * L[a] - 1.0) * dL[a]
    for k, (a, b) in enumerate(((0, 1), (1, 2), (0, 2))):
        N[3 + k] = 4.0 * L[a] * L[b]
        dN[3 + k] = 4.0 * (L[a] * dL[b] + L[b] * dL[a])
    return N, dN


def tri6_nodes(conn10: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """(n_f, 6) node ids of the 6-node faces over the vertex triangles tri:
    the three vertices, then the midpoints of (0,1), (1,2), (0,2)."""
    mid = edge_midpoints(conn10)
    out = np.empty((len(tri), 6), dtype=np.int64)
    for f, v in enumerate(np.asarray(tri)):
        out[f, :3] = v
        for k, (a, b) in enumerate(((0, 1), (1, 2), (0, 2))):
            out[f, 3 + k] = mid[(min(v[a], v[b]), max(v[a], v[b]))]
    return out


def p2_follower_pressure(X: np.ndarray, u: np.ndarray, tri6: np.ndarray, p: float) -> np.ndarray:
    """Residual part of a follower pressure p on 6-node faces: node a gains
    p int N_a (x_xi x x_eta) dxi deta over the reference triangle (the current
    area vector density, x = X + u interpolated quadratically; the same
    orientation as the linear faces).  The integrand has degree 4; the
    collapsed Gauss rule of degree 6 integrates it exactly.  Complex-safe."""
    x = np.asarray(X)[tri6] + np.asarray(u).reshape(-1, 3)[tri6]  # (f, 6, 3)
    out = np.zeros((X.shape[0], 3), dtype=x.dtype)
    pts, wts = _gauss_triangle(4)
    fv = np.zeros((tri6.shape[0], 6, 3), dtype=x.dtype)
    for (xi, eta), w in zip(pts, wts):
        N, dN = _tri6_shapes(xi, eta)
        xx = np.einsum("a,fai->fi", dN[:, 0], x)
        xe = np.einsum("a,fai->fi", dN[:, 1], x)
        nrm = np.cross(xx, xe)
        fv += w * p * N[None, :, None] * nrm[:, None, :]
    for f in range(tri6.shape[0]):
        for a in range(6):
            out[tri6[f, a]] += fv[f, a]
    return out.reshape(-1)


def p2_follower_pressure_jacobian(X: np.ndarray, u: np.ndarray, tri6: np.ndarray, p: float,
                                  h: float = 1e-30) -> sp.csr_matrix:
    """d(p2_follower_pressure)/du by complex steps of each face's 18 dofs."""
    X = np.asarray(X, dtype=np.float64)
    nf = tri6.shape[0]
    n = 3 * X.shape[0]
    rows, cols, vals = [], [], []
    for f in range(nf):
        nodes = tri6[f]
        dofs = (3 * nodes[:, None] + np.arange(3)[None, :]).reshape(-1)
        xf = X[nodes] + np.asarray(u, dtype=np.float64).reshape(-1, 3)[nodes]
        sub = np.arange(6)
        for j in range(18):
            uc = np.zeros((6, 3), dtype=np.complex128)
            uc[j // 3, j % 3] = 1j * h
            col = p2_follower_pressure(xf.astype(np.complex128) + uc, np.zeros(18, np.complex128),
                                       sub[None, :], p).imag / h
            rows.extend(dofs.tolist())
            cols.extend([dofs[j]] * 18)
            vals.extend(col.tolist())
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def p2_robin_matrix(X: np.ndarray, tri6: np.ndarray, k_perp: float, k_par: float) -> sp.csr_matrix:
    """Elastic Robin springs on flat 6-node faces: R_(a,b) = M_ab K with the
    face mass M_ab = int N_a N_b dA (reference area, collapsed Gauss rule,
    exact) and K = k_par I + (k_perp - k_par) N (x) N, N the face's
    reference unit normal."""
    X = np.asarray(X, dtype=np.float64)
    pts, wts = _gauss_triangle(4)
    Mref = np.zeros((6, 6))
    for (xi, eta), w in zip(pts, wts):
        N, _ = _tri6_shapes(xi, eta)
        Mref += w * np.outer(N, N)
    n = 3 * X.shape[0]
    rows, cols, vals = [], [], []
    for nodes in tri6:
        a2 = np.cross(X[nodes[1]] - X[nodes[0]], X[nodes[2]] - X[nodes[0]])
        jac = np.linalg.norm(a2)  # 2 A: the map's area factor
        Nn = a2 / jac
        K = k_par * np.eye(3) + (k_perp - k_par) * np.outer(Nn, Nn)
        for a in range(6):
            for b in range(6):
                blk = jac * Mref[a, b] * K
                for i in range(3):
                    for k in range(3):
                        rows.append(3 * nodes[a] + i)
                        cols.append(3 * nodes[b] + k)
                        vals.append(blk[i, k])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
