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


def follower_pressure(X: np.ndarray, u: np.ndarray, tri: np.ndarray, p: float) -> np.ndarray:
    """Nodal residual contribution of a follower pressure p on triangles tri.

    The pressure acts on the current surface (x = X + u) against the body's
    outward normal; on a flat linear triangle with current area vector
    a = (x1 - x0) x (x2 - x0) / 2 the consistent load is -p a / 3 per vertex
    (exact), so r gains +p a / 3 at each vertex.  Valid for complex u.
    """
    x = np.asarray(X)[tri] + np.asarray(u).reshape(-1, 3)[tri]  # (f, 3, 3)
    a2 = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    out = np.zeros((X.shape[0], 3), dtype=a2.dtype)
    for i in range(3):
        w = np.repeat(p * a2[:, i] / 6.0, 3)
        idx = tri.reshape(-1)
        if np.iscomplexobj(w):
            out[:, i] = (np.bincount(idx, weights=w.real, minlength=X.shape[0])
                         + 1j * np.bincount(idx, weights=w.imag, minlength=X.shape[0]))
        else:
            out[:, i] = np.bincount(idx, weights=w, minlength=X.shape[0])
    return out.reshape(-1)


def follower_pressure_jacobian(X: np.ndarray, u: np.ndarray, tri: np.ndarray, p: float,
                               h: float = 1e-30) -> sp.csr_matrix:
    """d(follower_pressure)/du, assembled from per-face complex-step blocks
    (9 x 9 per triangle).  Not symmetric in general."""
    X = np.asarray(X, dtype=np.float64)
    x = X[tri] + np.asarray(u, dtype=np.float64).reshape(-1, 3)[tri]
    nf = tri.shape[0]
    Kf = np.empty((nf, 3, 3, 3, 3))  # [f, a, i, b, k]
    for b in range(3):
        for k in range(3):
            xc = x.astype(np.complex128)
            xc[:, b, k] += 1j * h
            d = np.cross(xc[:, 1] - xc[:, 0], xc[:, 2] - xc[:, 0]).imag / h  # (f, 3)
            Kf[:, :, :, b, k] = (p / 6.0) * d[:, None, :]
    dofs = (3 * tri[:, :, None] + np.arange(3)[None, None, :]).reshape(nf, 9)
    rows = np.repeat(dofs, 9, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 9)).reshape(-1)
    n = 3 * X.shape[0]
    return sp.coo_matrix((Kf.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()


def follower_traction(X: np.ndarray, u: np.ndarray, tri: np.ndarray, t: Sequence[float]) -> np.ndarray:
    """Consistent nodal forces of a traction t of fixed spatial direction per
    unit CURRENT area (the Cook load "in the deformed configuration", Sec. 4,
    read as a Cauchy traction of fixed direction): on a flat linear triangle
    with current area |a|, a = (x1 - x0) x (x2 - x0) / 2, each vertex gets
    t |a| / 3 (exact).  Valid for complex u (complex-step derivatives)."""
    x = np.asarray(X)[tri] + np.asarray(u).reshape(-1, 3)[tri]
    a2 = np.cross(x[:, 1] - x[:, 0], x[:, 2] - x[:, 0])
    area = 0.5 * np.sqrt(np.sum(a2 * a2, axis=1))  # analytic, so complex-step safe
    tt = np.asarray(t)
    out = np.zeros((X.shape[0], 3), dtype=area.dtype)
    idx = tri.reshape(-1)
    for i in range(3):
        w = np.repeat(tt[i] * area / 3.0, 3)
        if np.iscomplexobj(w):
            out[:, i] = (np.bincount(idx, weights=w.real, minlength=X.shape[0])
                         + 1j * np.bincount(idx, weights=w.imag, minlength=X.shape[0]))
        else:
            out[:, i] = np.bincount(idx, weights=w, minlength=X.shape[0])
    return out.reshape(-1)


def follower_traction_jacobian(X: np.ndarray, u: np.ndarray, tri: np.ndarray, t: Sequence[float],
                               h: float = 1e-30) -> sp.csr_matrix:
    """d(follower_traction)/du from per-face complex-step blocks (9 x 9 per
    triangle); not symmetric."""
    X = np.asarray(X, dtype=np.float64)
    x = X[tri] + np.asarray(u, dtype=np.float64).reshape(-1, 3)[tri]
    tt = np.asarray(t, dtype=np.float64)
    nf = tri.shape[0]
    Kf = np.empty((nf, 3, 3, 3, 3))  # [f, a, i, b, k]
    for b in range(3):
        for k in range(3):
            xc = x.astype(np.complex128)
            xc[:, b, k] += 1j * h
            a2 = np.cross(xc[:, 1] - xc[:, 0], xc[:, 2] - xc[:, 0])
            darea = (0.5 * np.sqrt(np.sum(a2 * a2, axis=1))).imag / h  # (f,)
            Kf[:, :, :, b, k] = (darea[:, None, None] / 3.0) * tt[None, None, :]
    dofs = (3 * tri[:, :, None] + np.arange(3)[None, None, :]).reshape(nf, 9)
    rows = np.repeat(dofs, 9, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 9)).reshape(-1)
    n = 3 * X.shape[0]
    return sp.coo_matrix((Kf.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()


def robin_matrix(X: np.ndarray, tri: np.ndarray, k_perp: float, k_par: float) -> sp.csr_matrix:
    """Elastic Robin condition of Sec. 4 ("Heartbeat test", epicardium, without
    its damping terms): traction -[k_perp N (x) N + k_par (I - N (x) N)] u with
    the reference unit normal N.  Its residual contribution is R u with
    R_(a,b) = M_ab K, M_ab = A (1 + delta_ab) / 12 (exact P1 face mass)."""
    X = np.asarray(X, dtype=np.float64)
    a2 = np.cross(X[tri[:, 1]] - X[tri[:, 0]], X[tri[:, 2]] - X[tri[:, 0]])
    A = 0.5 * np.linalg.norm(a2, axis=1)
    N = a2 / (2.0 * A)[:, None]
    K = k_par * np.eye(3)[None] + (k_perp - k_par) * np.einsum("fi,fj->fij", N, N)
    M = (np.ones((3, 3)) + np.eye(3)) / 12.0
    Kf = np.einsum("f,ab,fik->faibk", A, M, K)
    nf = tri.shape[0]
    dofs = (3 * tri[:, :, None] + np.arange(3)[None, None, :]).reshape(nf, 9)
    rows = np.repeat(dofs, 9, axis=1).reshape(-1)
    cols = np.tile(dofs, (1, 9)).reshape(-1)
    n = 3 * X.shape[0]
    return sp.coo_matrix((Kf.reshape(-1), (rows, cols)), shape=(n, n)).tocsr()


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
    # optional surface loads: follower pressure (scaled by the load scale)
    # and elastic Robin springs
    pressure_tri: Optional[np.ndarray] = None
    pressure: float = 0.0
    robin_tri: Optional[np.ndarray] = None
    k_perp: float = 0.0
    k_par: float = 0.0
    # follower traction (fixed direction, per unit current area), scaled by
    # the load scale like f_ext
    ftrac_tri: Optional[np.ndarray] = None
    ftrac: tuple = (0.0, 0.0, 0.0)
    # inertia of an implicit time step (set_inertia): (c, m per dof, u_tilde)
    inertia: Optional[tuple] = None
    # viscous Robin damping on the spring faces (set_robin_damping): the
    # face matrix of the dashpot coefficients, and the step's velocity
    # v(u) = v_tilde + cv (u - u_tilde) (set_step_velocity): (cv, v_tilde)
    RC: Optional[object] = None
    step_velocity: Optional[tuple] = None

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
        self.R = (robin_matrix(self.X, np.asarray(self.robin_tri), self.k_perp, self.k_par)
                  if self.robin_tri is not None else None)

    def lumped_mass(self, rho: float) -> np.ndarray:
        """Row-sum lumped P1 mass per dof: rho V / 4 from each element to each
        of its vertices (every component)."""
        m = np.zeros(self.n_nodes)
        np.add.at(m, self.conn.reshape(-1), np.repeat(rho * self.V / 4.0, 4))
        return np.repeat(m, 3)

    def set_inertia(self, rho: float, c: float, u_tilde: np.ndarray) -> None:
        """Add c M (u - u_tilde) to the residual (M lumped with density rho):
        the inertia of an implicit Newmark step with c = 1 / (beta dt^2).
        rho = 0 or c = 0 removes it."""
        if rho == 0.0 or c == 0.0:
            self.inertia = None
        else:
            self.inertia = (c, self.lumped_mass(rho), np.array(u_tilde, dtype=np.float64))

    def set_robin_damping(self, c_perp: float, c_par: float) -> None:
        """Dashpots on the spring faces (the damping terms of the epicardial
        condition of Sec. 4): traction -[c_perp N (x) N + c_par (I - N (x) N)] v
        with v the velocity, integrated like the springs (consistent P1 face
        mass).  Zero coefficients remove them."""
        if self.robin_tri is None or (c_perp == 0.0 and c_par == 0.0):
            self.RC = None
        else:
            self.RC = robin_matrix(self.X, np.asarray(self.robin_tri), c_perp, c_par)

    def set_step_velocity(self, cv: float, v_tilde) -> None:
        """The implicit step's velocity as a function of u,
        v(u) = v_tilde + cv (u - u_tilde) (u_tilde from set_inertia), which the
        dashpots act on; for Newmark cv = gamma / (beta dt) and
        v_tilde = v_n + dt (1 - gamma) a_n.  cv = 0 removes it."""
        self.step_velocity = None if cv == 0.0 else (cv, np.array(v_tilde, dtype=np.float64))

    def _damping_active(self) -> bool:
        return (self.RC is not None and self.step_velocity is not None
                and self.inertia is not None)

    def surface_force(self, u: np.ndarray, load_scale: float = 1.0) -> np.ndarray:
        """Residual contribution of the follower pressure and the springs."""
        out = np.zeros(self.n_dofs)
        if self.pressure_tri is not None:
            out += follower_pressure(self.X, u, np.asarray(self.pressure_tri),
                                     load_scale * self.pressure)
        if self.R is not None:
            out += self.R @ u
        if self.ftrac_tri is not None:
            out -= load_scale * follower_traction(self.X, u, np.asarray(self.ftrac_tri),
                                                  self.ftrac)
        if self.inertia is not None:
            c, m, ut = self.inertia
            out += c * m * (u - ut)
        if self._damping_active():
            cv, vt = self.step_velocity
            out += self.RC @ (vt + cv * (u - self.inertia[2]))
        return out

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
        r = self.internal_force(u) - load_scale * self.f_ext + self.surface_force(u, load_scale)
        r[self.fixed] = 0.0
        return r

    def min_jacobian(self, u: np.ndarray) -> float:
        return float(materials.det(deformation_gradient(u, self.conn, self.G)).min())

    def energy(self, u: np.ndarray, load_scale: float = 1.0) -> float:
        F = deformation_gradient(u, self.conn, self.G)
        if self.pressure_tri is not None or self.ftrac_tri is not None:
            raise ValueError("a follower load has no potential")
        if self._damping_active():
            raise ValueError("the dashpots are not evaluated in the potential")
        psi = materials.energy(self.material, F, self.params)
        springs = 0.5 * float(u @ (self.R @ u)) if self.R is not None else 0.0
        kin = 0.0
        if self.inertia is not None:
            c, m, ut = self.inertia
            kin = 0.5 * c * float(np.sum(m * (u - ut) ** 2))
        return float(np.sum(self.V * psi) - load_scale * np.dot(self.f_ext, u)) + springs + kin

    # -- tangent ----------------------------------------------------------
    def element_stiffness(self, u: np.ndarray) -> np.ndarray:
        """K_e[(a,i),(b,k)] = V sum_{J,L} A_iJkL gradN_aJ gradN_bL, (n_e,12,12)."""
        F = deformation_gradient(u, self.conn, self.G)
        A = materials.tangent(self.material, F, self.params)
        Ke = np.einsum("e,eiJkL,eaJ,ebL->eaibk", self.V, A, self.G, self.G, optimize=True)
        return Ke.reshape(-1, 12, 12)

    def stiffness(self, u: np.ndarray, dirichlet: bool = True,
                  load_scale: float = 1.0) -> sp.csr_matrix:
        """Assembled tangent dr/du (CSR); identity rows/cols on Dirichlet dofs."""
        Ke = self.element_stiffness(u)
        dofs = (3 * self.conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        rows = np.repeat(dofs, 12, axis=1).reshape(-1)
        cols = np.tile(dofs, (1, 12)).reshape(-1)
        K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(self.n_dofs, self.n_dofs)).tocsr()
        if self.pressure_tri is not None:
            K = K + follower_pressure_jacobian(self.X, u, np.asarray(self.pressure_tri),
                                               load_scale * self.pressure)
        if self.R is not None:
            K = K + self.R
        if self.ftrac_tri is not None:
            K = K - load_scale * follower_traction_jacobian(self.X, u, np.asarray(self.ftrac_tri),
                                                            self.ftrac)
        if self.inertia is not None:
            K = K + sp.diags(self.inertia[0] * self.inertia[1])
        if self._damping_active():
            K = K + self.step_velocity[0] * self.RC
        if dirichlet:
            Dfree = sp.diags(self.free.astype(np.float64))
            K = (Dfree @ K @ Dfree + sp.diags(self.fixed.astype(np.float64))).tocsr()
        return K

    def jv(self, u: np.ndarray, v: np.ndarray, load_scale: float = 1.0) -> np.ndarray:
        """Jacobian action J(u) v with identity rows/cols on Dirichlet dofs."""
        return self.stiffness(u, load_scale=load_scale) @ v

    def diagonal(self, u: np.ndarray, load_scale: float = 1.0) -> np.ndarray:
        """Diagonal of the tangent (1 on Dirichlet dofs)."""
        return self.stiffness(u, load_scale=load_scale).diagonal()


def cook_problem(mesh, mu: float = 80.194, lam: float = 400.9, tau: float = 1.0,
                 material: str = materials.M1, c_vol: Optional[float] = None,
                 follower: bool = False) -> Problem:
    """Cook's membrane: clamp x = 0, shear traction (0, tau, 0) on x = 48:
    per unit reference area (dead load, the default) or, with follower=True,
    per unit current area with fixed direction (the load in the deformed
    configuration of Sec. 4).

    f_ext is for traction tau; the residual's load_scale multiplies it.
    """
    params = (mu, lam) if material == materials.M1 else (mu, lam, 0.25 if c_vol is None else c_vol)
    ddofs = mesh.dirichlet_dofs("clamp")
    if follower:
        return Problem(mesh.X, mesh.conn, material, params, np.zeros(3 * mesh.n_nodes), ddofs,
                       np.zeros(ddofs.size), ftrac_tri=mesh.faces["load"], ftrac=(0.0, tau, 0.0))
    f_ext = dead_traction(mesh.X, mesh.faces["load"], (0.0, tau, 0.0))
    return Problem(mesh.X, mesh.conn, material, params, f_ext, ddofs, np.zeros(ddofs.size))


def cardiac_problem(mesh, consts: dict, gamma: float = 0.0) -> Problem:
    """Cardiac-like shell (Sec. 4, "Heartbeat test", quasi-static): law M4 with
    the mesh's per-element fibres and active tension gamma, follower pressure
    p_max on the endocardium (times the load scale), elastic Robin springs on
    the epicardium, base plane held in z plus three circumferential pins."""
    from synthetic import shell_dirichlet

    c = consts
    params = (c["a"], c["b"], c["af"], c["bf"], c["kappa"], gamma, mesh.elem_fibre)
    ddofs = shell_dirichlet(mesh)
    return Problem(mesh.X, mesh.conn, materials.M4, params, np.zeros(3 * mesh.n_nodes), ddofs,
                   np.zeros(ddofs.size), pressure_tri=mesh.faces["endo"], pressure=c["p_max"],
                   robin_tri=mesh.faces["epi"], k_perp=c["k_perp"], k_par=c["k_par"])


def set_active_tension(problem: Problem, gamma: float) -> None:
    """Replace the active tension gamma of an M4 or M6 problem."""
    p = list(problem.params)
    p[8 if problem.material == materials.M6 else 5] = gamma
    problem.params = tuple(p)


def guccione_problem(mesh, consts: dict, law: tuple, gamma: float = 0.0) -> Problem:
    """The heartbeat with the paper's Guccione law (M6; law = (C, b_ff,
    b_ss, b_nn, b_fs, b_fn, b_sn, B)), the mesh's fibre and sheet
    directions, and the loads and constraints of cardiac_problem."""
    from synthetic import shell_dirichlet

    c = consts
    params = tuple(law) + (gamma, mesh.elem_fibre, mesh.elem_sheet)
    ddofs = shell_dirichlet(mesh)
    return Problem(mesh.X, mesh.conn, materials.M6, params, np.zeros(3 * mesh.n_nodes), ddofs,
                   np.zeros(ddofs.size), pressure_tri=mesh.faces["endo"], pressure=c["p_max"],
                   robin_tri=mesh.faces["epi"], k_perp=c["k_perp"], k_par=c["k_par"])
