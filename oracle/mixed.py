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

The paper's own twist statement (Sec. 4, "Twist test") is also provided: the
inf-sup stable pair quadratic displacement / piecewise-constant pressure
(P2-P0, one pressure unknown per element: pconn of shape (n_e, 1), the
pressure test function 1 on its element) and the polyconvex law M5

    Psi(F, p) = alpha_p (F:F - 3) + beta_p (cof F : cof F - 3)
                - (4 beta_s + 2 alpha_s) ln J - p (J - 1),

cof F = J F^-T, with the printed alpha_p = beta_p = alpha_s = beta_s = 9000
(the printed "log(F)" read as ln det F, the only reading with a stress-free
reference).  Its first Piola stress, with I1 = F:F and C = F^T F (so that
cof F : cof F = (I1^2 - C:C) / 2),

    P = 2 alpha_p F + 2 beta_p (I1 F - F C) - (4 beta_s + 2 alpha_s) F^-T
        - p J F^-T.
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


def m5_energy(F, p, params):
    """The polyconvex twist law (Sec. 4): alpha_p (I1 - 3) + beta_p (I2 - 3)
    - (4 beta_s + 2 alpha_s) ln J - p (J - 1), I2 = cof F : cof F; valid for
    complex input (complex-step pins)."""
    ap, bp, as_, bs = params
    J = materials.det(F)
    cof = J[..., None, None] * materials.inv_transpose(F)
    I1 = np.einsum("...ij,...ij->...", F, F)
    I2 = np.einsum("...ij,...ij->...", cof, cof)
    return ap * (I1 - 3.0) + bp * (I2 - 3.0) - (4.0 * bs + 2.0 * as_) * np.log(J) - p * (J - 1.0)


def m5_piola(F, p, params):
    """P = 2 alpha_p F + 2 beta_p (I1 F - F C) - (4 beta_s + 2 alpha_s) F^-T
    - p J F^-T, C = F^T F (valid for complex input)."""
    ap, bp, as_, bs = params
    J = materials.det(F)
    FiT = materials.inv_transpose(F)
    I1 = np.einsum("...ij,...ij->...", F, F)
    FC = F @ np.swapaxes(F, -1, -2) @ F
    return (2.0 * ap * F + 2.0 * bp * (I1[..., None, None] * F - FC)
            - ((4.0 * bs + 2.0 * as_) + p * J)[..., None, None] * FiT)


LAWS = {"M3": lambda F, p, prm: m3_piola(F, p, prm[0]), "M5": m5_piola}


@dataclass
class MixedProblem:
    X: np.ndarray          # (n_u, 3) displacement-node coordinates
    conn: np.ndarray       # (n_e, 10)
    pconn: np.ndarray      # (n_e, 4) linear pressure, or (n_e, 1) constant per element
    n_p: int
    mu: float              # law M3's mu (unused by M5)
    ddofs: np.ndarray      # constrained displacement dofs
    dvals: np.ndarray
    law: str = "M3"
    params: tuple = ()     # law M5: (alpha_p, beta_p, alpha_s, beta_s)

    def __post_init__(self):
        self.conn = np.asarray(self.conn, dtype=np.int64)
        self.pconn = np.asarray(self.pconn, dtype=np.int64)
        if self.pconn.ndim == 1:
            self.pconn = self.pconn[:, None]
        self.npe = self.pconn.shape[1]
        if self.npe not in (1, 4):
            raise ValueError("pressure: 4 vertex values (P1) or 1 per element (P0)")
        if self.law == "M3":
            self.params = (self.mu,)
        elif self.law != "M5" or len(self.params) != 4:
            raise ValueError("law M3 (mu) or M5 (alpha_p, beta_p, alpha_s, beta_s)")
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
        # pressure shape functions at the quadrature points: the barycentric
        # coordinates (P1) or the constant 1 (P0)
        self.pbasis = QUAD_BARY if self.npe == 4 else np.ones((4, 1))
        self.piola = LAWS[self.law]

    @property
    def mu_eff(self) -> float:
        """The shear modulus of the law's small-strain limit: mu (M3),
        2 (alpha_p + beta_p) (M5, whose linearisation at rest is isotropic
        elasticity with mu = 2 (alpha_p + beta_p), lambda = 4 beta_p)."""
        if self.law == "M3":
            return self.mu
        return 2.0 * (self.params[0] + self.params[1])

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
            pq = P_nodes @ self.pbasis[q]
            w = self.V / 4.0
            P = self.piola(F, pq, self.params)
            out[:, :30] += (w[:, None, None] * np.einsum("eiJ,eaJ->eai", P, gN)).reshape(-1, 30)
            J = materials.det(F)
            out[:, 30:] += -(w * (J - 1.0))[:, None] * self.pbasis[q][None, :]
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
            pq = xe[:, 30:] @ self.pbasis[q]
            if self.law == "M5":
                L = m5_energy(F, pq, self.params)
            else:
                I1 = np.einsum("eij,eij->e", F, F)
                L = 0.5 * self.mu * (I1 - 3.0) - self.mu * np.log(J) - pq * (J - 1.0)
            tot += float(np.sum(self.V / 4.0 * L))
        return tot

    def stiffness(self, x, dirichlet: bool = True, load_scale: float = 1.0,
                  h: float = 1e-30) -> sp.csr_matrix:
        xe = x[self.edofs].astype(np.complex128)
        ne, nd = xe.shape
        Ke = np.empty((ne, nd, nd))
        for j in range(nd):
            xp = xe.copy()
            xp[:, j] += 1j * h
            Ke[:, :, j] = self.element_residual(xp).imag / h
        rows = np.repeat(self.edofs, nd, axis=1).reshape(-1)
        cols = np.tile(self.edofs, (1, nd)).reshape(-1)
        K = sp.coo_matrix((Ke.reshape(-1), (rows, cols)), shape=(self.n_dofs, self.n_dofs)).tocsr()
        if dirichlet:
            D = sp.diags(self.free.astype(np.float64))
            K = (D @ K @ D + sp.diags(self.fixed.astype(np.float64))).tocsr()
        return K

    def jv(self, x, v):
        return self.stiffness(x) @ v

    def pressure_mass_lumped(self):
        """Row sums of the pressure mass matrix: V/4 per vertex and element
        (P1), the element volume V (P0, where the mass is diagonal)."""
        m = np.zeros(self.n_p)
        np.add.at(m, self.pconn.reshape(-1), np.repeat(self.V / self.npe, self.npe))
        return m


def twist_problem(mesh, mu: float, theta: float) -> MixedProblem:
    """Twist test: bottom clamped, top x/y rotated by theta about x = y = 1/2."""
    from synthetic import twist_dirichlet

    dofs, vals = twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], theta)
    return MixedProblem(mesh.X, mesh.conn, mesh.pconn, mesh.n_pressure, mu, dofs, vals)


TWIST_M5 = (9000.0, 9000.0, 9000.0, 9000.0)  # alpha_p, beta_p, alpha_s, beta_s (Sec. 4)


def twist_problem_p0(mesh, theta: float, params=TWIST_M5) -> MixedProblem:
    """The paper's twist statement (Sec. 4): quadratic displacement, one
    pressure per element (P2-P0), law M5 with the printed constants; bottom
    clamped, top x/y rotated by theta about x = y = 1/2."""
    from synthetic import twist_dirichlet

    dofs, vals = twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], theta)
    ne = mesh.conn.shape[0]
    return MixedProblem(mesh.X, mesh.conn, np.arange(ne)[:, None], ne, 0.0, dofs, vals,
                        law="M5", params=tuple(params))


def set_twist_angle(problem: MixedProblem, mesh, theta: float) -> None:
    from synthetic import twist_dirichlet

    dofs, vals = twist_dirichlet(mesh.X, mesh.sets["bottom"], mesh.sets["top"], theta)
    assert np.array_equal(dofs, problem.ddofs)
    problem.dvals = vals
