"""Aggregation algebraic multigrid for the assembled tangent (FP64).

Test infrastructure: only the tests, the smoke check and the CPU baseline
timing use this package.

The paper preconditions its Krylov solves with algebraic multigrid (Sec. 4
and App. A: hypre's BoomerAMG through PETSc, and one AMG V-cycle as the
initial inverse Hessian of BFGS-preonly), but it does not fix the AMG's
construction.  The method defined here is a plain aggregation multigrid with
the rigid-body modes as near-nullspace (the standard choice for elasticity
with block size 3 and known coordinates):

* Level 0 is the tangent K (identity rows and columns on Dirichlet dofs) on
  the mesh's node graph (nodes adjacent when they share an element; all ten
  nodes of a quadratic element), with
  candidates B_0 (n_dofs x 6): the translations e_x, e_y, e_z and the
  rotations e_k x X (X the reference position), zero on Dirichlet dofs.
* Aggregation of a graph, in two passes over the vertices in increasing
  order: (1) a vertex whose neighbours are all unaggregated, like itself,
  forms a new aggregate with them; (2) every vertex left over joins the
  aggregate of the lowest-numbered of its neighbours that pass 1 aggregated
  (it has one: otherwise pass 1 would have made it a root).
* Tentative prolongator: for each aggregate in order, the rows of its member
  vertices' dofs (members in increasing order, each member's dofs in order);
  modified Gram-Schmidt over the six candidate columns restricted to those
  rows, in column order, keeping a column when what remains of it has norm
  above 1e-8 of its own norm (and that norm is positive).  Kept columns,
  normalised, are the aggregate's coarse dofs, numbered consecutively with
  the aggregates in order; the next candidates are the coefficients
  B_{l+1}[(a, i), k] = q_i . b_k.  An aggregate with no kept column has no
  coarse dofs and is not a vertex of the next level.
* Coarse operator A_{l+1} = P_l^T A_l P_l on the graph where two aggregates
  are adjacent when a member of one is adjacent to a member of the other.
* Coarsening stops at a level with at most N_COARSE dofs, at MAX_LEVELS
  levels, or when aggregation would not reduce the vertex count; that level
  is solved exactly.
* One V(1,1)-cycle from a zero guess: a smoothing pass before and after the
  coarse correction x += P_l V_{l+1}(P_l^T (b - A_l x)).  rho_l is the
  power-iteration estimate of the spectral radius of D_l^-1 A_l (D_l =
  diag A_l): POWER_ITS steps x <- y / |y|, y = D_l^-1 A_l x, from the fixed
  vector x_i = frac(i * 2654435761 / 2^32) - 1/2, rho_l = |y| / |x| at the
  last step.  On the finest level the pass is the Chebyshev polynomial
  smoother of degree CHEB_DEGREE in D^-1 A on [hi / CHEB_RATIO, hi],
  hi = CHEB_SAFETY rho_0: with theta, delta the interval's centre and
  half-width and sigma = theta / delta, step 1 sets d = D^-1 (b - A x) / theta
  and rho_1 = 1 / sigma; step j > 1 sets rho_j = 1 / (2 sigma - rho_{j-1}),
  d <- rho_j rho_{j-1} d + (2 rho_j / delta) D^-1 (b - A x); every step adds
  d to x.  Its error factor is T_k((theta - lambda) / delta) / T_k(sigma) on
  an eigenvalue lambda of D^-1 A (T_k the Chebyshev polynomial).  On the
  coarser levels the pass is one step of damped Jacobi x += D_l^-1 (b - A_l x)
  / rho_l.  (A fixed Jacobi weight such as 2/3 makes the smoother diverge
  here: rho(D^-1 K) is about 4 for the P1 elasticity tangent; the
  estimate's safety factor covers its shortfall, 1-7% on these tangents.)

For a symmetric A the cycle is a symmetric operator (the post-smoother is
the adjoint of the pre-smoother and restriction is the transpose of
prolongation), so it can precondition CG as well as GMRES.

Smoothed aggregation (setup(..., smooth=True)): the finest level's
prolongator is the tentative one after one damped Jacobi step,
P_0 = (I - omega D_0^-1 A_0) P_tent with omega = 4 / (3 rho_0), rho_0 the
power estimate above; the coarser levels keep their tentative prolongators.
On a floating body A_0 annihilates the rigid motions, so P_0 still
reproduces them, and since |1 - omega lambda| <= 1 on the spectrum of
D^-1 A the smoothing never raises a column's energy.  The coarse graph of
level 1 is then the aggregates' member adjacency as before (A_1's own
pattern is wider).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

POWER_ITS = 15
CHEB_DEGREE = 2
CHEB_RATIO = 30.0
CHEB_SAFETY = 1.2
N_COARSE = 300
MAX_LEVELS = 10
DROP_TOL = 1e-8


def node_graph(conn: np.ndarray, n_nodes: int) -> list:
    """Sorted neighbour lists of the mesh's nodes (sharing an element)."""
    nb = [set() for _ in range(n_nodes)]
    for e in np.asarray(conn):
        for a in e:
            for b in e:
                if a != b:
                    nb[int(a)].add(int(b))
    return [sorted(s) for s in nb]


def aggregate(adj: list) -> tuple:
    """Two-pass greedy aggregation; returns (aggregate id per vertex, count)."""
    n = len(adj)
    agg = np.full(n, -1, dtype=np.int64)
    n_agg = 0
    for v in range(n):
        if agg[v] >= 0:
            continue
        if all(agg[w] < 0 for w in adj[v]):
            agg[v] = n_agg
            for w in adj[v]:
                agg[w] = n_agg
            n_agg += 1
    first = agg.copy()
    for v in range(n):
        if agg[v] < 0:
            joined = [w for w in adj[v] if first[w] >= 0]
            assert joined
            agg[v] = first[min(joined)]
    return agg, n_agg


def rigid_modes(X: np.ndarray, fixed: np.ndarray) -> np.ndarray:
    """Translations and rotations e_k x X as columns (node-interleaved), zero
    on Dirichlet dofs."""
    n = X.shape[0]
    B = np.zeros((3 * n, 6))
    for d in range(3):
        B[d::3, d] = 1.0
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    # e_x x X = (0, -z, y); e_y x X = (z, 0, -x); e_z x X = (-y, x, 0)
    B[1::3, 3], B[2::3, 3] = -z, y
    B[0::3, 4], B[2::3, 4] = z, -x
    B[0::3, 5], B[1::3, 5] = -y, x
    B[np.asarray(fixed, dtype=bool)] = 0.0
    return B


def tentative(B: np.ndarray, rows_of: list) -> tuple:
    """Modified Gram-Schmidt per aggregate.  rows_of[a] lists aggregate a's
    rows; returns (P as CSR, next candidates, coarse dof count per aggregate)."""
    n = B.shape[0]
    Pr, Pc, Pv, Bn, kcount = [], [], [], [], []
    col = 0
    for rows in rows_of:
        Ba = B[rows, :]
        qs, R = [], []
        for k in range(6):
            b = Ba[:, k]
            nb = np.linalg.norm(b)
            v = b.copy()
            for q in qs:
                v = v - (q @ v) * q
            nv = np.linalg.norm(v)
            if nb > 0.0 and nv > DROP_TOL * nb:
                qs.append(v / nv)
        for i, q in enumerate(qs):
            R.append([q @ Ba[:, k] for k in range(6)])
            Pr.extend(rows)
            Pc.extend([col + i] * len(rows))
            Pv.extend(q.tolist())
        Bn.extend(R)
        kcount.append(len(qs))
        col += len(qs)
    P = sp.csr_matrix((Pv, (Pr, Pc)), shape=(n, col))
    return P, np.array(Bn).reshape(-1, 6), np.array(kcount, dtype=np.int64)


@dataclass
class Hierarchy:
    A: list = field(default_factory=list)      # A_l (CSR), l = 0..L
    P: list = field(default_factory=list)      # P_l (CSR), l = 0..L-1
    D: list = field(default_factory=list)      # diag A_l
    w: list = field(default_factory=list)      # 1 / rho_l (Jacobi weight on levels > 0)
    aggs: list = field(default_factory=list)   # aggregate id per vertex, per level
    kcount: list = field(default_factory=list)

    @property
    def n_levels(self) -> int:
        return len(self.A)


SA_OMEGA = 4.0 / 3.0  # omega rho_0 of the smoothed prolongator


def setup(K, X: np.ndarray, conn: np.ndarray, fixed: np.ndarray,
          smooth: bool = False) -> Hierarchy:
    """The hierarchy of K for the mesh (X, conn) with Dirichlet mask `fixed`;
    smooth: smoothed aggregation on the finest level."""
    K = sp.csr_matrix(K)
    n_nodes = X.shape[0]
    H = Hierarchy()
    A = K
    adj = node_graph(conn, n_nodes)
    # the dofs of each vertex of the current level
    vdofs = [[3 * v, 3 * v + 1, 3 * v + 2] for v in range(n_nodes)]
    B = rigid_modes(X, fixed)
    while True:
        H.A.append(A)
        H.D.append(A.diagonal().copy())
        if A.shape[0] <= N_COARSE or len(H.A) == MAX_LEVELS:
            break
        H.w.append(1.0 / spectral_radius(A, H.D[-1]))
        agg, n_agg = aggregate(adj)
        if n_agg >= len(adj):
            break
        members = [[] for _ in range(n_agg)]
        for v in range(len(adj)):
            members[agg[v]].append(v)
        rows_of = [[r for v in m for r in vdofs[v]] for m in members]
        P, Bn, kc = tentative(B, rows_of)
        if smooth and not H.P:
            # one damped Jacobi step on the tentative columns
            omega = SA_OMEGA * H.w[-1]
            P = (P - omega * (sp.diags(1.0 / H.D[-1]) @ (A @ P))).tocsr()
        H.P.append(P)
        H.aggs.append(agg)
        H.kcount.append(kc)
        # next level: aggregates with coarse dofs, adjacency through members
        keep = np.flatnonzero(kc > 0)
        newid = -np.ones(n_agg, dtype=np.int64)
        newid[keep] = np.arange(keep.size)
        off = np.concatenate([[0], np.cumsum(kc)])
        vdofs = [list(range(off[a], off[a + 1])) for a in keep]
        nb = [set() for _ in range(keep.size)]
        for v in range(len(adj)):
            a = newid[agg[v]]
            if a < 0:
                continue
            for w in adj[v]:
                b = newid[agg[w]]
                if b >= 0 and b != a:
                    nb[a].add(int(b))
        adj = [sorted(s) for s in nb]
        A = (P.T @ A @ P).tocsr()
        B = Bn
    if len(H.w) == len(H.A):  # the last level turned out to be the coarsest
        H.w.pop()
    return H


def start_vector(n: int) -> np.ndarray:
    """x_i = frac(i * 2654435761 / 2^32) - 1/2 (exact integer arithmetic)."""
    i = np.arange(n, dtype=np.uint64)
    return ((i * np.uint64(2654435761)) % np.uint64(2 ** 32)).astype(np.float64) / 2.0 ** 32 - 0.5


def spectral_radius(A, D: np.ndarray) -> float:
    """Power-iteration estimate of rho(D^-1 A) (POWER_ITS steps)."""
    x = start_vector(A.shape[0])
    lam = 0.0
    for _ in range(POWER_ITS):
        y = (A @ x) / D
        ny = np.linalg.norm(y)
        lam = ny / np.linalg.norm(x)
        x = y / ny
    return lam


def vcycle(H: Hierarchy, b: np.ndarray, level: int = 0) -> np.ndarray:
    """One V(1,1)-cycle for A_level x = b from x = 0."""
    A = H.A[level]
    if level == H.n_levels - 1:
        return np.linalg.solve(A.toarray(), b)
    D = H.D[level]
    P = H.P[level]
    w = H.w[level]
    if level == 0:
        x = chebyshev(A, D, b, np.zeros_like(b), 1.0 / w)
    else:
        x = w * b / D
    r = b - A @ x
    x = x + P @ vcycle(H, P.T @ r, level + 1)
    if level == 0:
        return chebyshev(A, D, b, x, 1.0 / w)
    return x + w * (b - A @ x) / D


def chebyshev(A, D: np.ndarray, b: np.ndarray, x: np.ndarray, rho: float,
              degree: int = None) -> np.ndarray:
    """CHEB_DEGREE steps of the Chebyshev smoother for A x = b from x."""
    k = CHEB_DEGREE if degree is None else degree
    hi = CHEB_SAFETY * rho
    lo = hi / CHEB_RATIO
    theta, delta = 0.5 * (hi + lo), 0.5 * (hi - lo)
    sigma = theta / delta
    x = np.array(x, dtype=np.float64, copy=True)
    d = (b - A @ x) / D / theta
    x = x + d
    rho_prev = 1.0 / sigma
    for _ in range(k - 1):
        rho_j = 1.0 / (2.0 * sigma - rho_prev)
        d = rho_j * rho_prev * d + (2.0 * rho_j / delta) * (b - A @ x) / D
        x = x + d
        rho_prev = rho_j
    return x


def gmres_amg(K, H: Hierarchy, b: np.ndarray, rtol: float, atol: float = 0.0,
              max_it: int = 1000) -> tuple:
    """Unrestarted right-preconditioned GMRES (modified Gram-Schmidt) with the
    V-cycle, from x = 0; returns (x, iterations).  Stops when the least-squares
    residual norm is at most max(rtol ||b||, atol)."""
    n = b.size
    beta = np.linalg.norm(b)
    tol = max(rtol * beta, atol)
    if beta <= tol:
        return np.zeros(n), 0
    V = [b / beta]
    Z = []
    Hm = np.zeros((max_it + 1, max_it))
    g = np.zeros(max_it + 1)
    g[0] = beta
    it = 0
    for j in range(max_it):
        z = vcycle(H, V[j])
        Z.append(z)
        w = K @ z
        for i in range(j + 1):
            Hm[i, j] = V[i] @ w
            w = w - Hm[i, j] * V[i]
        Hm[j + 1, j] = np.linalg.norm(w)
        it = j + 1
        y, res = _lsq(Hm[:j + 2, :j + 1], g[:j + 2])
        if res <= tol or Hm[j + 1, j] == 0.0:
            break
        V.append(w / Hm[j + 1, j])
    y, _ = _lsq(Hm[:it + 1, :it], g[:it + 1])
    return np.array(Z).T @ y, it


def _lsq(Hs, g):
    y, *_ = np.linalg.lstsq(Hs, g, rcond=None)
    return y, float(np.linalg.norm(g - Hs @ y))
