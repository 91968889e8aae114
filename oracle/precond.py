"""Jacobi-type preconditioners of the assembled tangent (FP64).

Test infrastructure: only the tests, the smoke check and the CPU baseline
timing use this package.

The Krylov solvers of the paper are preconditioned (Sec. 3 and App. A, where
the nonlinear solvers' linear systems run through PETSc with a
preconditioner and block size 3).  Two diagonal preconditioners are defined
here from the assembled tangent K of `fem.Problem.stiffness`:

* point Jacobi: M = diag(K);
* nodal block Jacobi (point-block Jacobi with block size 3): M is block
  diagonal with, for node k, the 3x3 block K[3k:3k+3, 3k:3k+3].

The strain-energy and Robin-spring parts of a node's own block are
symmetric.  A follower pressure adds a skew-symmetric part only: the load at
vertex a of a face is p/6 times (x_b - x_a) x (x_c - x_a), whose derivative
with respect to x_a is the cross-product map d -> d x (x_b - x_c).  The block
preconditioner takes the symmetric part of each block, which is then the
strain-energy and spring part.  Dirichlet dofs have identity rows and
columns in K, hence in the blocks.
"""

from __future__ import annotations

import numpy as np


def node_blocks(K, n_nodes: int) -> np.ndarray:
    """Symmetric parts of the 3x3 diagonal blocks of K, shape (n_nodes, 3, 3)."""
    K = K.tocsr()
    B = np.empty((n_nodes, 3, 3))
    for k in range(n_nodes):
        blk = K[3 * k:3 * k + 3, 3 * k:3 * k + 3].toarray()
        B[k] = 0.5 * (blk + blk.T)
    return B


def block_jacobi_apply(blocks: np.ndarray, x: np.ndarray) -> np.ndarray:
    """z with blocks[k] z_k = x_k for every node k (z, x node-interleaved).

    A block that is not positive definite (some leading principal minor
    <= 0) is replaced by its diagonal, so the preconditioner is positive
    definite wherever point Jacobi is (the reading of the nodal block Jacobi
    used here)."""
    B = np.array(blocks, dtype=np.float64, copy=True)
    m1 = B[:, 0, 0]
    m2 = B[:, 0, 0] * B[:, 1, 1] - B[:, 0, 1] * B[:, 1, 0]
    m3 = np.linalg.det(B)
    bad = ~((m1 > 0) & (m2 > 0) & (m3 > 0))
    if np.any(bad):
        diag = np.einsum("kii->ki", B[bad])
        B[bad] = np.einsum("ki,ij->kij", diag, np.eye(3))
    xk = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    return np.linalg.solve(B, xk[:, :, None])[:, :, 0].reshape(-1)


def point_jacobi_apply(K, x: np.ndarray) -> np.ndarray:
    """z = x / diag(K)."""
    return np.asarray(x, dtype=np.float64) / K.diagonal()


def pcg(K, b: np.ndarray, apply_minv, rtol: float = 1e-10, max_it: int = 10000):
    """Textbook preconditioned CG from x = 0 (Hestenes-Stiefel form); returns
    (x, iterations).  Stops when ||b - K x|| <= rtol ||b||."""
    x = np.zeros_like(b)
    r = b.copy()
    z = apply_minv(r)
    p = z.copy()
    rz = r @ z
    nb = np.linalg.norm(b)
    for it in range(max_it):
        if np.linalg.norm(r) <= rtol * nb:
            return x, it
        q = K @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = apply_minv(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, max_it


# ---- block preconditioners of the displacement / pressure saddle point ------
# App. B: with the tangent in blocks M = [[A, B1], [B2, C]] (displacement
# rows first), a Schur complement preconditioner comes from the block LU
# factorisation M = L D U, L = [[I, 0], [B2 A^-1, I]], D = diag(A, S),
# S = C - B2 A^-1 B1.  The lower form keeps L D = [[A, 0], [B2, S]]; its
# inverse applied to r = (r_u, r_p) is
#     z_u = A^-1 r_u,   z_p = S^-1 (r_p - B2 z_u).
# The twist test (Sec. 4) approximates A^-1 by the displacement block's
# preconditioner and S by SIMPLE, S ~ C - B2 diag(A)^-1 B1 (here C = 0, the
# law is linear in p), whose diagonal stands in for the Schur block's own
# preconditioner.  The block-diagonal form (middle factor only) is available
# too; with C = 0 it is the variant App. B allows.

def saddle_blocks(K, n_u: int):
    """(A, B2) of the assembled tangent: the displacement block and the
    pressure rows' displacement columns (Dirichlet columns are already zero
    in K's pressure rows, Dirichlet rows of A are identity rows)."""
    K = K.tocsr()
    return K[:n_u, :n_u], K[n_u:, :n_u]


def simple_schur_diagonal(K, n_u: int) -> np.ndarray:
    """The diagonal of B2 diag(A)^-1 B2^T (positive): minus the diagonal of
    the SIMPLE Schur approximation C - B2 diag(A)^-1 B1 with C = 0, B1 = B2^T."""
    A, B = saddle_blocks(K, n_u)
    d = A.diagonal()
    Bsq = B.multiply(B)
    return np.asarray(Bsq @ (1.0 / d)).reshape(-1)


def schur_lower_apply(K, n_u: int, r: np.ndarray, apply_a, s_diag: np.ndarray) -> np.ndarray:
    """z = (L D)^-1 r for the lower block-triangular preconditioner with the
    Schur block approximated by -diag(s_diag) (s_diag > 0):
    z_u = apply_a(r_u), z_p = -(r_p - B2 z_u) / s_diag."""
    _, B = saddle_blocks(K, n_u)
    zu = apply_a(r[:n_u])
    zp = -(r[n_u:] - B @ zu) / s_diag
    return np.concatenate([zu, zp])
