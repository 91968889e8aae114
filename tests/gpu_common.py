"""Shared helpers for the GPU tests (not collected as tests itself)."""

import numpy as np

import synthetic as syn

MU = 80.194


def smooth_state(mesh, n_dofs, seed, amp=0.02):
    """A deformation with moderate gradients: affine part plus scaled noise."""
    rng = np.random.default_rng(seed)
    A = amp * rng.standard_normal((3, 3))
    c = mesh.conn[:, :4]
    h = min(np.linalg.norm(mesh.X[c[:, a]] - mesh.X[c[:, b]], axis=1).min()
            for a in range(4) for b in range(a))
    u = (mesh.X @ A.T).reshape(-1) + 0.03 * h * syn.random_field(n_dofs, 1.0, seed=seed + 1)
    return u


def relmax(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


EPS32 = 2.0 ** -23


def row_magnitude(K, v, P=None, u=None):
    """(|K| |v|)_i, the size of the terms that make up entry i of K v: the
    assembled operator's absolute values, and for P1 problems also the sum
    over elements of |K_e| |v_e| (entries of K that cancel in the assembly
    still carry their own rounding)."""
    import scipy.sparse as sp

    m = abs(sp.csr_matrix(K)) @ np.abs(v)
    conn = getattr(P, "conn", None)
    if P is not None and conn is not None and conn.shape[1] == 4 and hasattr(P, "element_stiffness"):
        Ke = np.abs(P.element_stiffness(u))                     # (e, 12, 12)
        dofs = (3 * conn[:, :, None] + np.arange(3)[None, None, :]).reshape(-1, 12)
        ve = np.abs(v)[dofs]                                    # (e, 12)
        me = np.einsum("eij,ej->ei", Ke, ve)
        m = np.maximum(m, np.bincount(dofs.reshape(-1), weights=me.reshape(-1), minlength=v.size))
    return m


def assert_fp32_entrywise(y32, ref, mag, c=64.0, dir_dofs=None, v=None, what="J v"):
    """Entry by entry: |y32_i - ref_i| <= c eps32 (|K| |v|)_i, and, on the
    Dirichlet dofs (identity rows), y32 equal to v rounded to FP32 bit for
    bit."""
    y = np.asarray(y32, dtype=np.float64)
    bound = c * EPS32 * np.asarray(mag) + 1e-300
    ratio = np.abs(y - ref) / bound
    k = int(np.argmax(ratio))
    assert ratio[k] <= 1.0, (f"{what}: FP32 entry {k} off by {abs(y[k] - ref[k]):.3e}, "
                             f"bound {bound[k]:.3e} (ratio {ratio[k]:.2f})")
    if dir_dofs is not None and len(dir_dofs) > 0:
        want = np.asarray(v, dtype=np.float64).astype(np.float32)[dir_dofs]
        assert np.array_equal(np.asarray(y32, dtype=np.float32)[dir_dofs], want), \
            f"{what}: Dirichlet rows differ from v"
    return float(ratio[k])
