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
