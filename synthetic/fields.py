"""Seeded vectors, load schedules, Dirichlet targets and the batch recipe.

Nothing here evaluates the method: these are the numbers a user would feed
into a solve (prescribed displacements, load factors, sampled instance
parameters) and random probe vectors for kernel parity checks.
"""

from __future__ import annotations

import math

import numpy as np


def random_field(n: int, scale: float = 1.0, seed: int = 0, dtype=np.float64) -> np.ndarray:
    """n normally distributed values N(0, scale^2) from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal(n)).astype(dtype)


def cook_load_schedule(tau: float) -> list:
    """Doubling load steps ending at tau: n_s = ceil(log2 tau) + 1 steps.

    tau = 16 gives 1, 2, 4, 8, 16; tau <= 1 gives the single step tau.
    """
    if tau <= 1.0:
        return [float(tau)]
    n_s = int(math.ceil(math.log2(tau) - 1e-12)) + 1
    return [float(tau) / 2.0 ** (n_s - 1 - s) for s in range(n_s)]


def batch_recipe(count: int = 256, seed: int = 0, mu: float = 80.194) -> list:
    """Sampled batch of Cook's-membrane instances (uneven sizes and loads).

    Draw order with rng = default_rng(seed), vectorised over the batch:
      n    = rng.integers(8, 49, count)    (nx = ny = n hexahedra)
      nz   = rng.integers(1, 4, count)
      ratio = 10 ** rng.uniform(1, 4, count)   (lambda / mu)
      tau  = 2 ** rng.uniform(0, 5, count)     (traction, N/mm^2)
    """
    rng = np.random.default_rng(seed)
    n = rng.integers(8, 49, count)
    nz = rng.integers(1, 4, count)
    ratio = 10.0 ** rng.uniform(1.0, 4.0, count)
    tau = 2.0 ** rng.uniform(0.0, 5.0, count)
    return [
        dict(nx=int(n[i]), ny=int(n[i]), nz=int(nz[i]), mu=mu, lam=float(ratio[i] * mu),
             tau=float(tau[i]))
        for i in range(count)
    ]


def twist_angles(n_steps: int = 9, total_deg: float = 90.0) -> list:
    """Rotation angles (radians) of the top face: total/n_steps * s, s = 1..n."""
    return [math.radians(total_deg * s / n_steps) for s in range(1, n_steps + 1)]


def twist_dirichlet(X: np.ndarray, bottom: np.ndarray, top: np.ndarray, theta: float,
                    axis=(0.5, 0.5)):
    """Prescribed dofs and values of the twist test at rotation angle theta.

    Bottom nodes: all three components zero.  Top nodes: the x and y
    components follow a rigid rotation by theta about the vertical line
    through `axis`; the z component stays free.  Returns (dofs int64, values
    float64) sorted by dof.
    """
    b = np.nonzero(bottom)[0].astype(np.int64)
    t = np.nonzero(top)[0].astype(np.int64)
    cx, cy = axis
    xr = X[t, 0] - cx
    yr = X[t, 1] - cy
    c, s = math.cos(theta), math.sin(theta)
    ux = c * xr - s * yr - xr
    uy = s * xr + c * yr - yr
    dofs = np.concatenate([3 * b, 3 * b + 1, 3 * b + 2, 3 * t, 3 * t + 1])
    vals = np.concatenate([np.zeros(3 * b.size), ux, uy])
    order = np.argsort(dofs, kind="stable")
    return dofs[order], vals[order]
