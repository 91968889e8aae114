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


# Cardiac-like workload (heartbeat test of Sec. 4 with a substitute law; units
# mm, N, MPa).  Builder-chosen constants: passive a, b (isotropic exponential),
# af = 2a, bf (fibre exponential), kappa = 1000 a (volumetric penalty); peak
# active tension 60 kPa and endocardial pressure 2 kPa; epicardial springs
# K_perp, K_par per unit reference area.  The passive stiffness a = 0.1 MPa is
# the softest tried (0.01, 0.05, 0.1) for which every one of the 20 steps
# converges with full Newton steps from the previous step.
CARDIAC = dict(a=0.1, b=5.0, af=0.2, bf=5.0, kappa=100.0, gamma_max=0.06, p_max=0.002,
               k_perp=2e-4, k_par=2e-5, period=0.8, dt=0.02, n_steps=20)


def heartbeat_schedule(n_steps: int = 20, dt: float = 0.02, period: float = 0.8) -> list:
    """Time steps t_n = n dt (n = 1..n_steps) and the activation shape
    max(sin(2 pi t_n / period), 0) of Sec. 4 ("Heartbeat test"); the active
    tension and the endocardial pressure both follow this shape."""
    return [(n * dt, max(math.sin(2.0 * math.pi * n * dt / period), 0.0))
            for n in range(1, n_steps + 1)]


def shell_dirichlet(mesh) -> np.ndarray:
    """Constrained dofs of the ventricle shell: u_z = 0 on the base plane,
    plus three circumferential pins on the endocardial base ring (at its
    +x, +y and -x extremes: u_y, u_x and u_y) against rigid rotation about
    z and in-plane translation.  Returns sorted dof numbers (values zero)."""
    base = np.nonzero(mesh.sets["base"])[0]
    ring = base[mesh.sets["endo"][base]]
    X = mesh.X
    px = ring[np.argmax(X[ring, 0])]
    py = ring[np.argmax(X[ring, 1])]
    mx = ring[np.argmin(X[ring, 0])]
    dofs = np.concatenate([3 * base + 2, [3 * px + 1, 3 * py + 0, 3 * mx + 1]])
    return np.sort(dofs.astype(np.int64))
