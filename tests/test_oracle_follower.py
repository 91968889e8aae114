"""Pins of the oracle's follower Cook traction (a traction of fixed spatial
direction per unit current area, the Cook load in the deformed configuration
of Sec. 4): checked against the dead load and closed forms, not against its
own formula.

* at u = 0, and after any rigid motion (translation or rotation), the current
  face areas equal the reference ones, so the forces equal the dead load's;
* a uniform in-plane stretch of the loaded face by (s_y, s_z) scales every
  area, hence the forces, by s_y s_z;
* the complex-step Jacobian agrees with central differences of the forces;
* the follower Cook residual at u = 0 equals the dead-load Cook residual.
"""

import math

import numpy as np

import synthetic as syn
from oracle import fem

T = (0.0, 1.3, 0.0)


def _mesh():
    return syn.cook_mesh(4, 4, 2)


def test_rest_and_rigid_motions_give_the_dead_load():
    m = _mesh()
    tri = m.faces["load"]
    dead = fem.dead_traction(m.X, tri, T)
    assert np.abs(fem.follower_traction(m.X, np.zeros(3 * m.n_nodes), tri, T) - dead).max() \
        <= 1e-14 * np.abs(dead).max()
    shift = np.tile([0.3, -1.2, 2.0], m.n_nodes)
    assert np.abs(fem.follower_traction(m.X, shift, tri, T) - dead).max() <= 1e-12 * np.abs(dead).max()
    ang = 0.7
    c, s = math.cos(ang), math.sin(ang)
    R = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]]) @ \
        np.array([[1.0, 0.0, 0.0], [0.0, math.cos(0.4), -math.sin(0.4)], [0.0, math.sin(0.4), math.cos(0.4)]])
    u = (m.X @ R.T - m.X).reshape(-1)
    assert np.abs(fem.follower_traction(m.X, u, tri, T) - dead).max() <= 1e-12 * np.abs(dead).max()


def test_in_plane_stretch_scales_the_forces():
    m = _mesh()
    tri = m.faces["load"]
    sy, sz = 1.3, 0.8
    u = np.zeros((m.n_nodes, 3))
    u[:, 1] = (sy - 1.0) * m.X[:, 1]
    u[:, 2] = (sz - 1.0) * m.X[:, 2]
    f = fem.follower_traction(m.X, u.reshape(-1), tri, T)
    dead = fem.dead_traction(m.X, tri, T)
    assert np.abs(f - sy * sz * dead).max() <= 1e-12 * np.abs(dead).max()


def test_jacobian_matches_central_differences():
    m = _mesh()
    tri = m.faces["load"]
    rng = np.random.default_rng(8)
    u = 0.05 * rng.standard_normal(3 * m.n_nodes)
    K = fem.follower_traction_jacobian(m.X, u, tri, T)
    v = rng.standard_normal(3 * m.n_nodes)
    h = 1e-6
    fd = (fem.follower_traction(m.X, u + h * v, tri, T)
          - fem.follower_traction(m.X, u - h * v, tri, T)) / (2 * h)
    assert np.abs(K @ v - fd).max() <= 1e-7 * np.abs(fd).max()
    assert np.abs((K - K.T).toarray()).max() > 1e-6 * np.abs(K.toarray()).max()  # not symmetric


def test_follower_cook_at_rest_equals_dead_cook():
    m = _mesh()
    Pd = fem.cook_problem(m, tau=1.3)
    Pf = fem.cook_problem(m, tau=1.3, follower=True)
    z = np.zeros(Pd.n_dofs)
    for s in (0.5, 2.0):
        rd, rf = Pd.residual(z, s), Pf.residual(z, s)
        assert np.abs(rd - rf).max() <= 1e-13 * np.abs(rd).max()
