"""Structured tetrahedral meshes standing in for the paper's test geometries.

Every hexahedral cell of a structured index grid is cut into six tetrahedra
along its (0,0,0)-(1,1,1) diagonal (Kuhn / Freudenthal split).  The split is
the same in every cell, so neighbouring cells cut their shared quadrilateral
face along the same diagonal and the tetrahedral mesh is conforming.  Each
tetrahedron is stored with positive orientation: det[X1-X0, X2-X0, X3-X0] > 0.

Geometries (Sec. 4 of the paper, with the synthetic sizes of the workloads):

* Cook's membrane: the quadrilateral (0,0), (48,44), (48,60), (0,44) mm,
  extruded 10 mm in z, clamped on x = 0, loaded on x = 48.
* Unit cube (twist test), optionally with quadratic (10-node) tetrahedra
  and a linear pressure grid for the mixed displacement / pressure form.
* Truncated prolate-ellipsoid shell (idealised left ventricle) with a
  circumferentially periodic grid, base at z = 0, apex towards -z.

Node numbering is lexicographic in the grid indices (first index fastest).
Vectors built on these meshes interleave the three displacement components
per node: dof = 3 * node + component.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

COOK_CORNERS = np.array([[0.0, 0.0], [48.0, 44.0], [48.0, 60.0], [0.0, 44.0]])
COOK_THICKNESS = 10.0

# Kuhn split: for each permutation p of the axes the tetrahedron walks
# 000 -> e_p0 -> e_p0 + e_p1 -> 111 along the cell's edges.
_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def _kuhn_offsets() -> np.ndarray:
    """(6, 4, 3) integer corner offsets of the six tetrahedra of a cell."""
    out = np.zeros((6, 4, 3), dtype=np.int64)
    for t, p in enumerate(_PERMS):
        cur = np.zeros(3, dtype=np.int64)
        out[t, 0] = cur
        for s in range(2):
            cur = cur.copy()
            cur[p[s]] += 1
            out[t, s + 1] = cur
        out[t, 3] = (1, 1, 1)
    return out


_KUHN = _kuhn_offsets()

# local face -> the vertex it does not contain
_TET_FACES = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
_TET_OPPOSITE = np.array([0, 1, 2, 3])


@dataclass
class Mesh:
    """A tetrahedral mesh plus the node / face sets the workloads need.

    X      : (n_nodes, 3) float64 reference coordinates.
    conn   : (n_elems, 4) or (n_elems, 10) int32 connectivity.
    pconn  : optional (n_elems, 4) int32 connectivity into a separate linear
             pressure grid of n_pressure nodes (mixed form only).
    sets   : named boolean node masks (e.g. 'clamp', 'load', 'base').
    faces  : named (n_faces, 3) int32 outward-oriented boundary triangles.
    elem_fibre : optional (n_elems, 3) unit fibre direction per element.
    elem_sheet : optional (n_elems, 3) unit sheet direction per element,
             orthogonal to the fibre (the transmural direction).
    grid   : the hexahedral grid size the mesh came from.
    """

    X: np.ndarray
    conn: np.ndarray
    pconn: Optional[np.ndarray] = None
    n_pressure: int = 0
    sets: Dict[str, np.ndarray] = field(default_factory=dict)
    faces: Dict[str, np.ndarray] = field(default_factory=dict)
    elem_fibre: Optional[np.ndarray] = None
    elem_sheet: Optional[np.ndarray] = None
    grid: tuple = ()
    name: str = ""

    @property
    def n_nodes(self) -> int:
        return int(self.X.shape[0])

    @property
    def n_elems(self) -> int:
        return int(self.conn.shape[0])

    @property
    def n_dofs(self) -> int:
        return 3 * self.n_nodes

    def dirichlet_dofs(self, set_name: str, components=(0, 1, 2)) -> np.ndarray:
        nodes = np.nonzero(self.sets[set_name])[0].astype(np.int64)
        comps = np.asarray(components, dtype=np.int64)
        return (3 * nodes[:, None] + comps[None, :]).reshape(-1)


def _kuhn_connectivity(nx: int, ny: int, nz: int, node_id) -> np.ndarray:
    """Connectivity of the Kuhn split of an nx*ny*nz cell grid.

    node_id(i, j, k) maps integer grid indices (arrays) to node numbers;
    cells are ordered lexicographically, six consecutive tets per cell.
    """
    ci, cj, ck = np.meshgrid(
        np.arange(nx, dtype=np.int64),
        np.arange(ny, dtype=np.int64),
        np.arange(nz, dtype=np.int64),
        indexing="ij",
    )
    # lexicographic cell order with the first index fastest
    ci = ci.transpose(2, 1, 0).reshape(-1)
    cj = cj.transpose(2, 1, 0).reshape(-1)
    ck = ck.transpose(2, 1, 0).reshape(-1)
    conn = np.empty((ci.size, 6, 4), dtype=np.int64)
    for t in range(6):
        for v in range(4):
            o = _KUHN[t, v]
            conn[:, t, v] = node_id(ci + o[0], cj + o[1], ck + o[2])
    return conn.reshape(-1, 4)


def _orient_positive(X: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """Swap vertices 2 and 3 of every tetrahedron with negative volume."""
    x0 = X[conn[:, 0]]
    d1 = X[conn[:, 1]] - x0
    d2 = X[conn[:, 2]] - x0
    d3 = X[conn[:, 3]] - x0
    det = np.einsum("ij,ij->i", d1, np.cross(d2, d3))
    neg = det < 0
    conn = conn.copy()
    conn[neg, 2], conn[neg, 3] = conn[neg, 3].copy(), conn[neg, 2].copy()
    return conn


def boundary_faces(X: np.ndarray, conn: np.ndarray, node_mask: np.ndarray) -> np.ndarray:
    """Outward-oriented element faces whose three vertices all lie in node_mask.

    Meant for a set of nodes forming one layer of the structured grid; such a
    face then lies on the boundary and belongs to exactly one tetrahedron.
    The returned triangle (a, b, c) has (X_b - X_a) x (X_c - X_a) pointing
    away from the element's fourth vertex.
    """
    c4 = conn[:, :4]
    out = []
    for f in range(4):
        tri = c4[:, _TET_FACES[f]]
        sel = node_mask[tri].all(axis=1)
        if not sel.any():
            continue
        tri = tri[sel].copy()
        opp = c4[sel, _TET_OPPOSITE[f]]
        xa = X[tri[:, 0]]
        nrm = np.cross(X[tri[:, 1]] - xa, X[tri[:, 2]] - xa)
        inward = np.einsum("ij,ij->i", nrm, X[opp] - xa) > 0
        tri[inward, 1], tri[inward, 2] = tri[inward, 2].copy(), tri[inward, 1].copy()
        out.append(tri)
    if not out:
        return np.zeros((0, 3), dtype=np.int32)
    return np.concatenate(out).astype(np.int32)


def cook_mesh(nx: int, ny: int, nz: int, with_faces: bool = True) -> Mesh:
    """Cook's membrane, nx*ny*nz hexahedra, six P1 tetrahedra each.

    The unit square is mapped bilinearly onto the quadrilateral with corners
    COOK_CORNERS and extruded to thickness 10.  All four sides of the
    quadrilateral are straight, so the tetrahedra tile the body exactly
    (total volume 1440 * 10 = 14400).  Sets: 'clamp' (x = 0), 'load' (x = 48);
    faces: 'load' (the 2*ny*nz triangles on x = 48).
    """
    nnx, nny, nnz = nx + 1, ny + 1, nz + 1
    xi = np.arange(nnx) / nx
    eta = np.arange(nny) / ny
    zeta = np.arange(nnz) / nz
    Z, E, XI = np.meshgrid(zeta, eta, xi, indexing="ij")  # k slowest, i fastest
    XI, E, Z = XI.reshape(-1), E.reshape(-1), Z.reshape(-1)
    p00, p10, p11, p01 = COOK_CORNERS
    xy = (
        ((1 - XI) * (1 - E))[:, None] * p00
        + (XI * (1 - E))[:, None] * p10
        + (XI * E)[:, None] * p11
        + ((1 - XI) * E)[:, None] * p01
    )
    X = np.column_stack([xy, COOK_THICKNESS * Z])
    # exact x on the two vertical sides (the bilinear map already gives them)
    X[np.isclose(XI, 0.0), 0] = 0.0
    X[np.isclose(XI, 1.0), 0] = 48.0

    def nid(i, j, k):
        return i + nnx * (j + nny * k)

    conn = _orient_positive(X, _kuhn_connectivity(nx, ny, nz, nid)).astype(np.int32)
    ii = np.tile(np.arange(nnx), nny * nnz)
    sets = {"clamp": ii == 0, "load": ii == nx}
    faces = {}
    if with_faces:
        faces["load"] = boundary_faces(X, conn, sets["load"])
    return Mesh(X=X, conn=conn, sets=sets, faces=faces, grid=(nx, ny, nz),
                name=f"cook{nx}x{ny}x{nz}")


def cube_mesh(n: int) -> Mesh:
    """Unit cube, n^3 hexahedra, six P1 tetrahedra each.

    Sets: 'bottom' (z = 0), 'top' (z = 1).
    """
    nn = n + 1
    g = np.arange(nn) / n
    Z, Y, Xc = np.meshgrid(g, g, g, indexing="ij")
    X = np.column_stack([Xc.reshape(-1), Y.reshape(-1), Z.reshape(-1)])

    def nid(i, j, k):
        return i + nn * (j + nn * k)

    conn = _orient_positive(X, _kuhn_connectivity(n, n, n, nid)).astype(np.int32)
    kk = np.repeat(np.arange(nn), nn * nn)
    return Mesh(X=X, conn=conn, sets={"bottom": kk == 0, "top": kk == n},
                grid=(n, n, n), name=f"cube{n}")


# Quadratic tetrahedron node order: the four vertices, then the edge
# midpoints of edges (0,1), (1,2), (0,2), (0,3), (1,3), (2,3).
P2_EDGES = ((0, 1), (1, 2), (0, 2), (0, 3), (1, 3), (2, 3))


def twist_p2_mesh(n: int) -> Mesh:
    """Unit cube with quadratic displacement / linear pressure tetrahedra.

    Displacement nodes live on the doubled grid (2n+1)^3: a vertex (i,j,k)
    of the cell grid is node (2i,2j,2k) and the midpoint of an edge is the
    average of its end points in doubled indices.  The pressure grid is the
    vertex grid (n+1)^3 with its own lexicographic numbering.
    Sets: 'bottom' (z = 0), 'top' (z = 1) over displacement nodes.
    """
    m = 2 * n + 1
    g = np.arange(m) / (2 * n)
    Z, Y, Xc = np.meshgrid(g, g, g, indexing="ij")
    X = np.column_stack([Xc.reshape(-1), Y.reshape(-1), Z.reshape(-1)])
    nn = n + 1

    # vertex connectivity in doubled indices, oriented on the vertex grid
    def pid(i, j, k):
        return i + nn * (j + nn * k)

    gv = np.arange(nn) / n
    Zp, Yp, Xp = np.meshgrid(gv, gv, gv, indexing="ij")
    Xpres = np.column_stack([Xp.reshape(-1), Yp.reshape(-1), Zp.reshape(-1)])
    pconn = _orient_positive(Xpres, _kuhn_connectivity(n, n, n, pid))
    # pressure node (i,j,k) -> displacement node (2i,2j,2k)
    pk, rem = np.divmod(pconn, nn * nn)
    pj, pi = np.divmod(rem, nn)
    di, dj, dk = 2 * pi, 2 * pj, 2 * pk
    conn = np.empty((pconn.shape[0], 10), dtype=np.int64)
    conn[:, :4] = di + m * (dj + m * dk)
    for e, (a, b) in enumerate(P2_EDGES):
        conn[:, 4 + e] = ((di[:, a] + di[:, b]) // 2
                          + m * ((dj[:, a] + dj[:, b]) // 2 + m * ((dk[:, a] + dk[:, b]) // 2)))
    kk = np.repeat(np.arange(m), m * m)
    return Mesh(X=X, conn=conn.astype(np.int32), pconn=pconn.astype(np.int32),
                n_pressure=nn ** 3, sets={"bottom": kk == 0, "top": kk == m - 1},
                grid=(n, n, n), name=f"twist{n}")


def shell_mesh(n_t: int = 8, n_s: int = 80, n_c: int = 256,
               inner=(25.0, 70.0), outer=(35.0, 80.0), theta_apex: float = 0.1) -> Mesh:
    """Truncated prolate-ellipsoid shell (idealised left ventricle).

    Parameter grid: transmural t = i/n_t (0 endocardium, 1 epicardium),
    longitudinal theta from theta_apex (near the apex) to pi/2 (the base),
    circumferential phi = 2 pi k / n_c (periodic).  With a(t), c(t) the
    interpolated equatorial and longitudinal semi-axes:
        x = a sin(theta) cos(phi), y = a sin(theta) sin(phi), z = -c cos(theta),
    so the base is the plane z = 0 and the body lies in z <= 0.  A small
    opening at the apex (theta >= theta_apex) avoids degenerate tetrahedra.

    Per-element fibre: angle alpha = -60 deg + 120 deg * t at the element
    centroid, f = cos(alpha) e_circ + sin(alpha) e_long in the local
    circumferential / longitudinal tangent plane.
    Sets: 'endo', 'epi', 'base'; faces: 'endo', 'epi' (outward from the wall).
    """
    nti, nsi = n_t + 1, n_s + 1
    t = np.arange(nti) / n_t
    th = theta_apex + (np.pi / 2 - theta_apex) * np.arange(nsi) / n_s
    ph = 2 * np.pi * np.arange(n_c) / n_c
    K, J, I = np.meshgrid(np.arange(n_c), np.arange(nsi), np.arange(nti), indexing="ij")
    I, J, K = I.reshape(-1), J.reshape(-1), K.reshape(-1)
    a = inner[0] + (outer[0] - inner[0]) * t[I]
    c = inner[1] + (outer[1] - inner[1]) * t[I]
    X = np.column_stack([
        a * np.sin(th[J]) * np.cos(ph[K]),
        a * np.sin(th[J]) * np.sin(ph[K]),
        -c * np.cos(th[J]),
    ])
    X[J == n_s, 2] = 0.0

    def nid(i, j, k):
        return i + nti * (j + nsi * (k % n_c))

    conn = _orient_positive(X, _kuhn_connectivity(n_t, n_s, n_c, nid)).astype(np.int32)
    sets = {"endo": I == 0, "epi": I == n_t, "base": J == n_s}
    faces = {"endo": boundary_faces(X, conn, sets["endo"]),
             "epi": boundary_faces(X, conn, sets["epi"])}
    # fibres from centroid parameters (periodic phi handled via the unit circle)
    ic = I[conn].mean(axis=1) / n_t
    jc = J[conn].mean(axis=1)
    thc = theta_apex + (np.pi / 2 - theta_apex) * jc / n_s
    phc = np.arctan2(np.sin(ph[K[conn]]).mean(axis=1), np.cos(ph[K[conn]]).mean(axis=1))
    ac = inner[0] + (outer[0] - inner[0]) * ic
    cc = inner[1] + (outer[1] - inner[1]) * ic
    e_circ = np.column_stack([-np.sin(phc), np.cos(phc), np.zeros_like(phc)])
    e_long = np.column_stack([ac * np.cos(thc) * np.cos(phc), ac * np.cos(thc) * np.sin(phc),
                              cc * np.sin(thc)])
    e_long /= np.linalg.norm(e_long, axis=1)[:, None]
    alpha = np.deg2rad(-60.0 + 120.0 * ic)
    fib = np.cos(alpha)[:, None] * e_circ + np.sin(alpha)[:, None] * e_long
    fib /= np.linalg.norm(fib, axis=1)[:, None]
    # sheet: the transmural unit normal of the (circumferential, longitudinal)
    # tangent plane, orthogonal to the fibre
    sheet = np.cross(e_circ, e_long)
    sheet /= np.linalg.norm(sheet, axis=1)[:, None]
    return Mesh(X=X, conn=conn, sets=sets, faces=faces, elem_fibre=fib, elem_sheet=sheet,
                grid=(n_t, n_s, n_c), name=f"shell{n_t}x{n_s}x{n_c}")


def p2_from_p1(mesh: Mesh) -> Mesh:
    """Quadratic (10-node) version of a P1 mesh: one node at the midpoint of
    every edge (straight-sided), appended after the vertices, which keep their
    ids; conn[:, 4:] are the midpoints of edges (0,1), (1,2), (0,2), (0,3),
    (1,3), (2,3).  Node sets are extended to a midpoint when both ends of its
    edge belong to the set; faces keep their three vertex ids."""
    c1 = np.asarray(mesh.conn)[:, :4].astype(np.int64)
    ne = c1.shape[0]
    ends = np.stack([np.sort(np.stack([c1[:, a], c1[:, b]], 1), axis=1) for a, b in P2_EDGES], 1)
    flat = ends.reshape(-1, 2)
    uniq, inv = np.unique(flat, axis=0, return_inverse=True)
    n1 = mesh.n_nodes
    X = np.vstack([mesh.X, 0.5 * (mesh.X[uniq[:, 0]] + mesh.X[uniq[:, 1]])])
    conn = np.empty((ne, 10), dtype=np.int64)
    conn[:, :4] = c1
    conn[:, 4:] = n1 + inv.reshape(ne, 6)
    sets = {k: np.concatenate([v, v[uniq[:, 0]] & v[uniq[:, 1]]]) for k, v in mesh.sets.items()}
    return Mesh(X=X, conn=conn.astype(np.int32), sets=sets, faces=dict(mesh.faces),
                elem_fibre=mesh.elem_fibre, elem_sheet=mesh.elem_sheet, grid=mesh.grid,
                name=mesh.name + "_p2")


def cook_p2_mesh(nx: int, ny: int, nz: int) -> Mesh:
    """Cook's membrane with quadratic tetrahedra (the P1 mesh's edges halved)."""
    return p2_from_p1(cook_mesh(nx, ny, nz))
