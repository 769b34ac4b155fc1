"""Seeded unstructured simplex meshes of the unit square and unit cube.

Conventions shared by every consumer (they are part of the library's C-ABI):

* ``coords``  float64 [n_vert, d]
* ``e2v``     int32   [n_elem, d+1], positively oriented (det of the edge
  matrix > 0); local face ``i`` of an element is the facet opposite its local
  vertex ``i``.
* ``face_bc`` int8    [n_elem, d+1]; 0 = Dirichlet, 1 = Neumann; the value is
  only read on boundary facets.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    coords: np.ndarray
    e2v: np.ndarray
    face_bc: np.ndarray

    @property
    def dim(self):
        return self.coords.shape[1]

    @property
    def n_elem(self):
        return self.e2v.shape[0]

    @property
    def n_vert(self):
        return self.coords.shape[0]


def _orient(coords, e2v):
    """Swap two vertices of every negatively oriented simplex."""
    d = coords.shape[1]
    v0 = coords[e2v[:, 0]]
    J = np.stack([coords[e2v[:, k + 1]] - v0 for k in range(d)], axis=2)
    det = np.linalg.det(J)
    neg = det < 0
    e2v = e2v.copy()
    e2v[neg, 0], e2v[neg, 1] = e2v[neg, 1].copy(), e2v[neg, 0].copy()
    return e2v


def mesh2d_jittered_delaunay(n, seed, jitter=0.25, bc=0):
    """(n+1)^2 grid points of [0,1]^2, interior points moved by U(+-jitter*h)^2,
    boundary points fixed, Delaunay-triangulated (2 n^2 triangles)."""
    import scipy.spatial

    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)
    inner = (P[:, 0] > 0) & (P[:, 0] < 1) & (P[:, 1] > 0) & (P[:, 1] < 1)
    P[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 2))
    tri = scipy.spatial.Delaunay(P)
    e2v = _orient(P, tri.simplices.astype(np.int32)).astype(np.int32)
    face_bc = np.full(e2v.shape, bc, dtype=np.int8)
    return Mesh(P, e2v, face_bc)


def mesh2d_square_neumann_sides(n):
    """Uniform n x n grid of [0,1]^2, every square split by its (0,0)-(1,1)
    diagonal (2 n^2 right triangles); Neumann facets (1) on x = 0 and x = 1,
    Dirichlet (0) on y = 0 and y = 1."""
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel()], axis=1)

    def vid(i, j):
        return i * (n + 1) + j

    tris = []
    for i in range(n):
        for j in range(n):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            tris += [(a, b, c), (a, c, d)]
    e2v = _orient(P, np.asarray(tris, dtype=np.int32)).astype(np.int32)
    face_bc = np.zeros(e2v.shape, dtype=np.int8)
    for e in range(e2v.shape[0]):
        for i in range(3):
            f = [int(v) for k, v in enumerate(e2v[e]) if k != i]
            xs = P[f, 0]
            if np.all(xs == 0.0) or np.all(xs == 1.0):
                face_bc[e, i] = 1
    return Mesh(P, e2v, face_bc)


def mesh3d_kuhn(n, seed, jitter=0.15, bc=0):
    """(n+1)^3 grid of [0,1]^3, interior vertices moved by U(+-jitter*h)^3,
    every cube split into the 6 Kuhn tetrahedra sharing its main diagonal."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    g = np.linspace(0.0, 1.0, n + 1)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    P = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    inner = np.all((P > 0) & (P < 1), axis=1)
    P[inner] += rng.uniform(-jitter * h, jitter * h, size=(int(inner.sum()), 3))

    def vid(i, j, k):
        return (i * (n + 1) + j) * (n + 1) + k

    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    I, J, K = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    tets = []
    for perm in perms:
        cur = np.stack([I, J, K], axis=1)
        verts = [vid(cur[:, 0], cur[:, 1], cur[:, 2])]
        for ax in perm:
            cur = cur.copy()
            cur[:, ax] += 1
            verts.append(vid(cur[:, 0], cur[:, 1], cur[:, 2]))
        tets.append(np.stack(verts, axis=1))
    # cube-major order: all six tets of a cube are consecutive
    e2v = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    e2v = _orient(P, e2v).astype(np.int32)
    face_bc = np.full(e2v.shape, bc, dtype=np.int8)
    return Mesh(P, e2v, face_bc)


def quad_grid(n):
    """Element->vertex incidence of a structured n x n quadrilateral grid
    (counter-clockwise vertex order) and its edge-neighbour pairs.  Used only
    to exercise the agglomeration on the structured case."""
    def vid(i, j):
        return j * (n + 1) + i

    elems = []
    for j in range(n):
        for i in range(n):
            elems.append([vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)])
    pairs = []
    for j in range(n):
        for i in range(n):
            e = j * n + i
            if i + 1 < n:
                pairs.append((e, e + 1))
            if j + 1 < n:
                pairs.append((e, e + n))
    return np.array(elems, dtype=np.int32), np.array(pairs, dtype=np.int32)
