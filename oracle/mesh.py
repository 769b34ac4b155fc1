"""Facet table of a conforming simplex mesh.

Local facet i of an element is the one opposite its local vertex i.  Facets
are identified by their sorted vertex tuple; two elements sharing a tuple are
face neighbours.  Interior facets are numbered in increasing order of
(lower element id, higher element id).
"""
import numpy as np


class Topology:
    def __init__(self, e2v, coords):
        e2v = np.asarray(e2v)
        coords = np.asarray(coords, dtype=np.float64)
        self.n_elem, nf = e2v.shape
        self.dim = nf - 1
        d = self.dim
        # positive volumes (affine simplices)
        v0 = coords[e2v[:, 0]]
        J = np.stack([coords[e2v[:, k + 1]] - v0 for k in range(d)], axis=2)
        det = np.linalg.det(J)
        if np.any(det <= 0):
            raise ValueError("mesh: non-positive element volume")
        table = {}
        for e in range(self.n_elem):
            for i in range(nf):
                key = tuple(sorted(int(e2v[e, k]) for k in range(nf) if k != i))
                table.setdefault(key, []).append((e, i))
        nbr = -np.ones((self.n_elem, nf), dtype=np.int64)
        interior = []
        boundary = []
        for key, sides in table.items():
            if len(sides) > 2:
                raise ValueError("mesh: non-manifold facet")
            if len(sides) == 1:
                boundary.append(sides[0])
            else:
                (ea, ia), (eb, ib) = sorted(sides)
                nbr[ea, ia] = eb
                nbr[eb, ib] = ea
                interior.append((ea, ia, eb, ib))
        interior.sort(key=lambda t: (t[0], t[2]))
        self.interior = interior          # list of (e_lo, i_lo, e_hi, i_hi)
        self.boundary = sorted(boundary)  # list of (e, i)
        self.nbr = nbr                    # [n_elem, d+1], -1 on the boundary
        self.face_id = -np.ones((self.n_elem, nf), dtype=np.int64)
        for fid, (ea, ia, eb, ib) in enumerate(interior):
            self.face_id[ea, ia] = fid
            self.face_id[eb, ib] = fid

    def neighbor_pairs(self):
        return np.array([(a, b) for (a, _, b, _) in self.interior], dtype=np.int64).reshape(-1, 2)
