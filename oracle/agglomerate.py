"""Greedy element agglomeration (Sec. 3.1 Alg. 1, Sec. 3.2 Alg. 2).

Readings where the paper leaves the algorithm open (all deterministic, so the
element->aggregate maps are a function of (mesh, seed)):

* "Neighbours" of an element are its face neighbours: elements sharing at
  least one (d-1)-facet of the input mesh.  The vertices of an aggregate are
  the union of the vertices of its input-mesh elements.
* N(e) is the number of face neighbours of e still in the queue P; the
  queue pops the smallest key (N(e), rank(e), e), where
  rank(e) = splitmix64(seed ^ (level << 32) ^ e).
* Vertex-patch branch (N >= 2): v_max is the vertex of e touching the most
  elements still in P; ties go to the smallest (vrank(v), v) with
  vrank(v) = splitmix64(seed ^ (level << 32) ^ (1 << 62) ^ v).  The new block
  is e plus every element in P touching v_max (members listed by id).
* Small branch (N < 2): e joins the adjacent existing block with the fewest
  members counted at the current level (ties: smallest block id).  If no
  adjacent block exists yet, the vertex-patch branch is taken instead.
* Removing elements from P decrements N of each remaining face neighbour once
  per removed neighbour, so N(e) always equals the number of face
  neighbours still in P.
* Block ids are given in creation order; Alg. 1 is repeated on the
  aggregated mesh until the requested number of levels, a single element,
  or a coarse size bound is reached.

Pins: partition validity, the structured quad-grid case of the Fig. 2
caption and the regular hierarchy of Fig. 5, and the O(n log n) cost claim.
Beyond those, the maps themselves are parity unpinned: the paper prints none.
"""
import heapq

import numpy as np

MASK64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood 2014) of the state x."""
    z = (int(x) + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def greedy_agglomerate(elem_verts, pairs, n_elem, seed, level):
    """One application of Alg. 2.  Returns parent[e] (block id per element).

    elem_verts: list of iterables of vertex ids, one per element.
    pairs: iterable of face-neighbour pairs (a, b).
    """
    nbrs = [set() for _ in range(n_elem)]
    for a, b in pairs:
        a, b = int(a), int(b)
        if a != b:
            nbrs[a].add(b)
            nbrs[b].add(a)
    vert_elems = {}
    for e in range(n_elem):
        for v in elem_verts[e]:
            vert_elems.setdefault(int(v), []).append(e)
    base = (int(seed) ^ (int(level) << 32)) & MASK64
    rank = [splitmix64(base ^ e) for e in range(n_elem)]

    def vrank(v):
        return splitmix64(base ^ (1 << 62) ^ v)

    in_p = np.ones(n_elem, dtype=bool)
    N = [len(nbrs[e]) for e in range(n_elem)]
    heap = [(N[e], rank[e], e) for e in range(n_elem)]
    heapq.heapify(heap)
    parent = -np.ones(n_elem, dtype=np.int64)
    size = []

    def remove(members):
        for e in members:
            in_p[e] = False
        for e in members:
            for k in nbrs[e]:
                if in_p[k]:
                    N[k] -= 1
                    heapq.heappush(heap, (N[k], rank[k], k))

    while heap:
        key, _, e = heapq.heappop(heap)
        if not in_p[e] or key != N[e]:
            continue  # stale queue entry
        adjacent = sorted({int(parent[k]) for k in nbrs[e] if parent[k] >= 0})
        if N[e] >= 2 or not adjacent:
            in_p[e] = False
            best = None
            for v in sorted(set(int(x) for x in elem_verts[e])):
                cnt = sum(1 for k in vert_elems[v] if in_p[k])
                cand = (-cnt, vrank(v), v)
                if best is None or cand < best:
                    best = cand
            vmax = best[2]
            members = sorted({e} | {k for k in vert_elems[vmax] if in_p[k]})
            in_p[e] = True
            bid = len(size)
            size.append(len(members))
            for k in members:
                parent[k] = bid
            remove(members)
        else:
            bid = min(adjacent, key=lambda b: (size[b], b))
            parent[e] = bid
            size[bid] += 1
            remove([e])
    return parent


def coarsen_topology(elem_verts, pairs, parent):
    """Vertices (union) and face-neighbour pairs of the aggregated mesh."""
    nb = int(parent.max()) + 1
    verts = [set() for _ in range(nb)]
    for e, vs in enumerate(elem_verts):
        verts[parent[e]].update(int(v) for v in vs)
    new_pairs = set()
    for a, b in pairs:
        pa, pb = int(parent[a]), int(parent[b])
        if pa != pb:
            new_pairs.add((min(pa, pb), max(pa, pb)))
    return [sorted(v) for v in verts], sorted(new_pairs)


def build_hierarchy(e2v, pairs, n_levels, seed, coarse_dofs=None, n_p=None):
    """Alg. 1: repeat Alg. 2 until `n_levels` levels exist (level 0 = input
    mesh), a level has one element, or (if coarse_dofs is given) the level's
    n_elem * n_p <= coarse_dofs.  Returns the list of parent maps, one per
    coarsening step."""
    elem_verts = [sorted(int(v) for v in row) for row in np.asarray(e2v)]
    pairs = [tuple(int(x) for x in pr) for pr in np.asarray(pairs)]
    n = len(elem_verts)
    parents = []
    level = 0
    while True:
        if n <= 1:
            break
        if n_levels is not None and level + 1 >= n_levels:
            break
        if coarse_dofs is not None and n * n_p <= coarse_dofs:
            break
        parent = greedy_agglomerate(elem_verts, pairs, n, seed, level)
        parents.append(parent)
        elem_verts, pairs = coarsen_topology(elem_verts, pairs, parent)
        n = len(elem_verts)
        level += 1
    return parents


def vertex_connected(elem_verts, members):
    """True if the members form one component under vertex sharing."""
    members = list(members)
    if len(members) <= 1:
        return True
    seen = {members[0]}
    stack = [members[0]]
    mset = set(members)
    while stack:
        e = stack.pop()
        ve = set(elem_verts[e])
        for k in mset - seen:
            if ve & set(elem_verts[k]):
                seen.add(k)
                stack.append(k)
    return len(seen) == len(mset)
