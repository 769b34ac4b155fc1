"""CDG switch functions on interior facets.

Representation: ``host[f]`` = the element K on facet f = (K, K') with
S_K^{K'} = -1.  That element carries the facet's boundary gradient q^f, and
the single-valued trace u-hat on f is taken from the other side (Sec. 2.2).

* Natural switch (Sec. 2.2): given an enumeration N of the elements,
  S_K^{K'} > 0 iff N(K) > N(K'); the host is the side with the smaller N.
* Consistent switch (Sec. 4.2): |sum_i S_K^{K_i}| < #neighbours, i.e. every
  element with at least two interior neighbours hosts at least one of its
  facets and leaves at least one unhosted.  The paper gives no construction;
  this oracle orients the dual graph along Euler circuits (a balanced
  orientation), which gives |#hosted - #unhosted| <= 1 at every element.
"""
import numpy as np

from .agglomerate import splitmix64


def natural_switch(interior, n_elem, seed=None):
    """Host = element with the smaller enumeration number; the enumeration
    is the element id, or the splitmix64 rank of the id when seed is given."""
    if seed is None:
        num = np.arange(n_elem, dtype=np.uint64)
    else:
        num = np.array([splitmix64(seed ^ e) for e in range(n_elem)], dtype=np.uint64)
    host = np.empty(len(interior), dtype=np.int64)
    for f, (a, _, b, _) in enumerate(interior):
        host[f] = a if (num[a], a) < (num[b], b) else b
    return host


def consistent_switch(interior, n_elem):
    """Balanced orientation by Hierholzer's walk.

    Graph: elements 0..N-1, one edge per interior facet (edge id = facet id),
    plus a virtual vertex N joined by one extra edge to every odd-degree
    element (edge ids follow the facets, in increasing element order).  Walks
    start at the lowest element with unused edges and always leave a vertex
    by its lowest-id unused edge; traversing K -> K' makes K' the host of the
    facet.
    """
    nf = len(interior)
    ends = [(a, b) for (a, _, b, _) in interior]
    deg = np.zeros(n_elem, dtype=np.int64)
    for a, b in ends:
        deg[a] += 1
        deg[b] += 1
    V = n_elem
    for e in range(n_elem):
        if deg[e] % 2 == 1:
            ends.append((e, V))
    adj = [[] for _ in range(n_elem + 1)]
    for eid, (a, b) in enumerate(ends):
        adj[a].append(eid)
        adj[b].append(eid)
    for lst in adj:
        lst.sort()
    used = np.zeros(len(ends), dtype=bool)
    ptr = [0] * (n_elem + 1)
    host = -np.ones(nf, dtype=np.int64)
    for start in range(n_elem):
        stack = [start]
        while stack:
            v = stack[-1]
            lst = adj[v]
            while ptr[v] < len(lst) and used[lst[ptr[v]]]:
                ptr[v] += 1
            if ptr[v] == len(lst):
                stack.pop()
                continue
            eid = lst[ptr[v]]
            used[eid] = True
            a, b = ends[eid]
            w = b if a == v else a
            if eid < nf:
                host[eid] = w
            stack.append(w)
    return host


def is_consistent(interior, n_elem, host):
    """Per element: (#interior neighbours, #hosted); consistency flag per
    element with at least two neighbours."""
    deg = np.zeros(n_elem, dtype=np.int64)
    hosted = np.zeros(n_elem, dtype=np.int64)
    for f, (a, _, b, _) in enumerate(interior):
        deg[a] += 1
        deg[b] += 1
        hosted[host[f]] += 1
    ok = (deg < 2) | ((hosted >= 1) & (hosted <= deg - 1))
    return deg, hosted, ok
