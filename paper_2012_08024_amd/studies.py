"""Setup-only studies on the solver.

* Coarsening (Sec. 3.5 vs Sec. 4.1): primal A_{l+1} = L^T A_l L against the
  flux form A_{l+1} = C_{l+1} + G_{l+1}^T M_{l+1}^{-1} G_{l+1}, with the
  Dirichlet penalty gamma of C_D = kappa gamma / h_avg (Sec. 2.2, Sec. 5.1)
  swept, on meshes refined by factors of two.  The paper's claim is
  qualitative: primal coarsening degrades as h -> 0, flux coarsening does not.
* Switch (Sec. 2.2, Sec. 4.2): the consistent switch against the natural one
  (host = element with the smaller number in a seeded enumeration).  An
  element that hosts two interior facets couples the two neighbours across
  them in C (second neighbours); the count of such pairs and the iteration
  counts are compared.

Both run through the C ABI on the current GPU; the hierarchy is agglomerated
until one element remains (Sec. 5) and the V-cycle runs in FP64, so that
only the coarse operators differ between cases.
"""
import time

import numpy as np

from . import (COARSEN_FLUX, COARSEN_PRIMAL, MG_FP64, SWITCH_CONSISTENT, SWITCH_NATURAL, CdgmgError, Solver,
               agglomerate, n_basis, switch)


def face_neighbours(e2v):
    """nbr[e, i] = the element across facet i of e (the facet opposite local
    vertex i), -1 on the boundary."""
    e2v = np.asarray(e2v)
    n, nf = e2v.shape
    nbr = -np.ones((n, nf), dtype=np.int64)
    seen = {}
    for e in range(n):
        for i in range(nf):
            key = tuple(sorted(int(v) for k, v in enumerate(e2v[e]) if k != i))
            if key in seen:
                c, j = seen.pop(key)
                nbr[e, i], nbr[c, j] = c, e
            else:
                seen[key] = (e, i)
    return nbr


def second_neighbour_pairs(e2v, hosted):
    """Distinct unordered element pairs (a, b), not face neighbours, coupled
    in C because some element hosts an interior facet towards each."""
    nbr = face_neighbours(e2v)
    pairs = set()
    for j in range(nbr.shape[0]):
        hs = [int(nbr[j, i]) for i in range(nbr.shape[1]) if hosted[j, i] and nbr[j, i] >= 0]
        for a in range(len(hs)):
            for b in range(a + 1, len(hs)):
                x, y = sorted((hs[a], hs[b]))
                if y not in nbr[x]:
                    pairs.add((x, y))
    return len(pairs)


def _solve_case(mesh, p, parents, sizes, f_of_nodes, max_iter, **opts):
    import torch
    kappa = torch.ones(mesh.n_elem, dtype=torch.float64, device="cuda")
    row = {}
    try:
        s = Solver(mesh, p, kappa, parents, sizes, mg_precision=MG_FP64, tol=1e-10, max_iter=max_iter, **opts)
    except CdgmgError as e:
        row.update(status="setup failed (%d)" % e.code)
        return row
    try:
        ne, nnzb = s.level_info()
        row["operator_complexity"] = float(np.sum(nnzb) / nnzb[0])
        f = torch.tensor(f_of_nodes(s.node_coords().reshape(-1, mesh.dim)), device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = s.solve(f)
        torch.cuda.synchronize()
        row.update(iterations=info.iterations, rel_residual=info.rel_residual,
                   solve_ms=(time.perf_counter() - t0) * 1e3,
                   status="converged" if info.rel_residual <= 1e-10 else "not converged")
    except CdgmgError as e:
        row.update(status="breakdown (%d)" % e.code)
    finally:
        s.close()
    return row


def study_coarsening(ns=(8, 16, 32, 64, 128), ps=(1, 2), gammas=(1e1, 1e2, 1e3, 1e4), seed=1, max_iter=300,
                     log=print):
    """Primal vs flux coarsening on 2D jittered Delaunay meshes refined by 2."""
    from workloads import mesh2d_jittered_delaunay, source_sine
    rows = []
    for p in ps:
        for n in ns:
            mesh = mesh2d_jittered_delaunay(n, seed)
            parents, sizes = agglomerate(mesh, 64, seed, p=p)
            for gamma in gammas:
                for name, c in (("primal", COARSEN_PRIMAL), ("flux", COARSEN_FLUX)):
                    row = dict(p=p, n=n, elements=int(mesh.n_elem), levels=len(sizes), gamma=gamma,
                               coarsening=name)
                    row.update(_solve_case(mesh, p, parents, sizes, source_sine, max_iter, gamma=gamma,
                                           coarsening=c))
                    log("coarsening p=%d n=%d gamma=%.0e %s: %s" % (p, n, gamma, name, row))
                    rows.append(row)
    return rows


def study_switch(cases=((2, 16, 2), (2, 32, 2), (2, 64, 2), (2, 128, 2), (3, 4, 1), (3, 8, 1), (3, 12, 1)),
                 seed=1, natural_seed=0, max_iter=300, log=print):
    """Consistent vs natural switch: second-neighbour pairs of C and
    iterations with primal and flux coarsening."""
    from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine
    rows = []
    for d, n, p in cases:
        mesh = mesh2d_jittered_delaunay(n, seed) if d == 2 else mesh3d_kuhn(n, seed)
        parents, sizes = agglomerate(mesh, 64, seed, p=p)
        for sname, mode in (("consistent", SWITCH_CONSISTENT), ("natural", SWITCH_NATURAL)):
            hosted = switch(mesh, mode=mode, seed=natural_seed)
            pairs = second_neighbour_pairs(mesh.e2v, hosted)
            for cname, c in (("primal", COARSEN_PRIMAL), ("flux", COARSEN_FLUX)):
                row = dict(d=d, n=n, p=p, n_p=n_basis(d, p), elements=int(mesh.n_elem), levels=len(sizes),
                           switch=sname, second_neighbour_pairs=pairs, coarsening=cname)
                row.update(_solve_case(mesh, p, parents, sizes, source_sine, max_iter, coarsening=c,
                                       switch_mode=mode, switch_seed=natural_seed))
                log("switch d=%d n=%d %s %s: %s" % (d, n, sname, cname, row))
                rows.append(row)
    return rows
