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
* Convection-diffusion (Sec. 5): beta v . grad u with v = (1, 0), f = 1 and
  zero Dirichlet data, GMRES iterations under refinement for a range of beta.
* Size (not a claim of the paper): the benchmark's solve (2D p = 3, V(2,2)
  FP32 in FP64 FCG(1), tol 1e-10) on meshes from 2e4 to 1.6e6 triangles,
  agglomerated until n_l n_p <= 2000: throughput and the level-0 sweep's
  rate as the V-cycle operator grows past the last-level cache.

All run through the C ABI on the current GPU with the V-cycle in FP64, so
that only the operators differ between cases; the hierarchy is agglomerated
until one element remains (Sec. 5).  Two solver settings:
  "paper":    p = 1, V(0, 3) block Jacobi with damping 2/3, right-preconditioned
              GMRES(50), tolerance 1e-8 (the settings of Sec. 5);
  "workload": V(2, 2) with damping 0.7, FCG(1), tolerance 1e-10.
"""
import time

import numpy as np

from . import (COARSEN_FLUX, COARSEN_PRIMAL, MG_FP64, OUTER_FCG, OUTER_GMRES, SWITCH_CONSISTENT, SWITCH_NATURAL,
               CdgmgError, Solver, agglomerate, n_basis, switch)
from .bytemodel import facet_nodes, row_block, smoother_bytes

SETTINGS = {
    "paper": dict(nu1=0, nu2=3, omega=2.0 / 3.0, outer=OUTER_GMRES, restart=50, tol=1e-8),
    "workload": dict(nu1=2, nu2=2, omega=0.7, outer=OUTER_FCG, tol=1e-10),
}


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


def _solve_case(mesh, p, parents, sizes, f_of_nodes, max_iter, setting, **opts):
    import torch
    kappa = torch.ones(mesh.n_elem, dtype=torch.float64, device="cuda")
    cfg = dict(SETTINGS[setting])
    cfg.update(opts)
    tol = cfg["tol"]
    row = {}
    try:
        s = Solver(mesh, p, kappa, parents, sizes, mg_precision=MG_FP64, max_iter=max_iter, **cfg)
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
                   status="converged" if info.rel_residual <= tol else "not converged")
    except CdgmgError as e:
        row.update(status="breakdown (%d)" % e.code)
    finally:
        s.close()
    return row


def study_coarsening(setting="workload", ns=(8, 16, 32, 64, 128), ps=None, gammas=(1e1, 1e2, 1e3, 1e4), seed=1,
                     max_iter=300, log=print):
    """Primal vs flux coarsening under refinement.  "workload": 2D jittered
    Delaunay meshes, all boundaries Dirichlet, p = 1, 2.  "paper": the square
    of Sec. 5.1 (uniform grid, here split into right triangles) with Neumann
    sides x = 0, 1 and Dirichlet y = 0, 1, p = 1."""
    from workloads import mesh2d_jittered_delaunay, mesh2d_square_neumann_sides, source_sine
    if ps is None:
        ps = (1,) if setting == "paper" else (1, 2)
    rows = []
    for p in ps:
        for n in ns:
            mesh = mesh2d_square_neumann_sides(n) if setting == "paper" else mesh2d_jittered_delaunay(n, seed)
            parents, sizes = agglomerate(mesh, 64, seed, p=p)
            for gamma in gammas:
                for name, c in (("primal", COARSEN_PRIMAL), ("flux", COARSEN_FLUX)):
                    row = dict(setting=setting, p=p, n=n, elements=int(mesh.n_elem), levels=len(sizes), gamma=gamma,
                               coarsening=name)
                    row.update(_solve_case(mesh, p, parents, sizes, source_sine, max_iter, setting, gamma=gamma,
                                           coarsening=c))
                    log("coarsening %s p=%d n=%d gamma=%.0e %s: %s" % (setting, p, n, gamma, name, row))
                    rows.append(row)
    return rows


def study_switch(setting="workload", cases=None, seed=1, natural_seed=0, max_iter=300, log=print):
    """Consistent vs natural switch: second-neighbour pairs of C and
    iterations with primal and flux coarsening."""
    from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine
    if cases is None:
        p2 = 1 if setting == "paper" else 2
        cases = ((2, 16, p2), (2, 32, p2), (2, 64, p2), (2, 128, p2), (3, 4, 1), (3, 8, 1), (3, 12, 1))
    rows = []
    for d, n, p in cases:
        mesh = mesh2d_jittered_delaunay(n, seed) if d == 2 else mesh3d_kuhn(n, seed)
        parents, sizes = agglomerate(mesh, 64, seed, p=p)
        for sname, mode in (("consistent", SWITCH_CONSISTENT), ("natural", SWITCH_NATURAL)):
            hosted = switch(mesh, mode=mode, seed=natural_seed)
            pairs = second_neighbour_pairs(mesh.e2v, hosted)
            for cname, c in (("primal", COARSEN_PRIMAL), ("flux", COARSEN_FLUX)):
                row = dict(setting=setting, d=d, n=n, p=p, n_p=n_basis(d, p), elements=int(mesh.n_elem),
                           levels=len(sizes), switch=sname, second_neighbour_pairs=pairs, coarsening=cname)
                row.update(_solve_case(mesh, p, parents, sizes, source_sine, max_iter, setting, coarsening=c,
                                       switch_mode=mode, switch_seed=natural_seed))
                log("switch %s d=%d n=%d %s %s: %s" % (setting, d, n, sname, cname, row))
                rows.append(row)
    return rows


def study_size(ns=(100, 158, 224, 316, 448, 632, 894), p=3, seed=2, agg_seed=12, steps=3, log=print):
    """DOFs/s, iterations and the level-0 sweep's algorithmic bytes per
    second against the mesh size (2D jittered Delaunay, kappa = 1, sine
    source, FP32 V-cycle in FP64 FCG(1) to 1e-10)."""
    import torch
    from workloads import mesh2d_jittered_delaunay, source_sine
    from . import MG_FP32
    rows = []
    for n in ns:
        mesh = mesh2d_jittered_delaunay(n, seed)
        parents, sizes = agglomerate(mesh, 50, agg_seed, p=p, coarse_dofs=2000)
        log("size n=%d: mesh and hierarchy %s" % (n, list(sizes)))
        s = Solver(mesh, p, torch.ones(mesh.n_elem, dtype=torch.float64, device="cuda"), parents, sizes,
                   mg_precision=MG_FP32, **SETTINGS["workload"])
        try:
            ne, nnzb = s.level_info()
            f = torch.tensor(source_sine(s.node_coords().reshape(-1, 2)), device="cuda")
            s.solve(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, info = s.solve(f)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3 / steps
            s.set_profile(True)
            _, pinfo = s.solve(f)
            s.set_profile(False)
            npb = n_basis(2, p)
            off = int(nnzb[0]) - mesh.n_elem
            sweep_bytes = smoother_bytes(int(nnzb[0]), mesh.n_elem, npb, 4, facet_nodes(2, npb), 3)
            sweep_us = 1e3 * pinfo.kernel_ms["smooth0"] / max(pinfo.kernel_launches["smooth0"], 1)
            row = dict(n=n, elements=int(mesh.n_elem), dofs=int(mesh.n_elem * npb), levels=len(sizes),
                       iterations=info.iterations, rel_residual=info.rel_residual, solve_ms=ms,
                       dofs_per_s=mesh.n_elem * npb / (ms * 1e-3), sweep_mb=sweep_bytes / 1e6,
                       vcycle_operator_mb=(off * npb * facet_nodes(2, npb) + mesh.n_elem * row_block(npb)) * 4 / 1e6,
                       sweep_us=sweep_us, sweep_gbs=sweep_bytes / (sweep_us * 1e-6) / 1e9,
                       device_gb=s.device_bytes() / 1e9)
        finally:
            s.close()
        log("size n=%d: %s" % (n, row))
        rows.append(row)
    return rows


def study_convection(ns=(8, 16, 32, 64, 128), betas=(0.0, 0.1, 1.0, 10.0, 100.0), p=1, seed=1, max_iter=500,
                     log=print):
    """GMRES iterations for beta v . grad u - laplace u = 1 (v = (1, 0), zero
    Dirichlet data) under refinement, the paper's settings (2D jittered
    Delaunay meshes stand in for the airfoil mesh)."""
    from workloads import mesh2d_jittered_delaunay

    def ones(x):
        return np.ones(x.shape[0])

    rows = []
    for n in ns:
        mesh = mesh2d_jittered_delaunay(n, seed)
        parents, sizes = agglomerate(mesh, 64, seed, p=p)
        for beta in betas:
            row = dict(setting="paper", p=p, n=n, elements=int(mesh.n_elem), levels=len(sizes), beta=beta)
            row.update(_solve_case(mesh, p, parents, sizes, ones, max_iter, "paper", beta=beta, velocity=(1.0, 0.0),
                                   coarsening=COARSEN_PRIMAL))
            log("convection n=%d beta=%g: %s" % (n, beta, row))
            rows.append(row)
    return rows
