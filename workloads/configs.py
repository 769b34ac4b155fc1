"""The five synthetic workloads: mesh family and size, polynomial degree,
coefficient field, hierarchy depth, cycle and outer solver, and seeds."""
from .meshes import mesh2d_jittered_delaunay, mesh2d_square_neumann_sides, mesh3d_kuhn
from .fields import kappa_grf, kappa_spheres

CONFIGS = {
    # 2D jittered Delaunay, 512 triangles, p=2, kappa=1, 3 levels, PCG, FP64 throughout
    "c1": dict(dim=2, n=16, p=2, kappa="one", levels=3, outer="pcg", mg="fp64",
               mesh_seed=1, agg_seed=11, tol=1e-10),
    # 2D jittered Delaunay, 199712 triangles, p=3 (1 997 120 DOFs), kappa=1, 6 levels
    "c2": dict(dim=2, n=316, p=3, kappa="one", levels=6, outer="fcg", mg="fp32",
               mesh_seed=2, agg_seed=12, tol=1e-10),
    # 3D Kuhn tetrahedra, 105456 tets, p=2 (1 054 560 DOFs), kappa=1, 5 levels
    "c3": dict(dim=3, n=26, p=2, kappa="one", levels=5, outer="fcg", mg="fp32",
               mesh_seed=3, agg_seed=13, tol=1e-10),
    # 2D jittered Delaunay, 49928 triangles, p=3, log-normal kappa, adjoint gradient
    "c4": dict(dim=2, n=158, p=3, kappa="grf", kappa_seed=41, levels=None,
               coarse_dofs=2000, outer="fcg", mg="fp32", mesh_seed=4, agg_seed=14,
               fd_seed=42, fd_count=20, fd_step=1e-6, tol=1e-10),
    # 3D Kuhn tetrahedra, 384000 tets, p=3 (7 680 000 DOFs), high-contrast spheres
    "c5": dict(dim=3, n=40, p=3, kappa="spheres", kappa_seed=51, levels=6, outer="fcg",
               mg="fp32", mesh_seed=5, agg_seed=15, tol=1e-10),
    # the mesh class of Sec. 5.1 at the size of c2: uniform n x n square split
    # into 199712 right triangles, Neumann sides x = 0, 1, Dirichlet y = 0, 1;
    # p=3 (1 997 120 DOFs), kappa=1, 6 levels -- flux against primal coarsening
    "sq316": dict(dim=2, n=316, p=3, kappa="one", levels=6, outer="fcg", mg="fp32", mesh="square51",
                  mesh_seed=0, agg_seed=12, tol=1e-10),
}


def config_mesh(cfg, n=None):
    """Mesh and per-element kappa of a workload (optionally at another n)."""
    import numpy as np

    n = cfg["n"] if n is None else n
    if cfg.get("mesh") == "square51":
        mesh = mesh2d_square_neumann_sides(n)
    elif cfg["dim"] == 2:
        mesh = mesh2d_jittered_delaunay(n, cfg["mesh_seed"])
    else:
        mesh = mesh3d_kuhn(n, cfg["mesh_seed"])
    if cfg["kappa"] == "one":
        kappa = np.ones(mesh.n_elem)
    elif cfg["kappa"] == "grf":
        kappa = kappa_grf(mesh, cfg["kappa_seed"])
    else:
        kappa = kappa_spheres(mesh, cfg["kappa_seed"])
    return mesh, kappa
