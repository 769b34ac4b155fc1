"""Edge cases of the HIP path against the oracle (calls through the C ABI):
a zero right-hand side, a hierarchy of one level (the V-cycle is the dense
coarsest solve), meshes of fewer rows than one 64-row slice, mixed
Dirichlet/Neumann boundaries (Sec. 5.1), and the n_p = 20 kernels on a
one-cube mesh."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse.linalg as spl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from oracle.cdg import CDG  # noqa: E402
from oracle.multigrid import Hierarchy  # noqa: E402
from workloads import mesh2d_jittered_delaunay, mesh2d_square_neumann_sides, mesh3d_kuhn, source_sine  # noqa: E402


def _neumann_x_sides(mesh):
    """Neumann (1) on the boundary facets lying in x = 0 or x = 1."""
    fb = np.zeros_like(mesh.face_bc)
    X = mesh.coords[:, 0]
    nf = mesh.e2v.shape[1]
    for e in range(mesh.n_elem):
        for i in range(nf):
            xs = X[[mesh.e2v[e, k] for k in range(nf) if k != i]]
            if np.all(xs < 1e-12) or np.all(xs > 1 - 1e-12):
                fb[e, i] = 1
    return dataclasses.replace(mesh, face_bc=fb)


def _check_vcycle_and_levels(mesh, p, levels, seed, **opts):
    parents, sizes = cm.agglomerate(mesh, levels, seed, p=p)
    kappa = np.random.default_rng(seed).uniform(0.5, 2.0, mesh.n_elem)
    print("case edge", mesh.dim, mesh.n_elem, p, list(sizes), opts, flush=True)
    solver = cm.Solver(mesh, p, kappa, parents, sizes, mg_precision=cm.MG_FP64, **opts)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, p)
    H = Hierarchy(cdg, parents, kappa=kappa, coarsening="primal")
    for l in range(len(sizes)):
        A = cm.bsr_to_scipy(*solver.export_operator(l))
        assert abs(A - H.A[l]).max() <= 1e-12 * abs(H.A[l]).max(), l
    r = np.random.default_rng(1).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, 2, 2, 0.7)
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)
    return solver, cdg, H, sizes


@pytest.mark.parametrize("outer", [cm.OUTER_FCG, cm.OUTER_PCG, cm.OUTER_GMRES])
def test_zero_rhs_gives_zero_solution(outer):
    mesh = mesh2d_jittered_delaunay(9, 1)
    parents, sizes = cm.agglomerate(mesh, 3, 2, p=2)
    solver = cm.Solver(mesh, 2, np.ones(mesh.n_elem), parents, sizes, outer=outer)
    u, info = solver.solve(np.zeros(mesh.n_elem * 6))
    assert info.iterations == 0
    assert not np.any(u.cpu().numpy())
    solver.close()


@pytest.mark.parametrize("d,n,p", [(2, 6, 2), (3, 2, 2), (2, 3, 3)])
def test_single_level_hierarchy_is_a_direct_solve(d, n, p):
    # no agglomeration: the V-cycle is the dense coarsest inverse, so FCG
    # converges in one iteration
    mesh = mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)
    solver, cdg, H, sizes = _check_vcycle_and_levels(mesh, p, 1, 0)
    assert len(sizes) == 1
    f = source_sine(cdg.nodes_phys().reshape(-1, d))
    u, info = solver.solve(f)
    ref = spl.spsolve(H.A[0].tocsc(), cdg.M0() @ f)
    assert info.iterations <= 2
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    solver.close()


@pytest.mark.parametrize("d,n,p", [(2, 1, 3), (2, 2, 1), (3, 1, 1), (3, 1, 3)])
def test_meshes_below_one_slice(d, n, p):
    # 2 triangles, 8 triangles, 6 tetrahedra (one cube, n_p = 20 at p = 3):
    # one partial 64-row slice, agglomerated down to one element
    mesh = mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)
    solver, cdg, H, sizes = _check_vcycle_and_levels(mesh, p, 4, 3)
    assert sizes[-1] == 1
    f = source_sine(cdg.nodes_phys().reshape(-1, d))
    u, info = solver.solve(f)
    ref = spl.spsolve(H.A[0].tocsc(), cdg.M0() @ f)
    assert info.rel_residual <= 1e-10
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    solver.close()


@pytest.mark.parametrize("case", ["2d_square_p1", "2d_jittered_p3", "3d_p2"])
def test_mixed_dirichlet_neumann_boundaries(case):
    # Sec. 5.1: Neumann sides x = 0, 1 and Dirichlet y = 0, 1 (Neumann facets
    # are not hosted and carry no penalty)
    if case == "2d_square_p1":
        mesh, p = mesh2d_square_neumann_sides(12), 1
    elif case == "2d_jittered_p3":
        mesh, p = _neumann_x_sides(mesh2d_jittered_delaunay(10, 2)), 3
    else:
        mesh, p = _neumann_x_sides(mesh3d_kuhn(3, 2)), 2
    assert mesh.face_bc.any()
    solver, cdg, H, sizes = _check_vcycle_and_levels(mesh, p, 3, 5)
    f = source_sine(cdg.nodes_phys().reshape(-1, mesh.dim))
    u, info = solver.solve(f)
    ref = spl.spsolve(H.A[0].tocsc(), cdg.M0() @ f)
    assert info.rel_residual <= 1e-10
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    solver.close()


def test_coarsest_level_too_large_is_rejected():
    # the dense coarsest inverse is limited to 12000 unknowns: 3200 elements
    # at n_p = 10 with no agglomeration is refused with CDGMG_ERR_ARG
    mesh = mesh2d_jittered_delaunay(40, 1)
    parents, sizes = cm.agglomerate(mesh, 1, 0, p=3)
    with pytest.raises(cm.CdgmgError) as ei:
        cm.Solver(mesh, 3, np.ones(mesh.n_elem), parents, sizes)
    assert ei.value.code == -1
    parents, sizes = cm.agglomerate(mesh, 3, 0, p=3)
    cm.Solver(mesh, 3, np.ones(mesh.n_elem), parents, sizes).close()


@pytest.mark.parametrize("p,mg,cf", [(1, "fp64", 0), (3, "fp64", 0), (1, "fp32", 0), (3, "fp32", 1)])
def test_coarsest_aggregate_with_many_children(p, mg, cf):
    # one coarsest aggregate holding every level-1 aggregate (more than 64 of
    # them): the one-launch coarsest level (entry, dense solve, prolongation)
    # then prolongs into its children in more than one pass of its workgroup
    mesh = mesh2d_jittered_delaunay(24, 1)
    p1, s1 = cm.agglomerate(mesh, 2, 5, p=p)
    assert len(s1) == 2 and s1[1] > 64
    parents = [p1[0], np.zeros(s1[1], dtype=np.int32)]
    sizes = np.array([s1[0], s1[1], 1], dtype=np.int32)
    kappa = np.random.default_rng(4).uniform(0.5, 2.0, mesh.n_elem)
    print("case many-children", p, mg, cf, list(sizes), flush=True)
    prec = cm.MG_FP64 if mg == "fp64" else cm.MG_FP32
    solver = cm.Solver(mesh, p, kappa, parents, sizes, mg_precision=prec, coarse_fp64=cf)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, p)
    H = Hierarchy(cdg, parents, kappa=kappa, coarsening="primal")
    r = np.random.default_rng(2).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, 2, 2, 0.7)
    tol = 1e-11 if mg == "fp64" else 1e-4
    assert np.linalg.norm(z - ref) <= tol * np.linalg.norm(ref)
    solver.close()
