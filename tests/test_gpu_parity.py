"""GPU parity of the HIP path against the FP64 oracle (call through the C ABI)."""
import functools

import numpy as np
import pytest
import scipy.sparse.linalg as spl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from oracle.adjoint import grad_kappa as oracle_grad_kappa  # noqa: E402
from oracle.agglomerate import build_hierarchy  # noqa: E402
from oracle.cdg import CDG  # noqa: E402
from oracle.krylov import fcg, gmres, pcg  # noqa: E402
from oracle.multigrid import Hierarchy  # noqa: E402
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine  # noqa: E402

from kernel_coverage import (CASES, FP32_VARIANT_CASES, GROUP_CASES, GROUPS, NP, ROW_THREADS,  # noqa: E402
                             VARIANTS)


@functools.lru_cache(maxsize=None)
def _oracle_case(name, kappa_kind):
    d, n, p, levels, seed = CASES[name]
    mesh = mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)
    parents, sizes = cm.agglomerate(mesh, levels, seed, p=p)
    rng = np.random.default_rng(seed)
    kappa = rng.uniform(0.5, 2.0, mesh.n_elem) if kappa_kind == "random" else np.ones(mesh.n_elem)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, p)
    H = Hierarchy(cdg, parents, kappa=kappa, coarsening="primal")
    return mesh, cdg, H, kappa, parents, sizes


def _build(name, mg=cm.MG_FP64, kappa_kind="random", **opts):
    p = CASES[name][2]
    mesh, cdg, H, kappa, parents, sizes = _oracle_case(name, kappa_kind)
    print("case", name, "n_elem", mesh.n_elem, "sizes", list(sizes), "mg", mg, opts, flush=True)
    solver = cm.Solver(mesh, p, kappa, parents, sizes, mg_precision=mg, **opts)
    return mesh, solver, cdg, H, kappa, parents, sizes


@pytest.mark.parametrize("name", list(CASES))
def test_level_operators_match_oracle(name):
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name)
    for l in range(len(sizes)):
        A = cm.bsr_to_scipy(*solver.export_operator(l))
        R = H.A[l]
        err = abs(A - R).max() / abs(R).max()
        assert err <= 1e-12, (name, l, err)
    ne, nz = solver.level_info()
    assert list(ne) == list(sizes)
    solver.close()


@pytest.mark.parametrize("name", ["2d_p2", "3d_p2"])
def test_apply_A_fp64_and_fp32(name):
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, mg=cm.MG_FP32)
    rng = np.random.default_rng(1)
    for l in range(len(sizes)):
        x = rng.standard_normal(H.A[l].shape[0])
        ref = H.A[l] @ x
        y = solver.apply_A(l, x, 0).cpu().numpy()
        assert np.abs(y - ref).max() <= 1e-13 * np.abs(ref).max() * 10
        y32 = solver.apply_A(l, x.astype(np.float32), 1).cpu().numpy().astype(np.float64)
        assert np.linalg.norm(y32 - ref) <= 1e-5 * np.linalg.norm(ref)
    solver.close()




# kernel_variant = wavefronts per 64-row slice of the level-0 kernels (0 = auto)
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_fp64_matches_oracle(name, variant):
    if variant and NP[name] % variant:
        with pytest.raises(cm.CdgmgError) as ei:
            _build(name, kernel_variant=variant)
        assert ei.value.code == -1
        return
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, kernel_variant=variant)
    r = np.random.default_rng(2).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, 2, 2, 0.7)
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)
    solver.close()


@pytest.mark.parametrize("nu1,nu2,omega", [(0, 2, 0.7), (1, 1, 0.6), (3, 0, 0.5), (1, 3, 0.8)])
@pytest.mark.parametrize("name", ["2d_p2", "3d_p2"])
def test_vcycle_fp64_sweep_counts(name, nu1, nu2, omega):
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, nu1=nu1, nu2=nu2, omega=omega)
    r = np.random.default_rng(3).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, nu1, nu2, omega)
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)
    solver.close()


@pytest.mark.parametrize("name,variant", FP32_VARIANT_CASES)
def test_vcycle_fp32_close_to_oracle(name, variant):
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, mg=cm.MG_FP32, kernel_variant=variant)
    r = np.random.default_rng(2).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, 2, 2, 0.7)
    assert np.linalg.norm(z - ref) <= 1e-4 * np.linalg.norm(ref)
    solver.close()


@pytest.mark.parametrize("name", ["2d_p3", "3d_p3"])
def test_vcycle_fp32_with_fp64_coarsest(name):
    # the FP32 cycle with its coarsest solve in FP64 (coarse_fp64): the same
    # cycle as the oracle's up to the FP32 rounding of the other levels
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, mg=cm.MG_FP32, coarse_fp64=1)
    r = np.random.default_rng(2).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, 2, 2, 0.7)
    assert np.linalg.norm(z - ref) <= 1e-4 * np.linalg.norm(ref)
    solver.close()


def test_fp64_coarsest_one_level():
    # one level: the FP32 cycle is the FP64 inverse applied to the FP32-rounded
    # residual, so FCG converges to the direct solution
    mesh = mesh2d_jittered_delaunay(6, 3)
    parents, sizes = cm.agglomerate(mesh, 1, 1, p=2)
    solver = cm.Solver(mesh, 2, np.ones(mesh.n_elem), parents, sizes, mg_precision=cm.MG_FP32, coarse_fp64=1,
                       tol=1e-12)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, 2)
    f = source_sine(cdg.nodes_phys().reshape(-1, 2))
    u, info = solver.solve(f)
    ref = spl.spsolve(cdg.A().tocsc(), cdg.M0() @ f)
    assert info.rel_residual <= 1e-12
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    solver.close()


# Every kernel instantiation of the coarse levels: G lanes per row in the sweep
# and in the residual + restriction (the automatic choice takes 32 or 64 by
# the level's mean row length), and both workgroup sizes of the thread-per-row
# transfer kernels (the automatic choice takes 64).  The full-size tests check the benchmark workloads' launch
# configurations against kernel_coverage.COVERED.
@pytest.mark.parametrize("rt", ROW_THREADS)
@pytest.mark.parametrize("group", GROUPS)
@pytest.mark.parametrize("mg", [cm.MG_FP64, cm.MG_FP32])
@pytest.mark.parametrize("name", GROUP_CASES)
def test_vcycle_every_coarse_kernel(name, mg, group, rt):
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, mg=mg, coarse_group=group, row_threads=rt)
    li = solver.launch_info()
    L = len(sizes) - 1
    assert list(li["lanes_sweep"][1:L]) == [group] * (L - 1)
    assert list(li["lanes_restrict"][1:L]) == [group] * (L - 1)
    assert list(li["row_threads"][:L]) == [rt] * L
    r = np.random.default_rng(4).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, 2, 2, 0.7)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    print("case", name, "mg", mg, "G", group, "row threads", rt, "error", err, flush=True)
    assert err <= (1e-11 if mg == cm.MG_FP64 else 1e-4), err
    if mg == cm.MG_FP64:  # element by element as well
        assert np.abs(z - ref).max() <= 1e-11 * np.abs(ref).max()
    solver.close()


def test_coarse_options_out_of_range():
    for kw in ({"coarse_group": 12}, {"coarse_group": 128}, {"row_threads": 128}):
        with pytest.raises(cm.CdgmgError) as ei:
            _build("2d_p1", **kw)
        assert ei.value.code == -1


@pytest.mark.parametrize("name,mg", [("2d_p2", cm.MG_FP64), ("2d_p3", cm.MG_FP32), ("3d_p2", cm.MG_FP32),
                                     ("3d_p1", cm.MG_FP64), ("3d_p3", cm.MG_FP32), ("3d_p3", cm.MG_FP64)])
def test_solve_matches_direct_solve(name, mg):
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, mg=mg, tol=1e-12)
    x = solver.node_coords().reshape(-1, mesh.dim)
    assert np.allclose(x, cdg.nodes_phys().reshape(-1, mesh.dim), atol=1e-14)
    f = source_sine(x)
    u, info = solver.solve(f)
    ref = spl.spsolve(H.A[0].tocsc(), cdg.M0() @ f)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert info.rel_residual <= 1e-12
    assert err <= (1e-10 if mg == cm.MG_FP64 else 1e-9), err
    solver.close()


def test_pcg_fp64_iterations_match_oracle():
    # C1 shape: 2D p=2, 3 levels, PCG, all FP64; iteration counts within +-1
    mesh = mesh2d_jittered_delaunay(16, 1)
    parents, sizes = cm.agglomerate(mesh, 3, 11, p=2)
    kappa = np.ones(mesh.n_elem)
    solver = cm.Solver(mesh, 2, kappa, parents, sizes, mg_precision=cm.MG_FP64, outer=cm.OUTER_PCG, tol=1e-10)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, 2)
    H = Hierarchy(cdg, parents, coarsening="primal")
    f = source_sine(cdg.nodes_phys().reshape(-1, 2))
    b = cdg.M0() @ f
    xo, ito, reso = pcg(H.A[0], b, H.vcycle, tol=1e-10)
    u, info = solver.solve(f)
    assert abs(info.iterations - ito) <= 1
    assert np.linalg.norm(u.cpu().numpy() - xo) <= 1e-8 * np.linalg.norm(xo)
    solver.close()


def test_fcg_history_matches_oracle_fp64():
    mesh, solver, cdg, H, kappa, parents, sizes = _build("2d_p2", tol=1e-11)
    f = source_sine(cdg.nodes_phys().reshape(-1, 2))
    b = cdg.M0() @ f
    hist = []
    xo, ito, reso = fcg(H.A[0], b, H.vcycle, tol=1e-11, history=hist)
    u, info = solver.solve(f, history=True)
    assert abs(info.iterations - ito) <= 1
    oracle_rel = [np.linalg.norm(b - H.A[0] @ x) / np.linalg.norm(b) for x in hist[:5]]
    assert np.allclose(info.history[:5], oracle_rel, rtol=1e-6)
    solver.close()


@pytest.mark.parametrize("restart", [5, 50])
@pytest.mark.parametrize("name", ["2d_p2", "3d_p2"])
def test_gmres_fp64_matches_oracle(name, restart):
    # the paper's outer solver, right-preconditioned GMRES(m) (Sec. 4), against
    # the oracle's with the same FP64 V-cycle: residual estimates step by step,
    # iteration count and solution
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name, outer=cm.OUTER_GMRES, restart=restart, tol=1e-11)
    f = source_sine(cdg.nodes_phys().reshape(-1, mesh.dim))
    b = cdg.M0() @ f
    hist = []
    xo, ito, reso = gmres(H.A[0], b, lambda v: H.vcycle(v, 2, 2, 0.7), restart=restart, tol=1e-11, history=hist)
    u, info = solver.solve(f, history=True)
    assert info.rel_residual <= 1e-11
    assert abs(info.iterations - ito) <= 1, (info.iterations, ito)
    n = min(8, len(hist), info.iterations)
    assert np.allclose(info.history[:n], hist[:n], rtol=1e-6)
    ref = spl.spsolve(H.A[0].tocsc(), b)
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    solver.close()


def test_gmres_fp32_mg_reaches_tolerance():
    mesh, solver, cdg, H, kappa, parents, sizes = _build("2d_p3", mg=cm.MG_FP32, outer=cm.OUTER_GMRES, restart=20,
                                                         tol=1e-10)
    f = source_sine(cdg.nodes_phys().reshape(-1, mesh.dim))
    u, info = solver.solve(f)
    assert info.rel_residual <= 1e-10
    ref = spl.spsolve(H.A[0].tocsc(), cdg.M0() @ f)
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)
    solver.close()


def test_gmres_restart_out_of_range():
    with pytest.raises(cm.CdgmgError) as ei:
        _build("2d_p1", outer=cm.OUTER_GMRES, restart=0)
    assert ei.value.code == -1


@pytest.mark.parametrize("name", ["2d_p2", "3d_p2"])
def test_mass_and_grad_kappa_match_oracle(name):
    mesh, solver, cdg, H, kappa, parents, sizes = _build(name)
    rng = np.random.default_rng(5)
    n = H.A[0].shape[0]
    x = rng.standard_normal(n)
    assert np.allclose(solver.apply_mass(x).cpu().numpy(), cdg.M0() @ x, rtol=0, atol=1e-15 * np.abs(x).max())
    u, lam = rng.standard_normal(n), rng.standard_normal(n)
    g = solver.grad_kappa(u, lam).cpu().numpy()
    ref = oracle_grad_kappa(cdg, u, lam)
    assert np.abs(g - ref).max() <= 1e-12 * np.abs(ref).max()
    solver.close()


def test_update_kappa_rebuilds_operators():
    mesh, solver, cdg, H, kappa, parents, sizes = _build("2d_p2")
    k2 = np.random.default_rng(9).uniform(0.1, 10.0, mesh.n_elem)
    solver.update_kappa(k2)
    H2 = Hierarchy(cdg, parents, kappa=k2, coarsening="primal")
    for l in range(len(sizes)):
        A = cm.bsr_to_scipy(*solver.export_operator(l))
        assert abs(A - H2.A[l]).max() <= 1e-12 * abs(H2.A[l]).max()
    solver.close()


def test_error_paths():
    mesh = mesh2d_jittered_delaunay(6, 1)
    parents, sizes = cm.agglomerate(mesh, 2, 1, p=1)
    with pytest.raises(cm.CdgmgError) as ei:
        cm.Solver(mesh, 1, -np.ones(mesh.n_elem), parents, sizes)
    assert ei.value.code == -1
    solver = cm.Solver(mesh, 1, np.ones(mesh.n_elem), parents, sizes, max_iter=1, tol=1e-14)
    f = np.ones(mesh.n_elem * 3)
    u, info = solver.solve(f)  # NOT_CONVERGED is a warning; info is filled
    assert info.iterations == 1 and info.rel_residual > 1e-14
    with pytest.raises(cm.CdgmgError) as ei:
        solver.solve(np.full(mesh.n_elem * 3, np.nan))
    assert ei.value.code == -7
    solver.close()


@pytest.mark.parametrize("name", ["2d_p2", "2d_p3", "3d_p2", "3d_p1"])
def test_flux_coarse_operators_match_oracle(name):
    # GPU flux-form coarsening (Sec. 4.1) against the oracle, which coarsens
    # M, G, C separately and takes the Schur complement
    d, n, p, levels, seed = CASES[name]
    mesh = mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)
    parents, sizes = cm.agglomerate(mesh, levels, seed, p=p)
    kappa = np.random.default_rng(seed).uniform(0.5, 2.0, mesh.n_elem)
    print("case", name, "flux", list(sizes), flush=True)
    # these fixed cases keep every flux-coarsened diagonal block and the
    # coarsest operator nonsingular: setup must succeed
    solver = cm.Solver(mesh, p, kappa, parents, sizes, mg_precision=cm.MG_FP64, coarsening=cm.COARSEN_FLUX)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, p)
    H = Hierarchy(cdg, parents, kappa=kappa, coarsening="flux")
    for l in range(len(sizes)):
        A = cm.bsr_to_scipy(*solver.export_operator(l))
        R = H.A[l]
        err = abs(A - R).max() / abs(R).max()
        assert err <= 1e-11, (name, l, err)
    k2 = np.random.default_rng(3).uniform(0.2, 5.0, mesh.n_elem)
    solver.update_kappa(k2)
    H2 = Hierarchy(cdg, parents, kappa=k2, coarsening="flux")
    for l in range(len(sizes)):
        A = cm.bsr_to_scipy(*solver.export_operator(l))
        assert abs(A - H2.A[l]).max() <= 1e-11 * abs(H2.A[l]).max()
    solver.close()


@pytest.mark.parametrize("coarsening", ["primal", "flux"])
@pytest.mark.parametrize("gamma,mode,sseed", [(10.0, 0, 0), (1e2, 1, 0), (1e3, 1, 7)])
def test_level_operators_gamma_and_switch(gamma, mode, sseed, coarsening):
    # the coarsening and switch studies change only setup options: the Dirichlet
    # penalty gamma (Sec. 2.2) and the natural switch (Sec. 4.2)
    mesh = mesh2d_jittered_delaunay(11, 2)
    parents, sizes = cm.agglomerate(mesh, 3, 4, p=2)
    kappa = np.random.default_rng(6).uniform(0.5, 2.0, mesh.n_elem)
    cflag = cm.COARSEN_PRIMAL if coarsening == "primal" else cm.COARSEN_FLUX
    print("case gamma", gamma, "switch", mode, sseed, coarsening, list(sizes), flush=True)
    solver = cm.Solver(mesh, 2, kappa, parents, sizes, mg_precision=cm.MG_FP64, coarsening=cflag, gamma=gamma,
                       switch_mode=mode, switch_seed=sseed)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, 2, gamma=gamma,
              switch="consistent" if mode == cm.SWITCH_CONSISTENT else "natural", switch_seed=sseed)
    H = Hierarchy(cdg, parents, kappa=kappa, coarsening=coarsening)
    for l in range(len(sizes)):
        A = cm.bsr_to_scipy(*solver.export_operator(l))
        R = H.A[l]
        assert abs(A - R).max() <= 1e-11 * abs(R).max(), (l, abs(A - R).max())
    solver.close()


def test_flux_solve_small_mesh():
    # on a small mesh the flux-coarsened levels are still definite and the
    # flux-preconditioned FCG converges to the direct solution
    mesh = mesh2d_jittered_delaunay(8, 1)
    parents, sizes = cm.agglomerate(mesh, 3, 11, p=2)
    kappa = np.ones(mesh.n_elem)
    solver = cm.Solver(mesh, 2, kappa, parents, sizes, mg_precision=cm.MG_FP32, coarsening=cm.COARSEN_FLUX,
                       tol=1e-11)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, 2)
    f = source_sine(cdg.nodes_phys().reshape(-1, 2))
    u, info = solver.solve(f)
    ref = spl.spsolve(cdg.A().tocsc(), cdg.M0() @ f)
    assert info.rel_residual <= 1e-11
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    solver.close()


def test_compensated_outer_loop_reaches_below_fp64_floor():
    # 2D p=3 at n=72: the FP64 rounding noise of one residual is ~3e-11 of
    # ||b|| (eps || |A||u| || / ||b||); the compensated outer loop (Dot2 q and
    # true residual, double-double iterate) still reaches 1e-13
    mesh = mesh2d_jittered_delaunay(72, 2)
    parents, sizes = cm.agglomerate(mesh, 5, 12, p=3)
    solver = cm.Solver(mesh, 3, np.ones(mesh.n_elem), parents, sizes, tol=1e-13, max_iter=400)
    f = source_sine(solver.node_coords().reshape(-1, 2))
    u, info = solver.solve(f, history=True)
    print("iterations", info.iterations, "true residual", info.rel_residual, flush=True)
    assert info.rel_residual <= 1e-13
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, 3)
    A = cdg.A()
    b = cdg.M0() @ f
    floor = 2.2e-16 * np.linalg.norm(abs(A) @ np.abs(u.cpu().numpy())) / np.linalg.norm(b)
    assert floor > 1e-12  # the target is below what a plain FP64 residual can resolve
    ref = spl.spsolve(A.tocsc(), b)
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref)
    solver.close()


from hypothesis import assume, example, given, settings, strategies as st  # noqa: E402


@settings(max_examples=15, deadline=None)
@given(d=st.sampled_from([2, 3]), n=st.integers(2, 8), p=st.integers(1, 3), levels=st.integers(1, 5),
       seed=st.integers(0, 10**6), nu=st.sampled_from([(2, 2), (0, 3), (1, 1), (3, 1)]),
       omega=st.sampled_from([0.5, 2.0 / 3.0, 0.7]))
# a coarsest operator of condition 4.7e5: the pivot pairs of the coarsest
# Gauss-Jordan inverse must be as accurate as scalar pivots here
@example(d=2, n=4, p=3, levels=2, seed=564, nu=(2, 2), omega=0.5)
# a coarsest operator of condition 4.0e5 on which the two sides, rounding
# differently, differ by 1.9e-11 relative
@example(d=2, n=5, p=3, levels=3, seed=163, nu=(2, 2), omega=0.5)
def test_vcycle_fp64_random_cases(d, n, p, levels, seed, nu, omega):
    # the FP64 V-cycle against the oracle's on random meshes, hierarchies and
    # cycle settings (sizes from below one slice to several slices).  The two
    # sides round differently (summation orders of the sweeps, the explicit
    # Gauss-Jordan inverse against the oracle's LU solve), and the coarsest
    # direct solve amplifies rounding by up to the condition number of A_L
    # (the forward-error bound of a linear solve): 1e-11 up to condition 1e5,
    # eps-scaled beyond
    n = 2 + n % 4 if d == 3 else 2 * n  # up to 750 tetrahedra or 512 triangles
    mesh = mesh2d_jittered_delaunay(n, seed % 97) if d == 2 else mesh3d_kuhn(n, seed % 97)
    parents, sizes = cm.agglomerate(mesh, levels, seed, p=p)
    assume(int(sizes[-1]) * cm.n_basis(d, p) <= 3000)  # the oracle's dense coarsest solve stays quick
    kappa = np.random.default_rng(seed).uniform(0.5, 2.0, mesh.n_elem)
    print("case random", d, n, p, list(sizes), nu, omega, flush=True)
    solver = cm.Solver(mesh, p, kappa, parents, sizes, mg_precision=cm.MG_FP64, nu1=nu[0], nu2=nu[1], omega=omega)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, p)
    H = Hierarchy(cdg, parents, kappa=kappa, coarsening="primal")
    r = np.random.default_rng(seed + 1).standard_normal(H.A[0].shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, nu[0], nu[1], omega)
    AL = H.A[-1]
    cond = np.linalg.cond(AL.toarray() if hasattr(AL, "toarray") else np.asarray(AL))
    assert np.linalg.norm(z - ref) <= 1e-16 * max(1e5, cond) * np.linalg.norm(ref), cond
    solver.close()
