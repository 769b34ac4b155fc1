"""hp front end (Sec. 4, hp paragraph) on the GPU against the oracle: the
p-levels T^T A T (degree lowered by one per level, or in one jump to p = 1),
the agglomerated p = 1 levels, the V-cycle and the preconditioned solve
(calls through the C ABI)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from oracle.cdg import CDG  # noqa: E402
from oracle.multigrid import HpHierarchy  # noqa: E402
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine  # noqa: E402

# name: (dim, n, p, agglomeration levels, seed, p_jump)
CASES = {"2d_p3": (2, 12, 3, 4, 12, 0), "2d_p3_jump": (2, 12, 3, 4, 12, 1), "2d_p2": (2, 14, 2, 3, 11, 0),
         "3d_p2": (3, 4, 2, 3, 13, 0), "3d_p3": (3, 3, 3, 3, 7, 0), "3d_p3_jump": (3, 3, 3, 3, 7, 1)}


def _build(name, mg=cm.MG_FP64, **opts):
    d, n, p, levels, seed, jump = CASES[name]
    mesh = mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)
    parents, sizes = cm.agglomerate(mesh, levels, seed, p=p)
    kappa = np.random.default_rng(seed).uniform(0.5, 2.0, mesh.n_elem)
    degrees = [p, 1] if jump else list(range(p, 0, -1))
    print("case hp", name, "degrees", degrees, "sizes", list(sizes), flush=True)
    solver = cm.Solver(mesh, p, kappa, parents, sizes, mg_precision=mg, p_coarse=1, p_jump=jump, **opts)
    cdgs = [CDG(mesh.coords, mesh.e2v, mesh.face_bc, q) for q in degrees]
    H = HpHierarchy(cdgs, parents, kappa=kappa)
    return mesh, solver, cdgs[0], H, sizes


@pytest.mark.parametrize("name", list(CASES))
def test_hp_levels_match_oracle(name):
    mesh, solver, cdg, H, sizes = _build(name)
    ne, nz = solver.level_info()
    assert list(ne) == [mesh.n_elem] * len(H.A) + list(sizes)
    refs = list(H.A) + list(H.inner.A)
    for l, R in enumerate(refs):
        A = cm.bsr_to_scipy(*solver.export_operator(l))
        assert A.shape == R.shape, l
        assert abs(A - R).max() <= 1e-12 * abs(R).max(), l
    solver.close()


@pytest.mark.parametrize("nu1,nu2,omega", [(2, 2, 0.7), (0, 3, 2.0 / 3.0)])
@pytest.mark.parametrize("name", list(CASES))
def test_hp_vcycle_matches_oracle(name, nu1, nu2, omega):
    mesh, solver, cdg, H, sizes = _build(name, nu1=nu1, nu2=nu2, omega=omega)
    r = np.random.default_rng(2).standard_normal(H.A0.shape[0])
    z = solver.vcycle(r).cpu().numpy()
    ref = H.vcycle(r, nu1, nu2, omega)
    assert np.linalg.norm(z - ref) <= 1e-11 * np.linalg.norm(ref)
    solver.close()


@pytest.mark.parametrize("name", ["2d_p3", "3d_p3"])
def test_hp_apply_A_on_p_levels(name):
    mesh, solver, cdg, H, sizes = _build(name, mg=cm.MG_FP32)
    rng = np.random.default_rng(4)
    for l, R in enumerate(list(H.A) + list(H.inner.A)):
        x = rng.standard_normal(R.shape[0])
        ref = R @ x
        y = solver.apply_A(l, x, 0).cpu().numpy()
        assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    solver.close()


@pytest.mark.parametrize("name,outer", [("2d_p3", cm.OUTER_FCG), ("3d_p2", cm.OUTER_GMRES),
                                        ("3d_p3_jump", cm.OUTER_PCG)])
def test_hp_fp32_solve(name, outer):
    mesh, solver, cdg, H, sizes = _build(name, mg=cm.MG_FP32, outer=outer, tol=1e-10)
    f = source_sine(cdg.nodes_phys().reshape(-1, mesh.dim))
    u, info = solver.solve(f)
    assert info.rel_residual <= 1e-10
    ref = spl.spsolve(H.A0.tocsc(), cdg.M0() @ f)
    assert np.linalg.norm(u.cpu().numpy() - ref) <= 1e-8 * np.linalg.norm(ref)
    solver.close()


def test_hp_kappa_update_rebuilds_every_level():
    mesh, solver, cdg, H, sizes = _build("2d_p3")
    d, n, p, levels, seed, jump = CASES["2d_p3"]
    parents, _ = cm.agglomerate(mesh, levels, seed, p=p)
    kappa = np.random.default_rng(99).uniform(0.2, 5.0, mesh.n_elem)
    solver.update_kappa(kappa)
    cdgs = [CDG(mesh.coords, mesh.e2v, mesh.face_bc, q) for q in (3, 2, 1)]
    H2 = HpHierarchy(cdgs, parents, kappa=kappa)
    r = np.random.default_rng(5).standard_normal(H2.A0.shape[0])
    ref = H2.vcycle(r)
    assert np.linalg.norm(solver.vcycle(r).cpu().numpy() - ref) <= 1e-11 * np.linalg.norm(ref)
    solver.close()


def test_hp_options_checked():
    mesh = mesh2d_jittered_delaunay(6, 1)
    parents, sizes = cm.agglomerate(mesh, 2, 1, p=2)
    for bad in (dict(coarsening=cm.COARSEN_FLUX), dict(p_jump=2), dict(p_coarse=2)):
        with pytest.raises(cm.CdgmgError) as ei:
            cm.Solver(mesh, 2, np.ones(mesh.n_elem), parents, sizes, **dict(dict(p_coarse=1), **bad))
        assert ei.value.code == -1
