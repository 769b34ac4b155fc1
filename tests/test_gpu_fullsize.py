"""The 2D p=3 benchmark workload at full size (199 712 triangles, 1 997 120
DOFs, 6 levels), in the configuration the benchmark times (FP32 V-cycle in
FP64 FCG, automatic kernel choice): sampled rows of the GPU-built level-0
operator against the oracle element by element, and properties that hold at
any size for the solve and the V-cycle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from oracle.cdg import CDG  # noqa: E402
from oracle.mesh import Topology  # noqa: E402
from kernel_coverage import uncovered  # noqa: E402
from workloads import CONFIGS, config_mesh, source_sine  # noqa: E402


@pytest.fixture(scope="module")
def c2():
    cfg = CONFIGS["c2"]
    mesh, kappa = config_mesh(cfg)
    parents, sizes = cm.agglomerate(mesh, cfg["levels"], cfg["agg_seed"], p=cfg["p"])
    print("c2 full size", list(sizes), flush=True)
    solver = cm.Solver(mesh, cfg["p"], kappa, parents, sizes, mg_precision=cm.MG_FP32, tol=cfg["tol"])
    yield cfg, mesh, kappa, solver
    solver.close()


def test_sampled_level0_rows_match_oracle(c2):
    cfg, mesh, kappa, solver = c2
    rp, cols, blocks = solver.export_operator(0)
    rng = np.random.default_rng(17)
    boundary = np.array(sorted({e for (e, _) in Topology(mesh.e2v, mesh.coords).boundary}))
    sample = sorted(set(rng.choice(mesh.n_elem, 40, replace=False).tolist()) |
                    set(rng.choice(boundary, 8, replace=False).tolist()) | {0, mesh.n_elem - 1})
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, cfg["p"], subset=sample)
    rows = cdg.A_rows(sample, kappa)
    for e in sample:
        got = {int(cols[k]): blocks[k] for k in range(rp[e], rp[e + 1])}
        ref = rows[e]  # may hold exact-zero blocks of a host's stencil
        scale = max(np.abs(b).max() for b in ref.values())
        zero = np.zeros_like(blocks[0])
        for c in set(got) | set(ref):
            assert np.abs(got.get(c, zero) - ref.get(c, zero)).max() <= 1e-12 * scale, (e, c)
        assert len(got) <= 4  # the diagonal and at most three face neighbours


def test_solve_residual_with_the_exported_operator(c2):
    # the FP32-MG solution's FP64 residual, formed on the CPU from the
    # exported operator (checked row by row above): at this size the relative
    # rounding floor of one FP64 product is about 4.4e-10
    cfg, mesh, kappa, solver = c2
    f = source_sine(solver.node_coords().reshape(-1, 2))
    u, info = solver.solve(f)
    assert info.rel_residual <= 1e-10 and info.iterations < 100
    A = cm.bsr_to_scipy(*solver.export_operator(0))
    b = solver.apply_mass(f).cpu().numpy()
    r = b - A @ u.cpu().numpy()
    assert np.linalg.norm(r) <= 1e-9 * np.linalg.norm(b)


def test_vcycle_is_symmetric_at_full_size(c2):
    # V(2,2) with block-Jacobi sweeps is a symmetric operator; in FP32 to ~1e-6
    cfg, mesh, kappa, solver = c2
    n = mesh.n_elem * solver.np
    rng = np.random.default_rng(5)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    Bx, By = solver.vcycle(x).cpu().numpy(), solver.vcycle(y).cpu().numpy()
    assert abs(x @ By - y @ Bx) <= 1e-5 * np.linalg.norm(x) * np.linalg.norm(By)
    # and it is positive on these vectors
    assert x @ Bx > 0 and y @ By > 0


def test_launch_configuration_is_parity_covered(c2):
    # every coarse-level lane group, transfer workgroup size and level-0
    # wavefront split this workload dispatches is compared with the oracle's
    # V-cycle in test_gpu_parity.py (FP32 V-cycle, this block size)
    cfg, mesh, kappa, solver = c2
    info = solver.launch_info()
    print("launch configuration", {k: (list(v) if hasattr(v, "__len__") else v) for k, v in info.items()}, flush=True)
    assert not uncovered(info, 1, solver.np)
