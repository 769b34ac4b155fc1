"""Full-size solution parity at the 2D p = 3 gradient workload (49 928
jittered Delaunay triangles, 499 280 DOFs, log-normal kappa, levels until
n_l n_p <= 2000): the GPU's FP64-MG and FP32-MG solutions against the
oracle's, element by element.

The oracle solution is the oracle's own FP64 FCG with its V-cycle, refined
twice with extended-precision residuals (oracle.krylov.refine), so that it
is not limited by the FP64 rounding of A x (about 1e-10 of ||b|| at this
size): its residual reaches the floor that the rounding of x's own entries
sets.  The GPU solves run to a relative residual of 1e-13 with the
compensated outer loop (a double-double iterate).  A smooth right-hand side
bounds the relative error by about the relative residual, so both sit well
below the bounds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from oracle.cdg import CDG  # noqa: E402
from oracle.krylov import fcg, refine  # noqa: E402
from oracle.multigrid import Hierarchy  # noqa: E402
from workloads import CONFIGS, config_mesh, source_sine  # noqa: E402


@pytest.fixture(scope="module")
def c4():
    cfg = CONFIGS["c4"]
    mesh, kappa = config_mesh(cfg)
    parents, sizes = cm.agglomerate(mesh, 50, cfg["agg_seed"], p=cfg["p"], coarse_dofs=cfg["coarse_dofs"])
    print("c4 full size", list(sizes), flush=True)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, cfg["p"])
    A = cdg.A(kappa).tocsr()
    f = source_sine(cdg.nodes_phys().reshape(-1, 2))
    b = cdg.M0() @ f
    print("oracle operator assembled", flush=True)
    H = Hierarchy(cdg, parents, kappa=kappa, coarsening="primal")
    print("oracle hierarchy built", flush=True)
    x, res = refine(A, b, lambda r: fcg(A, r, H.vcycle, tol=1e-8)[0], rounds=2)
    # no FP64 vector has a smaller residual than the rounding of its entries
    # allows, eps || |A| |x| || / ||b||: the refinement has reached it
    floor = np.finfo(np.float64).eps * np.linalg.norm(abs(A) @ np.abs(x)) / np.linalg.norm(b)
    print("oracle solution: extended-precision relative residual per round", res,
          "representation floor %.2e" % floor, flush=True)
    assert res[-1] <= 2.0 * floor and res[0] > 1e2 * res[-1]
    return cfg, mesh, kappa, parents, sizes, f, x


@pytest.mark.parametrize("mg,bound", [(cm.MG_FP64, 1e-10), (cm.MG_FP32, 1e-9)])
def test_full_size_solution_matches_oracle(c4, mg, bound):
    cfg, mesh, kappa, parents, sizes, f, x = c4
    s = cm.Solver(mesh, cfg["p"], kappa, parents, sizes, mg_precision=mg, tol=1e-13, max_iter=1000)
    u, info = s.solve(f)
    s.close()
    u = u.cpu().numpy()
    e_inf = np.abs(u - x).max() / np.abs(x).max()
    e_2 = np.linalg.norm(u - x) / np.linalg.norm(x)
    print("mg", mg, "iterations", info.iterations, "residual %.2e" % info.rel_residual,
          "error max %.2e 2-norm %.2e" % (e_inf, e_2), flush=True)
    assert info.rel_residual <= 1e-13
    assert e_inf <= bound and e_2 <= bound
