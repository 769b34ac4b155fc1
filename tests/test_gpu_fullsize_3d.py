"""The 3D workloads at full size, in the configuration the benchmark times:
p = 2 on 105 456 Kuhn tetrahedra (n_p = 10, 1 054 560 DOFs, 5 levels) and
p = 3 on 384 000 (n_p = 20, 7 680 000 DOFs, 6 levels, a coefficient with
10^3 jumps across 32 spheres): sampled rows of the GPU-built level-0 product
A_0 x against the oracle row by row, and properties that hold at any size
for the V-cycle (one wavefront per 64-row slice, as at n_p = 10)."""
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


@pytest.fixture(scope="module", params=["c3", "c5"])
def c5(request):
    cfg = CONFIGS[request.param]
    mesh, kappa = config_mesh(cfg)
    parents, sizes = cm.agglomerate(mesh, cfg["levels"], cfg["agg_seed"], p=cfg["p"])
    print(request.param, "full size", list(sizes), flush=True)
    solver = cm.Solver(mesh, cfg["p"], kappa, parents, sizes, mg_precision=cm.MG_FP32, tol=cfg["tol"],
                       max_iter=1000)
    print(request.param, "setup done", flush=True)
    yield cfg, mesh, kappa, solver
    solver.close()


def test_sampled_rows_of_A0_x_match_oracle(c5):
    cfg, mesh, kappa, solver = c5
    npb = solver.np
    rng = np.random.default_rng(23)
    x = rng.standard_normal(mesh.n_elem * npb)
    y = solver.apply_A(0, x, 0).cpu().numpy()
    boundary = np.array(sorted({e for (e, _) in Topology(mesh.e2v, mesh.coords).boundary}))
    # elements inside the spheres and outside them (C5), on the boundary, and the ends
    hi = np.flatnonzero(kappa > 10.0)
    lo = np.flatnonzero(kappa <= 10.0)
    picks = set(rng.choice(lo, 12, replace=False).tolist())
    if len(hi):
        picks |= set(rng.choice(hi, 12, replace=False).tolist())
    sample = sorted(picks | set(rng.choice(boundary, 6, replace=False).tolist()) | {0, mesh.n_elem - 1})
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, cfg["p"], subset=sample)
    rows = cdg.A_rows(sample, kappa)
    X = x.reshape(-1, npb)
    for e in sample:
        ref = np.zeros(npb)
        mag = np.zeros(npb)
        for c, blk in rows[e].items():
            ref += blk @ X[c]
            mag += np.abs(blk) @ np.abs(X[c])
        got = y[e * npb:(e + 1) * npb]
        assert np.abs(got - ref).max() <= 1e-13 * mag.max(), e


def test_vcycle_is_symmetric_and_positive_at_full_size(c5):
    cfg, mesh, kappa, solver = c5
    n = mesh.n_elem * solver.np
    rng = np.random.default_rng(6)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    Bx, By = solver.vcycle(x).cpu().numpy(), solver.vcycle(y).cpu().numpy()
    assert abs(x @ By - y @ Bx) <= 1e-5 * np.linalg.norm(x) * np.linalg.norm(By)
    assert x @ Bx > 0 and y @ By > 0


def test_launch_configuration_is_parity_covered(c5):
    # every coarse-level lane group, transfer workgroup size and level-0
    # wavefront split this workload dispatches is compared with the oracle's
    # V-cycle in test_gpu_parity.py (FP32 V-cycle, this block size)
    cfg, mesh, kappa, solver = c5
    info = solver.launch_info()
    print("launch configuration", {k: (list(v) if hasattr(v, "__len__") else v) for k, v in info.items()}, flush=True)
    assert not uncovered(info, 1, solver.np)


def test_adjoint_homogeneity_identity_at_full_size(c5):
    # the gradient of L = 1/2 ||u - u_t||_M^2 through the FP32 V-cycle's FCG at
    # full size: sum_e kappa_e dL/dkappa_e = -(u - u_t)^T M_0 u (A is linear
    # and homogeneous in kappa, so lambda^T A u = (A lambda)^T u = g^T u; the
    # gap is -r_lambda^T u, of the order of the adjoint solve's residual).
    # u_t is the solution at kappa = 1 (the 3D p = 3 workload's target), or at
    # kappa = 2 where the workload's kappa is 1
    cfg, mesh, kappa, solver = c5
    f = torch.tensor(source_sine(solver.node_coords().reshape(-1, 3)), device="cuda")
    kt = np.ones(mesh.n_elem) * (2.0 if np.all(kappa == 1.0) else 1.0)
    solver.update_kappa(kt)
    ut, it_t = solver.solve(f, strict=True)
    solver.update_kappa(kappa)
    u, it_u = solver.solve(f, strict=True)
    g = solver.apply_mass(u - ut)
    lam, it_l = solver.solve_transpose(g, strict=True)
    gk = solver.grad_kappa(u, lam)
    lhs = float(torch.dot(torch.tensor(kappa, device="cuda"), gk))
    rhs = -float(torch.dot(u - ut, solver.apply_mass(u)))
    print("homogeneity: lhs %.12e rhs %.12e relative gap %.2e; iterations %d %d %d"
          % (lhs, rhs, abs(lhs - rhs) / abs(rhs), it_t.iterations, it_u.iterations, it_l.iterations), flush=True)
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)
