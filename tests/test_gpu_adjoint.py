"""Adjoint gradients through the GPU hierarchy: oracle gradient, difference-form
central FD, homogeneity identity and the exact dL/df."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2012_08024_amd as cm  # noqa: E402
from paper_2012_08024_amd import autograd as cga  # noqa: E402
from oracle.adjoint import gradients_direct  # noqa: E402
from oracle.cdg import CDG  # noqa: E402
from workloads import CONFIGS, config_mesh, kappa_grf, mesh2d_jittered_delaunay, source_sine  # noqa: E402


def _setup(mesh, kappa, p, tol, levels=None, coarse_dofs=2000):
    parents, sizes = cm.agglomerate(mesh, levels or 50, 14, p=p, coarse_dofs=coarse_dofs)
    print("levels", list(sizes), flush=True)
    return cm.Solver(mesh, p, kappa, parents, sizes, tol=tol, max_iter=1000)


def _loss_and_grads(solver, kappa_np, f_np, ut):
    kappa = torch.tensor(kappa_np, device="cuda", requires_grad=True)
    f = torch.tensor(f_np, device="cuda", requires_grad=True)
    u = cga.solve(solver, kappa, f)
    L = cga.mass_misfit(solver, u, ut)
    L.backward()
    return u.detach(), float(L.detach()), kappa.grad.detach(), f.grad.detach()


def test_gradients_match_oracle_small():
    # C4 family (p=3, log-normal kappa, l = 0.1) at n=24: oracle by direct solves
    mesh = mesh2d_jittered_delaunay(24, 4)
    p = 3
    kappa = kappa_grf(mesh, 41)
    solver = _setup(mesh, kappa, p, 1e-13)
    x = solver.node_coords().reshape(-1, 2)
    f = source_sine(x)
    ut, _ = solver.solve(f)  # target: solution at kappa = 1 ... recomputed below
    solver.update_kappa(np.ones(mesh.n_elem))
    ut, _ = solver.solve(f)
    u, L, gk, gf = _loss_and_grads(solver, kappa, f, ut)
    cdg = CDG(mesh.coords, mesh.e2v, mesh.face_bc, p)
    uo, Lo, gko, gfo, lam = gradients_direct(cdg, kappa, f, ut.cpu().numpy())
    assert np.linalg.norm(u.cpu().numpy() - uo) <= 1e-11 * np.linalg.norm(uo)
    assert abs(L - Lo) <= 1e-10 * abs(Lo)
    assert np.linalg.norm(gk.cpu().numpy() - gko) <= 1e-9 * np.linalg.norm(gko)
    assert np.linalg.norm(gf.cpu().numpy() - gfo) <= 1e-9 * np.linalg.norm(gfo)
    solver.close()


def test_c4_fd_homogeneity_and_grad_f():
    cfg = CONFIGS["c4"]
    mesh, kappa = config_mesh(cfg)
    p = cfg["p"]
    # solves at 1e-14: with the 1e4 Dirichlet penalty the error of du and lambda
    # can exceed their residual by orders of magnitude
    solver = _setup(mesh, kappa, p, 1e-14, coarse_dofs=cfg["coarse_dofs"])
    x = solver.node_coords().reshape(-1, 2)
    f_np = source_sine(x)
    f = torch.tensor(f_np, device="cuda")
    solver.update_kappa(np.ones(mesh.n_elem))
    ut, _ = solver.solve(f)
    u, L, gk, gf = _loss_and_grads(solver, kappa, f_np, ut)
    # homogeneity: sum_e kappa_e dL/dkappa_e = -(u - u_t)^T M0 u
    lhs = float(torch.dot(torch.tensor(kappa, device="cuda"), gk))
    rhs = -float(torch.dot(u - ut, solver.apply_mass(u)))
    assert abs(lhs - rhs) <= 1e-8 * abs(rhs)
    # dL/df: L is quadratic in f, so a central difference is exact for any
    # step; a unit step keeps the difference of the two losses large against
    # the solve error
    rng = np.random.default_rng(cfg["fd_seed"])
    dirn = torch.tensor(rng.standard_normal(f_np.shape), device="cuda")
    h = 1.0
    Ls = []
    for s in (1.0, -1.0):
        us, _ = solver.solve(f + s * h * dirn)
        r = us - ut
        Ls.append(0.5 * float(torch.dot(r, solver.apply_mass(r))))
    fd = (Ls[0] - Ls[1]) / (2 * h)
    assert abs(fd - float(torch.dot(gf, dirn))) <= 1e-7 * abs(fd)
    # dL/dkappa_e on 20 seeded elements: central FD (step 1e-6 kappa_e) in
    # difference form: A(k +- h e_e) du = -+ h A^(e) u.  A is linear in kappa,
    # so A^(e) u = (A(k + s e_e) - A(k - s e_e)) u / 2s holds for any step s;
    # s = kappa_e / 2 keeps the difference of the two products far above
    # their rounding (a step of 1e-6 would leave about 1e-10 relative noise
    # times the ratio of the penalty to the element's own terms)
    elems = rng.choice(mesh.n_elem, size=cfg["fd_count"], replace=False)
    r0 = u - ut
    Mr0 = solver.apply_mass(r0)
    errs, fds, gs = [], [], []
    kt = torch.tensor(kappa, device="cuda")
    for e in elems:
        hstep = cfg["fd_step"] * kappa[e]
        s_op = 0.5 * kappa[e]
        kp, km = kt.clone(), kt.clone()
        kp[e] += s_op
        km[e] -= s_op
        solver.update_kappa(kp)
        Apu = solver.apply_A(0, u)
        solver.update_kappa(km)
        Amu = solver.apply_A(0, u)
        Aeu = (Apu - Amu) / (2 * s_op)
        kp, km = kt.clone(), kt.clone()
        kp[e] += hstep
        km[e] -= hstep
        dLs = []
        for s, kk in ((1.0, kp), (-1.0, km)):
            solver.update_kappa(kk)
            du, _ = solver.solve_rhs(-s * hstep * Aeu)
            dLs.append(float(torch.dot(Mr0, du)) + 0.5 * float(torch.dot(du, solver.apply_mass(du))))
        fd_e = (dLs[0] - dLs[1]) / (2 * hstep)
        fds.append(fd_e)
        gs.append(float(gk[e]))
        errs.append(abs(fd_e - float(gk[e])) / abs(float(gk[e])))
    fds, gs = np.array(fds), np.array(gs)
    rel = np.linalg.norm(fds - gs) / np.linalg.norm(gs)
    print("FD vs adjoint over %d elements: relative 2-norm error %.2e, per-element max %.2e median %.2e"
          % (len(elems), rel, max(errs), float(np.median(errs))), flush=True)
    # relative error 1e-5 on every checked element and over the set
    assert rel <= 1e-5
    assert max(errs) <= 1e-5
    solver.close()


def test_unconverged_solves_raise_in_autograd():
    # a forward or adjoint solve stopped by max_iter must not return an
    # unconverged u, lambda or gradient through autograd
    mesh = mesh2d_jittered_delaunay(10, 4)
    parents, sizes = cm.agglomerate(mesh, 3, 14, p=2)
    solver = cm.Solver(mesh, 2, np.ones(mesh.n_elem), parents, sizes, tol=1e-12, max_iter=2)
    f_np = source_sine(solver.node_coords().reshape(-1, 2))
    kappa = torch.ones(mesh.n_elem, dtype=torch.float64, device="cuda", requires_grad=True)
    f = torch.tensor(f_np, device="cuda", requires_grad=True)
    with pytest.raises(cm.CdgmgError) as ei:
        cga.solve(solver, kappa, f)
    assert ei.value.code == cm.NOT_CONVERGED
    # the plain call keeps returning the last iterate with the warning in info
    u, info = solver.solve(f_np)
    assert info.iterations == 2 and info.rel_residual > 1e-12
    solver.close()
