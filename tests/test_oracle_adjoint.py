"""Pins for the oracle's adjoint gradients."""
import numpy as np

from oracle.adjoint import fd_kappa_difference_form, gradients_direct, loss
from oracle.cdg import CDG
from workloads import mesh2d_jittered_delaunay, source_sine


def _problem():
    m = mesh2d_jittered_delaunay(6, 4)
    cdg = CDG(m.coords, m.e2v, m.face_bc, 2)
    rng = np.random.default_rng(7)
    kappa = np.exp(rng.standard_normal(cdg.N) * 0.5)
    f = source_sine(cdg.nodes_phys().reshape(-1, 2))
    u_t, *_ = gradients_direct(cdg, np.ones(cdg.N), f, np.zeros(cdg.N * cdg.np))
    return cdg, kappa, f, u_t


def test_homogeneity_identity():
    # A is linear and homogeneous in kappa, so sum_e kappa_e dL/dkappa_e =
    # -lambda^T A u = -lambda^T b = -(u - u_t)^T M0 u.
    cdg, kappa, f, u_t = _problem()
    u, L, gk, gf, lam = gradients_direct(cdg, kappa, f, u_t)
    lhs = float(kappa @ gk)
    rhs = -float((u - u_t) @ (cdg.M0() @ u))
    assert abs(lhs - rhs) <= 1e-10 * abs(rhs)


def test_grad_f_central_difference():
    # L is quadratic in f, so a central difference is exact up to rounding.
    cdg, kappa, f, u_t = _problem()
    u, L, gk, gf, lam = gradients_direct(cdg, kappa, f, u_t)
    rng = np.random.default_rng(8)
    for _ in range(3):
        dirn = rng.standard_normal(f.shape)
        h = 1e-3
        Lp = gradients_direct(cdg, kappa, f + h * dirn, u_t)[1]
        Lm = gradients_direct(cdg, kappa, f - h * dirn, u_t)[1]
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - gf @ dirn) <= 1e-8 * abs(fd)


def test_grad_kappa_difference_form_fd():
    cdg, kappa, f, u_t = _problem()
    u, L, gk, gf, lam = gradients_direct(cdg, kappa, f, u_t)
    for e in (0, 17, 40, 63):
        fd = fd_kappa_difference_form(cdg, kappa, u, u_t, e, 1e-6)
        assert abs(fd - gk[e]) <= 1e-6 * np.abs(gk).max()
    assert loss(cdg, u, u_t) > 0
