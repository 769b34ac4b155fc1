"""Pins for the oracle's upwind convection term beta v . grad u (the
convection-diffusion example of Sec. 5): a closed-form integral, the upwind
energy identity, and the V-cycle / GMRES solve of the nonsymmetric system."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle.agglomerate import build_hierarchy
from oracle.cdg import CDG
from oracle.krylov import gmres
from oracle.multigrid import Hierarchy
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn


@pytest.mark.parametrize("p", [2, 3])
def test_integral_of_convective_derivative(p):
    # u = x y (exactly represented for p >= 2, continuous, zero on the inflow
    # side x = 0), w = 1: c(u, 1) = beta int_Omega d(xy)/dx = beta / 2
    m = mesh2d_jittered_delaunay(6, 3)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    X = cdg.nodes_phys().reshape(-1, 2)
    u = X[:, 0] * X[:, 1]
    beta = 2.5
    C = cdg.Cv(beta, (1.0, 0.0))
    assert abs(np.ones(len(u)) @ (C @ u) - beta / 2) <= 1e-12


def _jump_energy(cdg, u, beta, v):
    """1/2 sum_interior int |beta v.n| [u]^2 + 1/2 sum_boundary int |beta v.n| u^2,
    from the traces (independent of the matrix)."""
    npb = cdg.np
    U = u.reshape(cdg.N, npb)
    tot = 0.0
    for (a, ia, b, ib) in cdg.topo.interior:
        pts, wts, nrm, _ = cdg.fq[a, ia]
        ua = cdg.ref.eval(cdg.xi_of(a, pts)) @ U[a]
        ub = cdg.ref.eval(cdg.xi_of(b, pts)) @ U[b]
        tot += 0.5 * abs(beta * np.dot(v, nrm)) * np.sum(wts * (ua - ub) ** 2)
    for (e, i) in cdg.topo.boundary:
        pts, wts, nrm, _ = cdg.fq[e, i]
        ue = cdg.ref.eval(cdg.xi_of(e, pts)) @ U[e]
        tot += 0.5 * abs(beta * np.dot(v, nrm)) * np.sum(wts * ue ** 2)
    return tot


@pytest.mark.parametrize("d,p", [(2, 1), (2, 3), (3, 2)])
def test_upwind_energy_identity(d, p):
    # u^T C u = 1/2 sum |beta v.n| [u]^2 over facets (v constant, all boundaries
    # Dirichlet): the volume term integrates to half the boundary flux
    m = mesh2d_jittered_delaunay(5, 2) if d == 2 else mesh3d_kuhn(2, 2)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    v = np.array([1.0, 0.3, -0.4])[:d]
    beta = 1.7
    C = cdg.Cv(beta, v)
    u = np.random.default_rng(1).standard_normal(C.shape[0])
    assert abs(u @ (C @ u) - _jump_energy(cdg, u, beta, v)) <= 1e-11 * abs(u @ (C @ u))


def test_continuous_functions_see_only_the_inflow_boundary():
    # for functions without jumps across interior facets (global polynomials,
    # exactly represented) the form is the volume integral of beta (v . grad u) w
    # plus the inflow boundary term of the Dirichlet data 0
    m = mesh2d_jittered_delaunay(5, 1)
    cdg = CDG(m.coords, m.e2v, m.face_bc, 2)
    X = cdg.nodes_phys().reshape(-1, 2)
    u = 1.0 + X[:, 0] - 2 * X[:, 1] + X[:, 0] * X[:, 1]
    w = X[:, 1] ** 2
    beta = 3.0
    C = cdg.Cv(beta, (1.0, 0.0))
    # exact: beta int (1 + y) y^2 over the unit square minus the inflow (x = 0)
    # term -int beta (v.n) u w = +beta int_0^1 (1 - 2y) y^2 dy
    exact = beta * (1 / 3 + 1 / 4) + beta * (1 / 3 - 2 / 4)
    assert abs(w @ (C @ u) - exact) <= 1e-12


@pytest.mark.parametrize("beta", [1.0, 10.0])
def test_convection_diffusion_gmres_solve(beta):
    m = mesh2d_jittered_delaunay(8, 1)
    cdg = CDG(m.coords, m.e2v, m.face_bc, 2)
    A = (cdg.A() + cdg.Cv(beta, (1.0, 0.0))).tocsr()
    parents = build_hierarchy(m.e2v, cdg.topo.neighbor_pairs(), 3, 11)
    H = Hierarchy(cdg, parents, coarsening="primal", A0=A)
    assert H.coarse_lu is not None
    b = cdg.M0() @ np.ones(A.shape[0])
    x, it, res = gmres(A, b, H.vcycle, restart=50, tol=1e-12)
    ref = spl.spsolve(A.tocsc(), b)
    assert res <= 1e-12 and np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    # the transpose system with the V-cycle of the transposed hierarchy and
    # the pre/post sweep counts swapped
    Ht = Hierarchy(cdg, parents, coarsening="primal", A0=A.T.tocsr())
    for l in range(len(H.A)):
        assert abs(Ht.A[l] - H.A[l].T).max() <= 1e-13 * abs(H.A[l]).max()
    g = np.random.default_rng(2).standard_normal(A.shape[0])
    lam, it2, res2 = gmres(A.T.tocsr(), g, lambda r: Ht.vcycle(r, 2, 2, 0.7), restart=50, tol=1e-12)
    assert res2 <= 1e-12
    assert np.linalg.norm(lam - spl.spsolve(A.T.tocsc(), g)) <= 1e-9 * np.linalg.norm(lam)
