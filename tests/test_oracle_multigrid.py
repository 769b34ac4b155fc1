"""Pins for the hierarchy, transfers, coarsening, V-cycle and Krylov solvers."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spl

from oracle.agglomerate import build_hierarchy
from oracle.cdg import CDG
from oracle.krylov import fcg, pcg
from oracle.multigrid import Hierarchy, block_diag_blocks
from oracle.refelem import monomial_exponents
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine


def _setup(d=2, n=8, p=2, levels=3, seed=11, bc=0, coarsening="primal", kappa=None):
    m = mesh2d_jittered_delaunay(n, 1, bc=bc) if d == 2 else mesh3d_kuhn(n, 1, bc=bc)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    parents = build_hierarchy(m.e2v, cdg.topo.neighbor_pairs(), levels, seed)
    return cdg, Hierarchy(cdg, parents, kappa=kappa, coarsening=coarsening)


@pytest.mark.parametrize("d,p", [(2, 2), (3, 2)])
def test_transfers_orthonormal(d, p):
    # L^T M_l L = I: the coarse modal bases are L2-orthonormal on each aggregate.
    cdg, H = _setup(d=d, n=8 if d == 2 else 3, p=p, levels=4)
    M = cdg.M0()
    for P in H.P:
        Mc = (P.T @ M @ P).toarray()
        assert np.abs(Mc - np.eye(Mc.shape[0])).max() <= 1e-12
        M = P.T @ M @ P


def test_prolongation_reproduces_coarse_polynomials():
    # Injection (Sec. 3.4): a global polynomial of degree <= p, written in the
    # coarsest basis and prolongated to level 0, equals its nodal values.
    cdg, H = _setup(n=8, p=3, levels=4)
    rng = np.random.default_rng(2)
    exps = monomial_exponents(2, 3)
    c = rng.standard_normal(len(exps))

    def poly(x):
        return sum(ci * x[..., 0] ** e[0] * x[..., 1] ** e[1] for ci, e in zip(c, exps))

    L = H.L
    # coarsest coefficients of poly by L2 projection (orthonormal basis)
    uc = np.zeros(H.sizes[L] * H.np)
    for I in range(H.sizes[L]):
        fine = np.nonzero(H.anc[L] == I)[0]
        x = H.qpts[fine].reshape(-1, 2)
        w = H.qwts[fine].ravel()
        uc[I * H.np:(I + 1) * H.np] = H.basis_at(L, I, x).T @ (w * poly(x))
    u = uc
    for P in reversed(H.P):
        u = P @ u
    ref = poly(cdg.nodes_phys()).ravel()
    assert np.abs(u - ref).max() <= 1e-11 * np.abs(ref).max()


def test_flux_coarsening_dense_rederivation_and_loewner_order():
    # A_c(flux) = L^T C L + (Lq^T G L)^T (Lq^T M Lq)^{-1} (Lq^T G L), written with
    # dense global matrices and Lq = I_d (x) L, and A_c(primal) - A_c(flux) =
    # X^T (M^-1 - Lq (Lq^T M Lq)^-1 Lq^T) X >= 0 with X = G L.
    cdg, H = _setup(n=6, p=1, levels=2, coarsening="flux",
                    kappa=np.random.default_rng(5).uniform(0.5, 2.0, 72))
    d = cdg.d
    P = H.P[0].toarray()
    Cm = cdg.C(H.kappa).toarray()
    Gm = np.vstack([g.toarray() for g in cdg.G()])              # [d*n, n]
    Mm = sla.block_diag(*([cdg.Mflux(H.kappa).toarray()] * d))  # component-major
    Lq = sla.block_diag(*([P] * d))
    Gc = Lq.T @ Gm @ P
    Ac = P.T @ Cm @ P + Gc.T @ np.linalg.solve(Lq.T @ Mm @ Lq, Gc)
    assert np.abs(Ac - H.A[1].toarray()).max() <= 1e-11 * np.abs(Ac).max()
    Aprim = P.T @ cdg.A(H.kappa).toarray() @ P
    diff = Aprim - Ac
    assert np.abs(diff - diff.T).max() <= 1e-10 * np.abs(Aprim).max()
    assert np.linalg.eigvalsh(diff)[0] >= -1e-10 * np.abs(Aprim).max()


def test_flux_coarsening_polynomial_identity_all_neumann():
    # With no Dirichlet facet the coarse flux operator acts on coarse global
    # polynomials exactly like the fine operator (liftings of zero jumps vanish).
    cdg, H = _setup(n=8, p=2, levels=3, bc=1, coarsening="flux")
    rng = np.random.default_rng(4)
    for l in range(1, H.L + 1):
        # global polynomial in level-l coefficients
        exps = monomial_exponents(2, 2)
        c = rng.standard_normal(len(exps))
        uc = np.zeros(H.sizes[l] * H.np)
        for I in range(H.sizes[l]):
            fine = np.nonzero(H.anc[l] == I)[0]
            x = H.qpts[fine].reshape(-1, 2)
            w = H.qwts[fine].ravel()
            val = sum(ci * x[:, 0] ** e[0] * x[:, 1] ** e[1] for ci, e in zip(c, exps))
            uc[I * H.np:(I + 1) * H.np] = H.basis_at(l, I, x).T @ (w * val)
        Pl = None
        for k in range(l):
            Pl = H.P[k] if Pl is None else Pl @ H.P[k]
        lhs = H.A[l] @ uc
        rhs = Pl.T @ (H.A[0] @ (Pl @ uc))
        assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(rhs).max() + 1e-12


@pytest.mark.parametrize("p", [1, 2, 3])
def test_flux_coarse_operators_definite_on_the_uniform_square(p):
    # Sec. 5.1's mesh class (uniform square of right triangles, Neumann on
    # x = 0, 1, Dirichlet on y = 0, 1): the flux-form coarse operators are
    # definite, with no eigenvalue below the continuous problem's smallest,
    # pi^2 (mode sin(pi y)), up to the discretisation error; on the
    # orthonormal agglomerate bases of level 1 at p >= 2 they reach it.  The
    # same holds for primal coarsening.
    from workloads.meshes import mesh2d_square_neumann_sides
    m = mesh2d_square_neumann_sides(8)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    parents = build_hierarchy(m.e2v, cdg.topo.neighbor_pairs(), 3, 1)
    for coarsening in ("flux", "primal"):
        H = Hierarchy(cdg, parents, coarsening=coarsening)
        for l in (1, 2):
            lam = np.linalg.eigvalsh(H.A[l].toarray())[0]
            assert lam >= 0.95 * np.pi ** 2, (coarsening, l, lam)
            if l == 1 and p >= 2:
                assert lam <= 1.01 * np.pi ** 2, (coarsening, l, lam)


def test_flux_coarse_operator_indefinite_on_a_jittered_mesh():
    # the contrast: with vertex jitter the cross-facet lifting terms of C make
    # the flux-form A_1 indefinite (primal coarsening stays definite)
    cdg, H = _setup(n=16, p=1, levels=3, coarsening="flux")
    assert np.linalg.eigvalsh(H.A[1].toarray())[0] < 0
    _, Hp = _setup(n=16, p=1, levels=3, coarsening="primal")
    assert np.linalg.eigvalsh(Hp.A[1].toarray())[0] > 0


@pytest.mark.parametrize("coarsening", ["primal", "flux"])
def test_coarse_operators_symmetric(coarsening):
    cdg, H = _setup(n=8, p=2, levels=4, coarsening=coarsening)
    for A in H.A:
        A = A.toarray()
        assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()


def test_two_level_cycle_equals_error_propagation_matrix():
    # One V(nu1,nu2) cycle with an exact coarse solve applied to b gives
    # x = (I - E) A^{-1} b with E = S^nu2 (I - L A_c^{-1} L^T A) S^nu1,
    # S = I - omega D^{-1} A.
    cdg, H = _setup(n=6, p=1, levels=2)
    A = H.A[0].toarray()
    Dinv = sla.block_diag(*np.linalg.inv(block_diag_blocks(H.A[0], H.np)))
    P = H.P[0].toarray()
    Ac = P.T @ A @ P
    n = A.shape[0]
    w = 0.7
    S = np.eye(n) - w * Dinv @ A
    E = np.linalg.matrix_power(S, 2) @ (np.eye(n) - P @ np.linalg.solve(Ac, P.T @ A)) @ np.linalg.matrix_power(S, 2)
    b = np.random.default_rng(0).standard_normal(n)
    x = H.vcycle(b, 2, 2, w)
    ref = (np.eye(n) - E) @ np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("solver", [pcg, fcg])
def test_krylov_solution_matches_direct_solve(solver):
    cdg, H = _setup(n=8, p=2, levels=3)
    b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, 2))
    x, it, res = solver(H.A[0], b, H.vcycle, tol=1e-13)
    ref = spl.spsolve(H.A[0].tocsc(), b)
    assert res <= 1e-13
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_fcg1_iterates_equal_pcg_for_symmetric_preconditioner():
    cdg, H = _setup(n=8, p=2, levels=3)
    b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, 2))
    h1, h2 = [], []
    pcg(H.A[0], b, H.vcycle, tol=1e-30, maxiter=10, history=h1)
    fcg(H.A[0], b, H.vcycle, tol=1e-30, maxiter=10, history=h2)
    for a, c in zip(h1, h2):
        assert np.linalg.norm(a - c) <= 1e-10 * np.linalg.norm(a)
    # and the residual contracts
    r = [np.linalg.norm(b - H.A[0] @ x) for x in h1]
    assert (r[-1] / r[0]) ** (1.0 / (len(r) - 1)) < 1.0


def test_refinement_recovers_an_exact_integer_solution():
    # iterative refinement with an extended-precision residual: on an SPD
    # system with integer entries and an integer solution x* (b = A x* exact
    # in FP64), inner solves accurate to only 1e-3 still reach x* to the
    # rounding of x; the extended residual falls by about 1e-3 per round
    import scipy.sparse as sp
    from oracle.krylov import refine
    n = 40
    T = sp.diags([-np.ones(n - 1), 4.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    A = (sp.kron(sp.eye(n), T) + sp.kron(sp.diags([-np.ones(n - 1), -np.ones(n - 1)], [-1, 1]), sp.eye(n)))
    A = (A + sp.eye(n * n) * 0.25).tocsr()  # entries 4.25 and -1: exact in FP64, and so is b
    xs = np.random.default_rng(3).integers(-50, 50, n * n).astype(np.float64)
    b = A @ xs
    assert np.array_equal(b, np.asarray((A.astype(np.longdouble) @ xs.astype(np.longdouble)), dtype=np.float64))
    Dinv = 1.0 / A.diagonal()
    x, res = refine(A, b, lambda r: fcg(A, r, lambda v: Dinv * v, tol=1e-3)[0], rounds=6)
    assert np.abs(x - xs).max() <= 1e-13 * np.abs(xs).max()
    assert res[-1] <= 1e-15
    assert all(res[k + 1] <= 1e-2 * res[k] for k in range(3))
    # a plain FP64 solve to the same final residual is not available: FCG
    # at 1e-3 alone stays far from x*
    x0 = fcg(A, b, lambda v: Dinv * v, tol=1e-3)[0]
    assert np.abs(x0 - xs).max() > 1e-6 * np.abs(xs).max()
