"""Pins for the oracle's right-preconditioned GMRES(m) (Sec. 4): the Arnoldi
identity, the minimal-residual property against a brute-force least-squares
over the Krylov space, finite termination, and the solution of the CDG system."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle.agglomerate import build_hierarchy
from oracle.cdg import CDG
from oracle.krylov import arnoldi, gmres
from oracle.multigrid import Hierarchy
from workloads import mesh2d_jittered_delaunay, source_sine


def _cdg_system(n=6, p=1, levels=3, seed=11):
    m = mesh2d_jittered_delaunay(n, 1)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    parents = build_hierarchy(m.e2v, cdg.topo.neighbor_pairs(), levels, seed)
    H = Hierarchy(cdg, parents)
    b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, 2))
    return cdg, H, b


def test_arnoldi_identity_and_orthonormality():
    cdg, H, b = _cdg_system()
    A = H.A[0]
    V, Z, Hm = arnoldi(A, H.vcycle, b, 12)
    # modified Gram-Schmidt loses orthogonality in proportion to cond(AB) eps
    assert np.abs(V @ V.T - np.eye(V.shape[0])).max() <= 1e-10
    lhs = np.stack([A @ z for z in Z], axis=1)          # A Z^T
    assert np.abs(lhs - V.T @ Hm).max() <= 1e-12 * np.abs(lhs).max()
    for j in range(Hm.shape[1]):                          # upper Hessenberg
        assert np.all(Hm[j + 2:, j] == 0.0)
    for j in range(len(Z)):                               # z_j = B v_j
        assert np.allclose(Z[j], H.vcycle(V[j]), rtol=0, atol=1e-14 * np.abs(Z[j]).max())


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("preconditioned", [False, True])
def test_minimal_residual_over_the_krylov_space(k, preconditioned):
    # x_k = B y_k, y_k minimises ||b - A B y|| over span{b, (AB) b, ..., (AB)^(k-1) b};
    # brute force: explicit Krylov matrix, orthonormalised by QR, least squares
    rng = np.random.default_rng(k)
    n = 40
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    A = Q @ np.diag(np.linspace(1.0, 30.0, n)) @ Q.T + 0.3 * rng.standard_normal((n, n))
    Bm = np.diag(rng.uniform(0.5, 2.0, n)) if preconditioned else np.eye(n)
    b = rng.standard_normal(n)
    x, it, res = gmres(A, b, lambda v: Bm @ v, restart=k, tol=1e-30, maxiter=k)
    assert it == k
    AB = A @ Bm
    K = np.zeros((n, k))
    v = b.copy()
    for j in range(k):
        K[:, j] = v / np.linalg.norm(v)
        v = AB @ K[:, j]
    Qk = np.linalg.qr(K)[0]
    y = np.linalg.lstsq(AB @ Qk, b, rcond=None)[0]
    best = np.linalg.norm(b - AB @ (Qk @ y)) / np.linalg.norm(b)
    assert abs(res - best) <= 1e-10 * max(best, 1e-12) + 1e-14
    assert np.linalg.norm(x - Bm @ (Qk @ y)) <= 1e-8 * np.linalg.norm(x)


def test_finite_termination():
    rng = np.random.default_rng(3)
    n = 24
    A = rng.standard_normal((n, n)) + n * np.eye(n)   # nonsymmetric, well conditioned
    b = rng.standard_normal(n)
    x, it, res = gmres(A, b, lambda v: v, restart=n, tol=1e-12, maxiter=n)
    assert it <= n and res <= 1e-12
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("restart", [5, 50])
def test_gmres_solves_the_cdg_system(restart):
    cdg, H, b = _cdg_system(n=8, p=2)
    hist = []
    x, it, res = gmres(H.A[0], b, H.vcycle, restart=restart, tol=1e-12, history=hist)
    ref = spl.spsolve(H.A[0].tocsc(), b)
    assert res <= 1e-12
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    assert len(hist) == it
    if restart >= it:  # one cycle: the estimates never increase
        assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))
