"""Pins for the oracle's hp front end (Sec. 4, hp paragraph)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle.agglomerate import build_hierarchy
from oracle.cdg import CDG
from oracle.krylov import fcg
from oracle.multigrid import Hierarchy, HpHierarchy
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine


def _hp(d=2, n=8, p=3, levels=3, seed=11):
    m = mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)
    cdg, cdg1 = CDG(m.coords, m.e2v, m.face_bc, p), CDG(m.coords, m.e2v, m.face_bc, 1)
    parents = build_hierarchy(m.e2v, cdg.topo.neighbor_pairs(), levels, seed)
    return m, cdg, cdg1, parents


@pytest.mark.parametrize("d,p", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_embedding_reproduces_linear_functions(d, p):
    # T maps the P1 nodal values of a linear function to its degree-p nodal values
    m, cdg, cdg1, parents = _hp(d=d, n=4 if d == 2 else 2, p=p, levels=2)
    H = HpHierarchy(cdg, cdg1, parents)
    a = np.array([0.3, -1.2, 0.7, 2.0])[:d + 1]
    lin = lambda X: a[0] + X @ a[1:]  # noqa: E731
    u1 = lin(cdg1.nodes_phys().reshape(-1, d))
    up = lin(cdg.nodes_phys().reshape(-1, d))
    assert np.abs(H.Tb @ u1 - up).max() <= 1e-14
    assert np.allclose(H.T.sum(axis=1), 1.0)  # partition of unity


def test_coarse_correction_annihilates_the_p1_space():
    # with an exact p = 1 solve (one level), the two-level error propagation
    # I - Tb (Tb^T A Tb)^{-1} Tb^T A vanishes on Tb y
    m, cdg, cdg1, parents = _hp(n=6, p=3, levels=1)
    H = HpHierarchy(cdg, cdg1, [])
    y = np.random.default_rng(2).standard_normal(H.Tb.shape[1])
    e = H.Tb @ y
    A = H.A0
    ec = e - H.Tb @ H.inner.vcycle(H.Tb.T @ (A @ e))
    assert np.linalg.norm(ec) <= 1e-10 * np.linalg.norm(e)


def test_p1_input_is_the_plain_hierarchy():
    # at p = 1 the embedding is the identity and the p = 1 levels are those of
    # the plain hierarchy
    m, cdg, cdg1, parents = _hp(n=8, p=1, levels=3)
    Hp = HpHierarchy(cdg, cdg1, parents)
    H = Hierarchy(cdg, parents, coarsening="primal")
    assert np.allclose(Hp.T, np.eye(cdg.np))
    for l in range(len(H.A)):
        assert abs(Hp.inner.A[l] - H.A[l]).max() <= 1e-13 * abs(H.A[l]).max()


@pytest.mark.parametrize("d,p", [(2, 3), (3, 2)])
def test_hp_preconditioned_solve(d, p):
    m, cdg, cdg1, parents = _hp(d=d, n=8 if d == 2 else 3, p=p, levels=3)
    H = HpHierarchy(cdg, cdg1, parents)
    b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, d))
    x, it, res = fcg(H.A0, b, H.vcycle, tol=1e-12)
    ref = spl.spsolve(H.A0.tocsc(), b)
    assert res <= 1e-12 and it < 100
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
