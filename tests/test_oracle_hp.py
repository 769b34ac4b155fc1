"""Pins for the oracle's hp front end (Sec. 4, hp paragraph): p-multigrid
down to p = 1 by nodal embeddings, then agglomeration at p = 1."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle.agglomerate import build_hierarchy
from oracle.cdg import CDG
from oracle.krylov import fcg
from oracle.multigrid import Hierarchy, HpHierarchy
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, source_sine


def _mesh(d, n):
    return mesh2d_jittered_delaunay(n, 1) if d == 2 else mesh3d_kuhn(n, 1)


def _hp(d=2, n=8, degrees=(3, 1), levels=3, seed=11):
    m = _mesh(d, n)
    cdgs = [CDG(m.coords, m.e2v, m.face_bc, q) for q in degrees]
    parents = build_hierarchy(m.e2v, cdgs[0].topo.neighbor_pairs(), levels, seed) if levels > 1 else []
    return m, cdgs, parents


@pytest.mark.parametrize("d,degrees", [(2, (2, 1)), (2, (3, 1)), (2, (3, 2, 1)), (3, (2, 1)), (3, (3, 2, 1))])
def test_embedding_reproduces_lower_degree_polynomials(d, degrees):
    # T_k maps the degree-p_{k+1} nodal values of a polynomial of that degree
    # to its degree-p_k nodal values, exactly
    m, cdgs, parents = _hp(d=d, n=4 if d == 2 else 2, degrees=degrees, levels=1)
    H = HpHierarchy(cdgs, parents)
    rng = np.random.default_rng(3)
    for k in range(len(degrees) - 1):
        q = degrees[k + 1]
        # a random polynomial of total degree q in the physical coordinates
        c = rng.standard_normal((q + 1,) * d)

        def poly(X):
            out = np.zeros(X.shape[0])
            for idx in np.ndindex(*c.shape):
                if sum(idx) <= q:
                    out += c[idx] * np.prod(X ** np.array(idx), axis=1)
            return out
        lo = poly(cdgs[k + 1].nodes_phys().reshape(-1, d))
        hi = poly(cdgs[k].nodes_phys().reshape(-1, d))
        assert np.abs(H.Tb[k] @ lo - hi).max() <= 1e-12 * np.abs(hi).max()
        assert np.allclose(H.T[k].sum(axis=1), 1.0)  # partition of unity


@pytest.mark.parametrize("d", [2, 3])
def test_chain_and_jump_reach_the_same_p1_operator(d):
    # P1 is nested in P2 in P3: T_{3->2} T_{2->1} = T_{3->1}, so the p = 1
    # operator of the sequence 3, 2, 1 equals that of the single jump 3 -> 1
    m = _mesh(d, 5 if d == 2 else 2)
    cdgs = [CDG(m.coords, m.e2v, m.face_bc, q) for q in (3, 2, 1)]
    chain = HpHierarchy(cdgs, [])
    jump = HpHierarchy([cdgs[0], cdgs[2]], [])
    assert np.abs(chain.T[0] @ chain.T[1] - jump.T[0]).max() <= 1e-13
    A1c, A1j = chain.inner.A[0], jump.inner.A[0]
    assert abs(A1c - A1j).max() <= 1e-12 * abs(A1j).max()


def test_coarse_correction_annihilates_the_p1_space():
    # with an exact p = 1 solve (one level), the two-level error propagation
    # I - Tb (Tb^T A Tb)^{-1} Tb^T A vanishes on Tb y
    m, cdgs, parents = _hp(n=6, degrees=(3, 1), levels=1)
    H = HpHierarchy(cdgs, [])
    Tb = H.Tb[0]
    y = np.random.default_rng(2).standard_normal(Tb.shape[1])
    e = Tb @ y
    A = H.A0
    ec = e - Tb @ H.inner.vcycle(Tb.T @ (A @ e))
    assert np.linalg.norm(ec) <= 1e-10 * np.linalg.norm(e)


def test_p1_input_is_the_plain_hierarchy():
    # at p = 1 there is no p-level: the hierarchy and its V-cycle are those of
    # the plain agglomeration hierarchy
    m, cdgs, parents = _hp(n=8, degrees=(1,), levels=3)
    Hp = HpHierarchy(cdgs, parents)
    H = Hierarchy(cdgs[0], parents, coarsening="primal")
    assert not Hp.A
    for l in range(len(H.A)):
        assert abs(Hp.inner.A[l] - H.A[l]).max() <= 1e-13 * abs(H.A[l]).max()
    r = np.random.default_rng(1).standard_normal(H.A[0].shape[0])
    assert np.linalg.norm(Hp.vcycle(r) - H.vcycle(r)) <= 1e-13 * np.linalg.norm(H.vcycle(r))


@pytest.mark.parametrize("d,degrees", [(2, (3, 1)), (2, (3, 2, 1)), (3, (2, 1))])
def test_hp_preconditioned_solve(d, degrees):
    m, cdgs, parents = _hp(d=d, n=8 if d == 2 else 3, degrees=degrees, levels=3)
    H = HpHierarchy(cdgs, parents)
    cdg = cdgs[0]
    b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, d))
    x, it, res = fcg(H.A0, b, H.vcycle, tol=1e-12)
    ref = spl.spsolve(H.A0.tocsc(), b)
    assert res <= 1e-12 and it < 100
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
