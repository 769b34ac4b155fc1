"""Pins for the oracle's CDG operator (Sec. 2) and its flux form."""
import numpy as np
import pytest
import scipy.sparse.linalg as spl

from oracle.cdg import CDG
from oracle.multigrid import block_diag_blocks, block_diag_matrix
from oracle.refelem import monomial_exponents
from workloads import mesh2d_jittered_delaunay, mesh3d_kuhn, exact_sine, source_sine


def _mesh(d, n, seed=1, bc=0):
    return mesh2d_jittered_delaunay(n, seed, bc=bc) if d == 2 else mesh3d_kuhn(n, seed, bc=bc)


@pytest.mark.parametrize("d,p", [(2, 1), (2, 3), (3, 2)])
def test_symmetric_and_positive_definite(d, p):
    m = _mesh(d, 5 if d == 2 else 2)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    A = cdg.A(np.random.default_rng(0).uniform(0.5, 2.0, cdg.N)).toarray()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A)[0] > 0


def _poly_and_neg_laplacian(d, p, rng):
    exps = monomial_exponents(d, p)
    c = rng.standard_normal(len(exps))

    def u(x):
        return sum(ci * np.prod([x[..., k] ** e[k] for k in range(d)], axis=0) for ci, e in zip(c, exps))

    def neg_lap(x):
        out = np.zeros(x.shape[:-1])
        for ci, e in zip(c, exps):
            for k in range(d):
                if e[k] >= 2:
                    term = ci * e[k] * (e[k] - 1)
                    for kk in range(d):
                        pw = e[kk] - (2 if kk == k else 0)
                        term = term * x[..., kk] ** pw
                    out -= term
        return out
    return u, neg_lap


@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (2, 3), (3, 2)])
def test_patch_test_interior_rows(d, p):
    # For kappa = 1 and a global polynomial pi of degree <= p, jumps vanish and
    # every row of an element with no boundary facet gives int_e (-Lap pi) v.
    m = _mesh(d, 6 if d == 2 else 3)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    u, neg_lap = _poly_and_neg_laplacian(d, p, np.random.default_rng(3))
    nodes = cdg.nodes_phys()
    Au = (cdg.A() @ u(nodes).ravel()).reshape(cdg.N, cdg.np)
    rhs = np.einsum("eij,ej->ei", cdg.Mloc, neg_lap(nodes))
    interior = np.all(cdg.topo.nbr >= 0, axis=1)
    assert interior.sum() > 0
    scale = np.abs(Au).max()
    assert np.abs(Au[interior] - rhs[interior]).max() <= 1e-11 * scale


@pytest.mark.parametrize("d,p", [(2, 2), (3, 1)])
def test_all_neumann_constant_in_kernel(d, p):
    m = _mesh(d, 4 if d == 2 else 2, bc=1)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    A = cdg.A()
    one = np.ones(A.shape[0])
    assert np.abs(A @ one).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_order_p_plus_one_2d(p):
    errs = []
    for n in (4, 8, 16):
        m = _mesh(2, n)
        cdg = CDG(m.coords, m.e2v, m.face_bc, p)
        b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, 2))
        u = spl.spsolve(cdg.A().tocsc(), b)
        errs.append(cdg.l2_error(u, exact_sine))
    rate = np.log2(errs[-2] / errs[-1])
    assert rate >= p + 0.8, (errs, rate)


def test_order_p_plus_one_3d_p2():
    errs = []
    for n in (2, 4):
        m = _mesh(3, n)
        cdg = CDG(m.coords, m.e2v, m.face_bc, 2)
        b = cdg.M0() @ source_sine(cdg.nodes_phys().reshape(-1, 3))
        u = spl.spsolve(cdg.A().tocsc(), b)
        errs.append(cdg.l2_error(u, exact_sine))
    assert np.log2(errs[0] / errs[1]) >= 2.8, errs


@pytest.mark.parametrize("d,p", [(2, 2), (3, 1)])
def test_flux_form_identity(d, p):
    # A (from the CDG form) = C (from its own definition) + sum_c G_c^T M^{-1} G_c
    # (the LDG energy of the gradient operator), Sec. 2.3.
    m = _mesh(d, 5 if d == 2 else 2)
    cdg = CDG(m.coords, m.e2v, m.face_bc, p)
    kappa = np.random.default_rng(1).uniform(0.3, 3.0, cdg.N)
    A, C, G, M = cdg.A(kappa), cdg.C(kappa), cdg.G(), cdg.Mflux(kappa)
    Minv = block_diag_matrix(np.linalg.inv(block_diag_blocks(M, cdg.np)))
    S = sum(g.T @ Minv @ g for g in G)
    assert abs(A - C - S).max() <= 1e-13 * abs(A).max()


def test_second_neighbour_rule_of_C():
    # Sec. 4.2: a block (K_i, K_n) of C between two distinct non-neighbours is
    # non-zero iff some K_j hosts both the K_i|K_j and the K_j|K_n facets.
    m = _mesh(2, 6)
    cdg = CDG(m.coords, m.e2v, m.face_bc, 1)
    C = cdg.C().tocsr()
    npb = cdg.np
    nbrs = [set(int(x) for x in row if x >= 0) for row in cdg.topo.nbr]
    expected = set()
    for j in range(cdg.N):
        hosted = [nb for (_, nb) in cdg.hosted_faces(j) if nb >= 0]
        for a in hosted:
            for b in hosted:
                if a != b and b not in nbrs[a]:
                    expected.add((a, b))
    found = set()
    Cb = C.tobsr(blocksize=(npb, npb))
    Cb.sort_indices()
    for i in range(cdg.N):
        for k in range(Cb.indptr[i], Cb.indptr[i + 1]):
            j = int(Cb.indices[k])
            if j != i and j not in nbrs[i] and np.abs(Cb.data[k]).max() > 1e-12 * abs(C).max():
                found.add((i, j))
    assert len(expected) > 0
    assert found == expected


def test_sampled_rows_equal_the_full_operator():
    # the subset mode used for sampled checks on large meshes forms the same
    # rows as the full assembly
    m = mesh2d_jittered_delaunay(9, 2)
    kappa = np.random.default_rng(3).uniform(0.5, 2.0, m.n_elem)
    full = CDG(m.coords, m.e2v, m.face_bc, 2)
    A = full.A(kappa).tocsr()
    sample = [0, 5, 17, 40, m.n_elem - 1]
    part = CDG(m.coords, m.e2v, m.face_bc, 2, subset=sample)
    rows = part.A_rows(sample, kappa)
    npb = full.np
    for e in sample:
        dense = A[e * npb:(e + 1) * npb, :].toarray()
        got = np.zeros_like(dense)
        for c, blk in rows[e].items():
            got[:, c * npb:(c + 1) * npb] = blk
        assert np.abs(got - dense).max() <= 1e-14 * np.abs(dense).max()
