"""Pins for the oracle's reference element and quadrature."""
from math import factorial

import numpy as np
import pytest

from oracle.refelem import RefElement, simplex_quadrature, monomial_exponents, monomials


@pytest.mark.parametrize("d", [2, 3])
def test_quadrature_monomials_closed_form(d):
    # Integral of x^a y^b (z^c) over the reference simplex:
    # a! b! c! / (a + b + c + d)!  (Dirichlet / Eisenberg-Malvern formula).
    n = 5
    pts, wts = simplex_quadrature(d, n)
    exact_deg = 2 * n - 2 if d == 2 else 2 * n - 3
    for e in monomial_exponents(d, exact_deg):
        num = np.prod([factorial(k) for k in e])
        ref = num / factorial(sum(e) + d)
        val = float(wts @ monomials(pts, [e])[:, 0])
        assert abs(val - ref) <= 1e-14 * max(1.0, abs(ref)) + 1e-16


def test_p1_mass_matrix_closed_form():
    # P1 mass matrix on a triangle = |K|/12 [[2,1,1],[1,2,1],[1,1,2]].
    from oracle.cdg import CDG
    coords = np.array([[0.1, 0.2], [1.3, 0.4], [0.5, 1.7]])
    e2v = np.array([[0, 1, 2]])
    cdg = CDG(coords, e2v, np.zeros((1, 3), dtype=np.int8), 1)
    area = cdg.vol[0]
    ref = area / 12.0 * np.array([[2, 1, 1], [1, 2, 1], [1, 1, 2]])
    assert np.allclose(cdg.Mloc[0], ref, rtol=0, atol=1e-15)


def test_p1_tet_mass_matrix_closed_form():
    # P1 mass matrix on a tetrahedron = |K|/20 (1 + delta_ij).
    from oracle.cdg import CDG
    coords = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.1, 0.1], [0.1, 0.3, 0.9]])
    e2v = np.array([[0, 1, 2, 3]])
    cdg = CDG(coords, e2v, np.zeros((1, 4), dtype=np.int8), 1)
    ref = cdg.vol[0] / 20.0 * (np.ones((4, 4)) + np.eye(4))
    assert np.allclose(cdg.Mloc[0], ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("d,p", [(2, 1), (2, 2), (2, 3), (3, 1), (3, 2), (3, 3)])
def test_nodal_basis_is_lagrange(d, p):
    ref = RefElement(d, p)
    V = ref.eval(ref.nodes)
    assert np.allclose(V, np.eye(ref.np), atol=1e-12)
    # partition of unity and exact gradients of the coordinate functions
    xi = np.random.default_rng(0).uniform(0, 1.0 / d, size=(7, d))
    assert np.allclose(ref.eval(xi).sum(axis=1), 1.0, atol=1e-13)
    g = ref.grad(xi)  # sum_n node_n[k] grad phi_n = e_k
    for k in range(d):
        assert np.allclose(np.einsum("n,qnj->qj", ref.nodes[:, k], g), np.eye(d)[k], atol=1e-12)
