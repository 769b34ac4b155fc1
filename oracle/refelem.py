"""Reference simplex: quadrature, monomials, equispaced nodes, nodal P_p basis.

The DG spaces are P_p per element (Sec. 2.2).  On the input mesh the
oracle uses the nodal Lagrange basis on the equispaced nodes of the reference
simplex; the node order is part of the library's interface:

* d=2: for j in 0..p, for i in 0..p-j: (i/p, j/p)
* d=3: for k in 0..p, for j in 0..p-k, for i in 0..p-j-k: (i/p, j/p, k/p)

Reference simplex vertices: origin and the unit vectors; the physical
element maps x = v0 + J xi with J = [v1-v0, ..., vd-v0].
"""
from math import comb

import numpy as np


def gauss_legendre01(n):
    """n-point Gauss-Legendre rule on [0,1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def simplex_quadrature(d, n):
    """Collapsed (conical) product of n-point Gauss-Legendre rules.

    d=2: x = a(1-b), y = b, Jacobian (1-b); exact to degree 2n-2.
    d=3: x = a(1-b)(1-c), y = b(1-c), z = c, Jacobian (1-b)(1-c)^2; exact to
    degree 2n-3.  d=1: plain Gauss-Legendre on [0,1].
    """
    g, w = gauss_legendre01(n)
    if d == 1:
        return g[:, None].copy(), w.copy()
    if d == 2:
        pts, wts = [], []
        for ia in range(n):
            for ib in range(n):
                a, b = g[ia], g[ib]
                pts.append((a * (1 - b), b))
                wts.append(w[ia] * w[ib] * (1 - b))
        return np.array(pts), np.array(wts)
    if d == 3:
        pts, wts = [], []
        for ia in range(n):
            for ib in range(n):
                for ic in range(n):
                    a, b, c = g[ia], g[ib], g[ic]
                    pts.append((a * (1 - b) * (1 - c), b * (1 - c), c))
                    wts.append(w[ia] * w[ib] * w[ic] * (1 - b) * (1 - c) ** 2)
        return np.array(pts), np.array(wts)
    raise ValueError(d)


def n_basis(d, p):
    return comb(p + d, d)


def monomial_exponents(d, p):
    """Exponent tuples of the monomials of total degree <= p, by degree."""
    out = []
    for deg in range(p + 1):
        if d == 1:
            out.append((deg,))
        elif d == 2:
            for b in range(deg + 1):
                out.append((deg - b, b))
        else:
            for c in range(deg + 1):
                for b in range(deg - c + 1):
                    out.append((deg - b - c, b, c))
    return out


def monomials(x, exps):
    """Values [npts, nmono] of x^alpha."""
    x = np.atleast_2d(x)
    out = np.ones((x.shape[0], len(exps)))
    for m, e in enumerate(exps):
        for k, ek in enumerate(e):
            if ek:
                out[:, m] *= x[:, k] ** ek
    return out


def monomial_grads(x, exps):
    """Gradients [npts, nmono, d] of x^alpha."""
    x = np.atleast_2d(x)
    d = x.shape[1]
    out = np.zeros((x.shape[0], len(exps), d))
    for m, e in enumerate(exps):
        for k in range(d):
            if e[k] == 0:
                continue
            val = e[k] * np.ones(x.shape[0])
            for kk in range(d):
                pw = e[kk] - (1 if kk == k else 0)
                if pw:
                    val = val * x[:, kk] ** pw
            out[:, m, k] = val
    return out


def equispaced_nodes(d, p):
    pts = []
    if d == 2:
        for j in range(p + 1):
            for i in range(p + 1 - j):
                pts.append((i / p, j / p))
    elif d == 3:
        for k in range(p + 1):
            for j in range(p + 1 - k):
                for i in range(p + 1 - j - k):
                    pts.append((i / p, j / p, k / p))
    else:
        raise ValueError(d)
    return np.array(pts, dtype=np.float64)


class RefElement:
    """Nodal Lagrange P_p basis on the reference simplex.

    phi_n(xi) = sum_m C[m, n] xi^alpha_m with C = V^{-1}, V[i, m] = node_i^alpha_m,
    so that phi_n(node_i) = delta_{in}.
    """

    def __init__(self, d, p, nquad=None):
        self.d, self.p = d, p
        self.exps = monomial_exponents(d, p)
        self.nodes = equispaced_nodes(d, p)
        self.np = len(self.exps)
        V = monomials(self.nodes, self.exps)
        self.C = np.linalg.inv(V)
        nq = (p + 2) if nquad is None else nquad
        self.qpts, self.qwts = simplex_quadrature(d, nq)
        self.fqpts, self.fqwts = simplex_quadrature(d - 1, nq)

    def eval(self, xi):
        return monomials(xi, self.exps) @ self.C

    def grad(self, xi):
        g = monomial_grads(xi, self.exps)  # [npts, nmono, d]
        return np.einsum("qmk,mn->qnk", g, self.C)
