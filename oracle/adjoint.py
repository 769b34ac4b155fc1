"""Adjoint gradients of the CDG Poisson solve (not part of the paper).

Forward: A(kappa) u = b with b = M0 f, A(kappa) = sum_e kappa_e A^(e)
(A^(e) the kappa-free operator hosted by element e).  Loss
L = 1/2 (u - u_t)^T M0 (u - u_t).  Since A is symmetric:

* lambda solves A lambda = dL/du = M0 (u - u_t);
* dL/dkappa_e = -lambda^T A^(e) u;
* dL/df = M0 lambda.
"""
import numpy as np
import scipy.sparse.linalg as spl


def loss(cdg, u, u_t):
    r = u - u_t
    return 0.5 * float(r @ (cdg.M0() @ r))


def grad_kappa(cdg, u, lam):
    """g_e = -lambda_loc^T A^(e) u_loc over e's hosted stencil."""
    npb = cdg.np
    g = np.zeros(cdg.N)
    for e, (elems, A, C, G) in enumerate(cdg.local):
        dofs = np.concatenate([np.arange(el * npb, (el + 1) * npb) for el in elems])
        g[e] = -lam[dofs] @ (A @ u[dofs])
    return g


def gradients_direct(cdg, kappa, f, u_t):
    """Solution, loss and both gradients with direct sparse solves."""
    A = cdg.A(kappa).tocsc()
    M0 = cdg.M0()
    u = spl.spsolve(A, M0 @ f)
    lam = spl.spsolve(A, M0 @ (u - u_t))
    return u, loss(cdg, u, u_t), grad_kappa(cdg, u, lam), M0 @ lam, lam


def fd_kappa_difference_form(cdg, kappa, u, u_t, e, h_rel=1e-6, solve=None):
    """Central difference of L in kappa_e written for the increment du:
    A(kappa +- h e_e) du = -+ h A^(e) u, dL = (u - u_t)^T M0 du + 1/2 du^T M0 du,
    FD = (dL_+ - dL_-) / (2 h), h = h_rel * kappa_e.  This avoids subtracting
    two nearly equal losses."""
    npb = cdg.np
    M0 = cdg.M0()
    h = h_rel * kappa[e]
    elems, Ae, _, _ = cdg.local[e]
    dofs = np.concatenate([np.arange(el * npb, (el + 1) * npb) for el in elems])
    Aeu = np.zeros_like(u)
    Aeu[dofs] = Ae @ u[dofs]
    out = []
    for s in (+1.0, -1.0):
        kp = kappa.copy()
        kp[e] += s * h
        rhs = -s * h * Aeu
        Ak = cdg.A(kp).tocsc()
        du = spl.spsolve(Ak, rhs) if solve is None else solve(Ak, rhs)
        out.append(float((u - u_t) @ (M0 @ du)) + 0.5 * float(du @ (M0 @ du)))
    return (out[0] - out[1]) / (2.0 * h)
