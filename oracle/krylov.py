"""Outer Krylov solvers preconditioned by the V-cycle.

The paper wraps its V-cycle in right-preconditioned GMRES(50) (Sec. 4); for
the symmetric positive definite CDG Poisson operator this oracle uses
preconditioned CG and the flexible CG of Notay (2000) truncated to one
previous direction (FCG(1)), which also tolerates a preconditioner that is
not exactly linear or symmetric.  Both start from x = 0 and stop when the
relative residual ||b - A x|| / ||b|| of the true residual is <= tol.
"""
import numpy as np


def _norm(v):
    return float(np.sqrt(np.dot(v, v)))


def pcg(A, b, prec, tol=1e-10, maxiter=500, history=None):
    """Preconditioned CG with beta = (z_k, r_k) / (z_{k-1}, r_{k-1})."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = _norm(b)
    p = None
    rz_old = None
    it = 0
    while it < maxiter:
        z = prec(r)
        rz = float(np.dot(z, r))
        p = z.copy() if p is None else z + (rz / rz_old) * p
        q = A @ p
        alpha = rz / float(np.dot(p, q))
        x = x + alpha * p
        r = r - alpha * q
        rz_old = rz
        it += 1
        if history is not None:
            history.append(x.copy())
        if _norm(r) / nb <= tol:
            rt = b - A @ x
            if _norm(rt) / nb <= tol:
                break
            r = rt
    return x, it, _norm(b - A @ x) / nb


def fcg(A, b, prec, tol=1e-10, maxiter=500, history=None):
    """Flexible CG, FCG(1): p_k = z_k - [(z_k, q_{k-1}) / (p_{k-1}, q_{k-1})] p_{k-1},
    q_k = A p_k, alpha_k = (p_k, r_k) / (p_k, q_k)."""
    x = np.zeros_like(b)
    r = b.copy()
    nb = _norm(b)
    p_old = q_old = None
    pq_old = None
    it = 0
    while it < maxiter:
        z = prec(r)
        if p_old is None:
            p = z.copy()
        else:
            beta = float(np.dot(z, q_old)) / pq_old
            p = z - beta * p_old
        q = A @ p
        pq = float(np.dot(p, q))
        alpha = float(np.dot(p, r)) / pq
        x = x + alpha * p
        r = r - alpha * q
        p_old, q_old, pq_old = p, q, pq
        it += 1
        if history is not None:
            history.append(x.copy())
        if _norm(r) / nb <= tol:
            rt = b - A @ x
            if _norm(rt) / nb <= tol:
                break
            r = rt
    return x, it, _norm(b - A @ x) / nb
