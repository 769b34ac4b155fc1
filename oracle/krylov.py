"""Outer Krylov solvers preconditioned by the V-cycle.

The paper wraps its V-cycle in right-preconditioned GMRES(50) (Sec. 4),
given here as ``gmres``; for the symmetric positive definite CDG Poisson
operator the oracle also has preconditioned CG and the flexible CG of Notay
(2000) truncated to one previous direction (FCG(1)), which also tolerates a
preconditioner that is not exactly linear or symmetric.  All start from
x = 0 and stop when the relative residual ||b - A x|| / ||b|| of the true
residual is <= tol.
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


def arnoldi(A, prec, v0, m):
    """m steps of the Arnoldi process on A B (B = prec) from v0, by modified
    Gram-Schmidt: returns V [m+1, n] with orthonormal rows, Z [m, n] with
    z_j = B v_j, and the (m+1) x m Hessenberg matrix H with A Z^T = V^T H.
    Stops early (returning fewer columns) on an exact breakdown."""
    n = len(v0)
    V = np.zeros((m + 1, n))
    Z = np.zeros((m, n))
    H = np.zeros((m + 1, m))
    V[0] = v0 / _norm(v0)
    for j in range(m):
        Z[j] = prec(V[j])
        w = A @ Z[j]
        for i in range(j + 1):
            H[i, j] = float(np.dot(w, V[i]))
            w = w - H[i, j] * V[i]
        H[j + 1, j] = _norm(w)
        if H[j + 1, j] == 0.0:
            return V[:j + 2], Z[:j + 1], H[:j + 2, :j + 1]
        V[j + 1] = w / H[j + 1, j]
    return V, Z, H


def gmres(A, b, prec, restart=50, tol=1e-10, maxiter=500, history=None):
    """Right-preconditioned restarted GMRES(m) (the paper's outer solver,
    Sec. 4; Saad & Schultz 1986), in the flexible form of Saad (1993) that
    keeps z_j = B v_j so that x = x_0 + Z y.  Each cycle: r = b - A x,
    Arnoldi on A B from r by modified Gram-Schmidt, the least-squares problem
    min || beta e_1 - H y || by Givens rotations, whose last residual entry is
    the residual estimate.  A cycle ends after m steps or when the estimate
    reaches tol; the run ends when the true relative residual is <= tol.
    history (a list) receives the relative residual estimate of every step."""
    x = np.zeros_like(b)
    nb = _norm(b)
    it = 0
    while it < maxiter:
        r = b - A @ x
        beta = _norm(r)
        if beta / nb <= tol:
            break
        m = restart
        V = np.zeros((m + 1, len(b)))
        Z = np.zeros((m, len(b)))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = prec(V[j])
            w = A @ Z[j]
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            H[j + 1, j] = _norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):  # earlier rotations on the new column
                hi, hi1 = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * hi + sn[i] * hi1
                H[i + 1, j] = -sn[i] * hi + cs[i] * hi1
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            if history is not None:
                history.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) / nb <= tol or it >= maxiter or H[j, j] == 0.0:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):  # back substitution on the rotated H
            y[i] = (g[i] - float(np.dot(H[i, i + 1:k], y[i + 1:k]))) / H[i, i]
        x = x + Z[:k].T @ y
    return x, it, _norm(b - A @ x) / nb


def refine(A, b, solve, rounds=2):
    """Iterative refinement (Wilkinson): x_0 = solve(b); then, `rounds` times,
    r = b - A x_k with the product and the difference in extended precision
    (numpy longdouble, a 64-bit significand on x86), d = solve(r rounded to
    float64), x_{k+1} = x_k + d.  The FP64 rounding of a plain residual, about
    eps || |A| |x| ||, limits an FP64 Krylov solve; here only the inner solves
    run in FP64, each on a residual that is smaller by their own reduction
    factor, so the error falls by that factor per round until the rounding of
    x itself.  Returns (x, relative extended-precision residual per round)."""
    Al = A.astype(np.longdouble)
    bl = np.asarray(b, dtype=np.longdouble)
    nb = float(np.sqrt(np.dot(bl, bl)))
    x = solve(b)
    res = []
    for _ in range(rounds):
        r = bl - Al @ np.asarray(x, dtype=np.longdouble)
        res.append(float(np.sqrt(np.dot(r, r))) / nb)
        x = x + solve(np.asarray(r, dtype=np.float64))
    r = bl - Al @ np.asarray(x, dtype=np.longdouble)
    res.append(float(np.sqrt(np.dot(r, r))) / nb)
    return x, res
