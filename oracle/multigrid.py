"""Agglomerated hierarchy, transfers, operator coarsening and the V-cycle.

* Bases (Sec. 3.3): on every aggregate I the same-degree modal space P_p,
  spanned by monomials of (x - c_I) / h_I (c_I the centroid, h_I the largest
  distance from c_I to a vertex of I), orthonormalised in L2(I) by two passes
  of Cholesky.  Integrals over I sum the quadrature of its input-mesh
  elements (Sec. 3.3).
* Prolongation (Sec. 3.4): injection of the coarse polynomial into each
  child.  For an input-mesh child e (nodal basis) L_e[i, j] = psi_j^I(x_i^e);
  for an aggregate child e (orthonormal modal basis) L_e = (psi^e, psi^I)_e,
  which is the L2 projection and is exact because both spaces are P_p.
* Restriction of residuals: R = L^T on coefficient vectors (the adjoint of
  L for residuals viewed as functionals, Sec. 3.4).
* Flux coarsening (Sec. 4.1): M, G (per component) and C are each coarsened
  by Galerkin products L^T (.) L and A_{l+1} = C_{l+1} + G^T M^{-1} G with the
  coarse blocks.  Primal (RAT) coarsening A_{l+1} = L^T A_l L (Sec. 3.5) is
  kept for comparison.
* V-cycle (Alg. 3, read as a standard V(nu1, nu2) cycle over all levels):
  zero initial guess on every level, damped block-Jacobi sweeps
  x <- x + omega D^{-1} (b - A x), restriction of the residual, exact solve on
  the coarsest level (dense Cholesky), prolongation of the correction.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .refelem import monomial_exponents, monomials


def block_diag_blocks(A, npb):
    """Diagonal n_p x n_p blocks [N, n_p, n_p] of a sparse matrix."""
    A = A.tocsr()
    N = A.shape[0] // npb
    out = np.zeros((N, npb, npb))
    for e in range(N):
        out[e] = A[e * npb:(e + 1) * npb, e * npb:(e + 1) * npb].toarray()
    return out


def block_diag_matrix(blocks):
    return sp.block_diag(list(blocks), format="csr")


class Hierarchy:
    """Levels 0..L of an agglomerated CDG problem.

    parents: list of parent maps, parents[l][e] = aggregate at level l+1 of
    element e of level l.
    """

    def __init__(self, cdg, parents, kappa=None, coarsening="flux", A0=None):
        """A0: a given level-0 operator (e.g. diffusion plus convection, or its
        transpose) in place of cdg.A(kappa); primal coarsening only."""
        self.cdg = cdg
        self.d, self.p, self.np = cdg.d, cdg.p, cdg.np
        self.parents = [np.asarray(p, dtype=np.int64) for p in parents]
        self.L = len(parents)                      # index of the coarsest level
        self.kappa = np.ones(cdg.N) if kappa is None else np.asarray(kappa, dtype=np.float64)
        self.sizes = [cdg.N] + [int(p.max()) + 1 for p in self.parents]
        # input-mesh element -> aggregate id at each level
        anc = [np.arange(cdg.N)]
        for p in self.parents:
            anc.append(p[anc[-1]])
        self.anc = anc
        self._bases()
        self._transfers()
        self.coarsening = coarsening
        if A0 is not None and coarsening != "primal":
            raise ValueError("a given A0 is coarsened by the primal (Galerkin) rule only")
        self.A0_given = None if A0 is None else sp.csr_matrix(A0)
        self._operators()

    # -------------------------------------------------------------- bases
    def _bases(self):
        cdg = self.cdg
        self.qpts, self.qwts = cdg.quad_phys()     # [N0, nq, d], [N0, nq]
        self.exps = monomial_exponents(self.d, self.p)
        self.center, self.scale, self.coef = [None], [None], [None]
        for l in range(1, self.L + 1):
            nl = self.sizes[l]
            cen = np.zeros((nl, self.d))
            sca = np.zeros(nl)
            coef = np.zeros((nl, self.np, self.np))
            for I in range(nl):
                fine = np.nonzero(self.anc[l] == I)[0]
                x = self.qpts[fine].reshape(-1, self.d)
                w = self.qwts[fine].ravel()
                c = (w[:, None] * x).sum(axis=0) / w.sum()
                verts = np.unique(cdg.e2v[fine].ravel())
                h = np.max(np.linalg.norm(cdg.coords[verts] - c[None, :], axis=1))
                m = monomials((x - c) / h, self.exps)
                Cf = np.eye(self.np)
                for _ in range(2):                  # two Cholesky passes
                    psi = m @ Cf
                    gram = psi.T @ (w[:, None] * psi)
                    Lc = np.linalg.cholesky(gram)
                    Cf = Cf @ np.linalg.inv(Lc).T
                cen[I], sca[I], coef[I] = c, h, Cf
            self.center.append(cen)
            self.scale.append(sca)
            self.coef.append(coef)

    def basis_at(self, l, I, x):
        """Values [npts, n_p] of the level-l aggregate I's basis at points x."""
        m = monomials((x - self.center[l][I]) / self.scale[l][I], self.exps)
        return m @ self.coef[l][I]

    # ---------------------------------------------------------- transfers
    def _transfers(self):
        cdg = self.cdg
        nodes = cdg.nodes_phys()
        self.Lblocks = []                           # per level l: [N_l, n_p, n_p]
        self.P = []
        for l in range(self.L):
            par = self.parents[l]
            nl = self.sizes[l]
            blocks = np.zeros((nl, self.np, self.np))
            for e in range(nl):
                I = par[e]
                if l == 0:
                    blocks[e] = self.basis_at(l + 1, I, nodes[e])
                else:
                    fine = np.nonzero(self.anc[l] == e)[0]
                    x = self.qpts[fine].reshape(-1, self.d)
                    w = self.qwts[fine].ravel()
                    pe = self.basis_at(l, e, x)
                    pI = self.basis_at(l + 1, I, x)
                    blocks[e] = pe.T @ (w[:, None] * pI)
            self.Lblocks.append(blocks)
            rows, cols, vals = [], [], []
            for e in range(nl):
                R, C = np.meshgrid(np.arange(e * self.np, (e + 1) * self.np),
                                   np.arange(par[e] * self.np, (par[e] + 1) * self.np), indexing="ij")
                rows.append(R.ravel())
                cols.append(C.ravel())
                vals.append(blocks[e].ravel())
            self.P.append(sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                        shape=(nl * self.np, self.sizes[l + 1] * self.np)))

    # ---------------------------------------------------------- operators
    def _operators(self):
        cdg, k = self.cdg, self.kappa
        A0 = cdg.A(k) if self.A0_given is None else self.A0_given
        self.A = [A0]
        if self.coarsening == "flux":
            M = cdg.Mflux(k)
            G = cdg.G()
            C = cdg.C(k)
            self.Mf, self.Gf, self.Cf = [M], [G], [C]
            for l in range(self.L):
                P = self.P[l]
                M = (P.T @ M @ P).tocsr()
                G = [(P.T @ g @ P).tocsr() for g in G]
                C = (P.T @ C @ P).tocsr()
                Minv = block_diag_matrix(np.linalg.inv(block_diag_blocks(M, self.np)))
                A = C + sum((g.T @ Minv @ g) for g in G)
                self.Mf.append(M)
                self.Gf.append(G)
                self.Cf.append(C)
                self.A.append(A.tocsr())
        elif self.coarsening == "primal":
            for l in range(self.L):
                P = self.P[l]
                self.A.append((P.T @ self.A[-1] @ P).tocsr())
        else:
            raise ValueError(self.coarsening)
        self.Dinv = [np.linalg.inv(block_diag_blocks(A, self.np)) for A in self.A[:-1]]
        self.Dinv_mat = [block_diag_matrix(D) for D in self.Dinv]
        AL = self.A[-1].toarray()
        self.coarse_chol = self.coarse_lu = None
        if np.allclose(AL, AL.T, rtol=0, atol=1e-14 * np.abs(AL).max()):
            try:
                self.coarse_chol = sla.cho_factor(AL, lower=True)
            except np.linalg.LinAlgError:
                pass
        else:                                  # nonsymmetric (convection): LU
            self.coarse_lu = sla.lu_factor(AL)

    # ------------------------------------------------------------ V-cycle
    def vcycle(self, b, nu1=2, nu2=2, omega=0.7, level=0):
        """One V(nu1, nu2) cycle for A_level x = b from x = 0."""
        if level == self.L:
            if self.coarse_lu is not None:
                return sla.lu_solve(self.coarse_lu, b)
            return sla.cho_solve(self.coarse_chol, b)
        A, Dinv = self.A[level], self.Dinv_mat[level]
        x = np.zeros_like(b)
        for _ in range(nu1):
            x = x + omega * (Dinv @ (b - A @ x))
        r = b - A @ x
        xc = self.vcycle(self.P[level].T @ r, nu1, nu2, omega, level + 1)
        x = x + self.P[level] @ xc
        for _ in range(nu2):
            x = x + omega * (Dinv @ (b - A @ x))
        return x


class HpHierarchy:
    """hp-multigrid front end (Sec. 4, hp paragraph): p-multigrid on the fine
    mesh from degree p down to p = 1, then the agglomeration levels at p = 1.

    cdgs lists the CDG discretisations of the p-levels, of strictly
    decreasing degree and ending at p = 1: [p, p-1, ..., 1] for the standard
    p-multigrid sequence that lowers the degree by one per level, or [p, 1]
    for a single jump.  Level k carries the degree-p_k operator A_k with its
    block-Jacobi smoother.  The degree-p_{k+1} space is embedded element by
    element: the nodal basis of degree p_{k+1} on the reference simplex,
    evaluated at the degree-p_k nodes, gives T_k (n_{p_k} x n_{p_{k+1}}), the
    same for every element (both bases are nodal on the same reference
    element), and Tb_k = blockdiag(T_k).  The next operator is the Galerkin
    projection A_{k+1} = Tb_k^T A_k Tb_k; the p = 1 one is coarsened further
    by the agglomeration hierarchy at p = 1 (primal coarsening)."""

    def __init__(self, cdgs, parents, kappa=None):
        from .refelem import RefElement
        degs = [c.p for c in cdgs]
        assert degs[-1] == 1 and all(a > b for a, b in zip(degs, degs[1:]))
        self.cdgs = list(cdgs)
        cdg = cdgs[0]
        self.kappa = np.ones(cdg.N) if kappa is None else np.asarray(kappa, dtype=np.float64)
        N = cdg.N
        self.T, self.Tb, self.A, self.Dinv = [], [], [], []
        A = cdg.A(self.kappa).tocsr()
        for k in range(len(cdgs) - 1):
            T = RefElement(cdg.d, degs[k + 1]).eval(cdgs[k].ref.nodes)      # [n_pk, n_pk+1]
            Tb = sp.kron(sp.identity(N, format="csr"), sp.csr_matrix(T), format="csr")
            self.A.append(A)
            self.Dinv.append(block_diag_matrix(np.linalg.inv(block_diag_blocks(A, cdgs[k].np))))
            self.T.append(T)
            self.Tb.append(Tb)
            A = (Tb.T @ A @ Tb).tocsr()
        self.A0 = self.A[0] if self.A else A
        self.inner = Hierarchy(cdgs[-1], parents, kappa=self.kappa, coarsening="primal", A0=A)

    def vcycle(self, b, nu1=2, nu2=2, omega=0.7, k=0):
        """One V(nu1, nu2) cycle for A_k x = b from x = 0; below the last
        p-level the coarse correction is the p = 1 hierarchy's V-cycle."""
        if k == len(self.A):
            return self.inner.vcycle(b, nu1, nu2, omega)
        A, Dinv, Tb = self.A[k], self.Dinv[k], self.Tb[k]
        x = np.zeros_like(b)
        for _ in range(nu1):
            x = x + omega * (Dinv @ (b - A @ x))
        r = b - A @ x
        x = x + Tb @ self.vcycle(Tb.T @ r, nu1, nu2, omega, k + 1)
        for _ in range(nu2):
            x = x + omega * (Dinv @ (b - A @ x))
        return x
