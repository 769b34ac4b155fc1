"""Compact DG discretisation of -div(kappa grad u) = f (Sec. 2).

Readings of the paper (each listed in the design notes):

* PDE: -div(kappa grad u) = f, kappa constant per element; the flux variable
  is q = kappa grad u.  With kappa = 1 this is the paper's first-order system
  (Sec. 2.2) with the sign its weak form (volume equation) carries.
* Switch and hosts (Sec. 2.2): on an interior facet f between K and K' with
  S_K^{K'} = -1, K is the host: it owns the boundary gradient
  q^f = kappa_K (grad u_K + r_f(w_f(u))), with the jump
  w_f(u) = u_{K'}|_f - u_K|_f, and u-hat on f is u_{K'}.  Dirichlet facets
  are hosted by their element with w_f(u) = g_D - u_K (g_D = 0 here).
  Neumann facets are not hosted (q-hat = g_N n, u-hat = u_h).
* Lifting r_f(w) in [P_p(K)]^d: (r_f(w), tau)_K = int_f w tau.n_K ds.
* Dirichlet penalty C_D = kappa_K gamma / h_avg, h_avg = mean over Dirichlet
  facets of the element height d |K| / |f|; no interior penalty.

Eliminating q with these fluxes gives, per host K (kappa-free part A^(K)):

  a^(K)(u, v) = (grad u, grad v)_K
      + sum_{f in H(K)} [ int_f w_f(u) dv/dn + int_f w_f(v) du/dn
                          + (r_f(w_f u), r_f(w_f v))_K ]
      + (gamma / h_avg) sum_{f Dirichlet} int_f u v,

and A = sum_K kappa_K A^(K) (the compact primal form, Sec. 2.3).

Flux form (Sec. 2.3): with the per-element gradient functional
  (G u)_K = ( grad u_K + sum_{f in H(K)} r_f(w_f u), tau )_K
(stored per component c as G^c, kappa-free; the paper's G is its negative)
and M = blockdiag(kappa_K^{-1} M_K), the LDG energy is G^T M^{-1} G and
C = A - G^T M^{-1} G is the Dirichlet penalty minus the cross-facet lifting
terms -kappa_K sum_{f != f' in H(K)} (r_f(w_f u), r_{f'}(w_{f'} v))_K;
C couples second neighbours exactly as stated in Sec. 4.2.
"""
import numpy as np
import scipy.sparse as sp

from .mesh import Topology
from .refelem import RefElement
from .switch import consistent_switch, natural_switch


class CDG:
    def __init__(self, coords, e2v, face_bc, p, gamma=1e4, switch="consistent",
                 switch_seed=None, host=None, subset=None):
        """subset: element ids whose rows of A are wanted (``A_rows``); only
        their element-local matrices and their neighbours' are formed, for
        sampled checks on large meshes.  None: all (every global matrix)."""
        coords = np.asarray(coords, dtype=np.float64)
        e2v = np.asarray(e2v, dtype=np.int64)
        face_bc = np.asarray(face_bc)
        self.coords, self.e2v, self.face_bc = coords, e2v, face_bc
        self.topo = topo = Topology(e2v, coords)
        self.d = d = topo.dim
        self.p = p
        self.ref = ref = RefElement(d, p)
        self.np = ref.np
        self.N = topo.n_elem
        self.gamma = gamma
        if host is not None:
            self.host = np.asarray(host, dtype=np.int64)
        elif switch == "consistent":
            self.host = consistent_switch(topo.interior, self.N)
        else:
            self.host = natural_switch(topo.interior, self.N, switch_seed)
        if subset is None:
            self.need = None
        else:
            need = set(int(e) for e in subset)
            for e in list(need):
                need.update(int(c) for c in topo.nbr[e] if c >= 0)
            self.need = sorted(need)
        self._geometry()
        self._assemble_local()

    # ------------------------------------------------------------------ geometry
    def _geometry(self):
        d, N = self.d, self.N
        X = self.coords[self.e2v]                     # [N, d+1, d]
        self.v0 = X[:, 0, :]
        self.J = np.stack([X[:, k + 1, :] - X[:, 0, :] for k in range(d)], axis=2)
        self.det = np.linalg.det(self.J)
        self.Jinv = np.linalg.inv(self.J)
        self.vol = self.det / (1 if d == 1 else (2 if d == 2 else 6))
        # facets: quadrature points, weights, outward normal, measure
        self.fq = {}
        elems = range(N) if self.need is None else sorted(set(self.need) | {e for (e, _) in self.topo.boundary})
        for e in elems:
            for i in range(d + 1):
                w = [X[e, k] for k in range(d + 1) if k != i]
                if d == 2:
                    t = w[1] - w[0]
                    meas = np.linalg.norm(t)
                    nrm = np.array([t[1], -t[0]]) / meas
                else:
                    cr = np.cross(w[1] - w[0], w[2] - w[0])
                    meas = 0.5 * np.linalg.norm(cr)
                    nrm = cr / np.linalg.norm(cr)
                if np.dot(X[e, i] - w[0], nrm) > 0:
                    nrm = -nrm
                s = self.ref.fqpts
                pts = w[0][None, :] + sum(s[:, k:k + 1] * (w[k + 1] - w[0])[None, :]
                                          for k in range(d - 1))
                wts = self.ref.fqwts * meas / (self.ref.fqwts.sum())
                self.fq[e, i] = (pts, wts, nrm, meas)
        dirichlet = [(e, i) for (e, i) in self.topo.boundary if self.face_bc[e, i] == 0]
        self.dirichlet = dirichlet
        if dirichlet:
            hs = [d * self.vol[e] / self.fq[e, i][3] for (e, i) in dirichlet]
            self.h_avg = float(np.mean(hs))
        else:
            self.h_avg = 1.0
        self.CD = self.gamma / self.h_avg

    def xi_of(self, e, x):
        return (x - self.v0[e][None, :]) @ self.Jinv[e].T

    def nodes_phys(self):
        """Physical coordinates [N, n_p, d] of the level-0 nodal points."""
        return self.v0[:, None, :] + np.einsum("eij,nj->eni", self.J, self.ref.nodes)

    def quad_phys(self):
        """Volume quadrature points [N, nq, d] and weights [N, nq]."""
        pts = self.v0[:, None, :] + np.einsum("eij,qj->eqi", self.J, self.ref.qpts)
        wts = self.det[:, None] * self.ref.qwts[None, :]
        return pts, wts

    # ------------------------------------------------------------- local forms
    def hosted_faces(self, e):
        """Hosted facets of e: list of (local facet i, neighbour or -1)."""
        out = []
        for i in range(self.d + 1):
            nb = self.topo.nbr[e, i]
            if nb >= 0:
                if self.host[self.topo.face_id[e, i]] == e:
                    out.append((i, int(nb)))
            elif self.face_bc[e, i] == 0:
                out.append((i, -1))
        return out

    def _assemble_local(self):
        ref, d, npb = self.ref, self.d, self.np
        phi_q = ref.eval(ref.qpts)                 # [nq, np]
        gref_q = ref.grad(ref.qpts)                # [nq, np, d]
        self.Mloc = np.zeros((self.N, npb, npb))
        self.local = [None] * self.N               # (dofs elems, A^(K), C^(K), G^c rows)
        for e in (range(self.N) if self.need is None else self.need):
            w = ref.qwts * self.det[e]
            M = (phi_q * w[:, None]).T @ phi_q
            self.Mloc[e] = M
            Minv = np.linalg.inv(M)
            g = np.einsum("qnk,kj->qnj", gref_q, self.Jinv[e])     # physical grads
            S = np.einsum("q,qik,qjk->ij", w, g, g)
            Dc = [np.einsum("q,qi,qj->ij", w, phi_q, g[:, :, c]) for c in range(d)]
            hf = self.hosted_faces(e)
            elems = [e] + [nb for (_, nb) in hf if nb >= 0]
            col = {el: k for k, el in enumerate(elems)}
            nl = len(elems) * npb
            A = np.zeros((nl, nl))
            C = np.zeros((nl, nl))
            G = [np.zeros((npb, nl)) for _ in range(d)]
            A[:npb, :npb] += S
            for c in range(d):
                G[c][:, :npb] += Dc[c]
            Fs = []
            for (i, nb) in hf:
                pts, wts, nrm, _ = self.fq[e, i]
                TK = ref.eval(self.xi_of(e, pts))                  # [nfq, np]
                gK = np.einsum("qnk,kj->qnj", ref.grad(self.xi_of(e, pts)), self.Jinv[e])
                DnK = gK @ nrm                                     # [nfq, np]
                Jm = np.zeros((len(wts), nl))                      # jump w_f(u) at face points
                Jm[:, :npb] -= TK
                if nb >= 0:
                    TN = ref.eval(self.xi_of(nb, pts))
                    Jm[:, col[nb] * npb:(col[nb] + 1) * npb] += TN
                t1 = np.zeros((nl, nl))
                t1[:npb, :] = DnK.T @ (wts[:, None] * Jm)           # int_f w(u) dv/dn
                A += t1 + t1.T
                F = TK.T @ (wts[:, None] * Jm)                      # [np, nl]
                A += F.T @ Minv @ F                                 # (r_f(w u), r_f(w v))_K
                Fs.append((F, nrm))
                for c in range(d):
                    G[c] += nrm[c] * F
                if nb < 0:
                    P = self.CD * (TK.T @ (wts[:, None] * TK))      # Dirichlet penalty
                    A[:npb, :npb] += P
                    C[:npb, :npb] += P
            for a, (Fa, na) in enumerate(Fs):
                for b, (Fb, nb_) in enumerate(Fs):
                    if a != b:
                        C -= np.dot(na, nb_) * (Fb.T @ Minv @ Fa)
            self.local[e] = (elems, A, C, G)

    # --------------------------------------------------------- global matrices
    def _scatter(self, which, kappa):
        assert self.need is None, "global matrices need all elements (subset=None)"
        npb = self.np
        rows, cols, vals = [], [], []
        for e, (elems, A, C, G) in enumerate(self.local):
            Mloc = A if which == "A" else C
            dofs = np.concatenate([np.arange(el * npb, (el + 1) * npb) for el in elems])
            R, Cc = np.meshgrid(dofs, dofs, indexing="ij")
            rows.append(R.ravel())
            cols.append(Cc.ravel())
            vals.append(kappa[e] * Mloc.ravel())
        n = self.N * npb
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))

    def A_rows(self, elems, kappa=None):
        """Rows of A = sum_K kappa_K A^(K) for the given elements, as
        {e: {c: n_p x n_p block}}: the hosts whose stencil holds e are e and
        its face neighbours."""
        kappa = np.ones(self.N) if kappa is None else np.asarray(kappa, dtype=np.float64)
        npb = self.np
        out = {}
        for e in elems:
            e = int(e)
            row = {}
            for K in [e] + [int(c) for c in self.topo.nbr[e] if c >= 0]:
                stencil, AK, _, _ = self.local[K]
                if e not in stencil:
                    continue
                a = stencil.index(e)
                for b, c in enumerate(stencil):
                    blk = kappa[K] * AK[a * npb:(a + 1) * npb, b * npb:(b + 1) * npb]
                    row[c] = row.get(c, 0.0) + blk
            out[e] = row
        return out

    def Cv(self, beta, vel):
        """Upwind DG convection matrix of beta v . grad u, v constant (the
        convection-diffusion example of Sec. 5):
            c(u, w) = sum_K [ (beta v . grad u_K, w_K)_K
                              - sum_{f in dK, v.n_K < 0} int_f beta (v.n_K) (u_K - u_ext) w_K ds ],
        u_ext the neighbour's trace on interior facets, 0 on Dirichlet facets
        and u_K on Neumann facets (no term).  kappa-free; CSR, float64."""
        ref, d, npb = self.ref, self.d, self.np
        v = np.asarray(vel, dtype=np.float64)[:d]
        phi_q = ref.eval(ref.qpts)
        gref_q = ref.grad(ref.qpts)
        rows, cols, vals = [], [], []

        def put(e, c, blk):
            R, Cc = np.meshgrid(np.arange(e * npb, (e + 1) * npb), np.arange(c * npb, (c + 1) * npb),
                                indexing="ij")
            rows.append(R.ravel())
            cols.append(Cc.ravel())
            vals.append(blk.ravel())

        nbr = {}
        for (a, ia, b, ib) in self.topo.interior:
            nbr[a, ia] = b
            nbr[b, ib] = a
        for e in range(self.N):
            w = ref.qwts * self.det[e]
            g = np.einsum("qnk,kj->qnj", gref_q, self.Jinv[e])
            vg = g @ v                                         # [nq, np]: v . grad phi_j
            put(e, e, beta * (phi_q * w[:, None]).T @ vg)
            for i in range(d + 1):
                pts, wts, nrm, _ = self.fq[e, i]
                vn = float(np.dot(v, nrm))
                if vn >= 0.0:
                    continue
                c = nbr.get((e, i), -1)
                if c < 0 and self.face_bc[e, i] != 0:
                    continue                                   # Neumann inflow: no jump
                TK = ref.eval(self.xi_of(e, pts))
                put(e, e, -beta * vn * (TK.T @ (wts[:, None] * TK)))
                if c >= 0:
                    TN = ref.eval(self.xi_of(c, pts))
                    put(e, c, beta * vn * (TK.T @ (wts[:, None] * TN)))
        n = self.N * npb
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    def A(self, kappa=None):
        """Primal CDG operator A = sum_K kappa_K A^(K) (CSR, float64)."""
        kappa = np.ones(self.N) if kappa is None else np.asarray(kappa, dtype=np.float64)
        return self._scatter("A", kappa)

    def C(self, kappa=None):
        """Flux-form C = A - G^T M^{-1} G, from its definition (penalty minus
        cross-facet lifting products)."""
        kappa = np.ones(self.N) if kappa is None else np.asarray(kappa, dtype=np.float64)
        return self._scatter("C", kappa)

    def G(self):
        """Flux-form gradient blocks, one CSR matrix per component (kappa-free)."""
        assert self.need is None, "global matrices need all elements (subset=None)"
        npb = self.np
        out = []
        for c in range(self.d):
            rows, cols, vals = [], [], []
            for e, (elems, A, C, G) in enumerate(self.local):
                dofs = np.concatenate([np.arange(el * npb, (el + 1) * npb) for el in elems])
                R, Cc = np.meshgrid(np.arange(e * npb, (e + 1) * npb), dofs, indexing="ij")
                rows.append(R.ravel())
                cols.append(Cc.ravel())
                vals.append(G[c].ravel())
            n = self.N * npb
            out.append(sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                     shape=(n, n)))
        return out

    def Mflux(self, kappa=None):
        """Flux-form mass blockdiag(kappa_K^{-1} M_K) (one component)."""
        kappa = np.ones(self.N) if kappa is None else np.asarray(kappa, dtype=np.float64)
        return sp.block_diag([self.Mloc[e] / kappa[e] for e in range(self.N)], format="csr")

    def M0(self):
        """Plain mass matrix blockdiag(M_K); the load vector is b = M0 f."""
        return sp.block_diag(list(self.Mloc), format="csr")

    def l2_error(self, uh, exact):
        """|| u_h - exact ||_{L2} by volume quadrature."""
        pts, wts = self.quad_phys()
        phi = self.ref.eval(self.ref.qpts)
        uq = np.einsum("qn,en->eq", phi, uh.reshape(self.N, self.np))
        return float(np.sqrt(np.sum(wts * (uq - exact(pts)) ** 2)))
