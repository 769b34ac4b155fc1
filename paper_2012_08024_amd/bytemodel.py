"""Algorithmic byte models of the solver's kernels: what each kernel must
read and write once (operator values, indices, vectors), nothing for
re-reads.  They turn measured kernel durations into bandwidth figures."""


def facet_nodes(dim, npb):
    """Nodes of the degree-p simplex on one facet: the nonzero rows or columns
    of a level-0 off-diagonal block in facet-trace form."""
    p = {3: 1, 6: 2, 10: 3} if dim == 2 else {4: 1, 10: 2, 20: 3}
    q = p[npb]
    return q + 1 if dim == 2 else (q + 1) * (q + 2) // 2


def row_block(npb, sym=True):
    """Values per level-0 per-row block (D^{-1}, a diagonal block): its upper
    triangle for the symmetric operator, else the whole block."""
    return npb * (npb + 1) // 2 if sym else npb * npb


def smoother_bytes(nnzb0, n0, npb, s, nfn, nf, sym=True):
    """Algorithmic HBM bytes of one level-0 damped block-Jacobi sweep
    x <- (1 - omega) x + omega D^{-1} (b - A_off x) on the facet-trace form:
    the off-diagonal blocks' n_p x n_fn stored values, their column indices and
    kinds (one int32 and one byte per facet slot), D^{-1}, and b, x read, x
    written."""
    off = nnzb0 - n0
    return off * npb * nfn * s + 5 * n0 * nf + n0 * row_block(npb, sym) * s + 3 * n0 * npb * s


def transfer0_bytes(n0, n1, npb, s, nf):
    """What the level-0 transfers read to form L_e on the fly: each element's
    affine map into its parent's scaled coordinates (d + d^2 values), its
    parent index, and the parents' monomial coefficients (n_p^2 values per
    aggregate, read once)."""
    d = nf - 1
    return n0 * (d + d * d) * s + 4 * n0 + n1 * npb * npb * s


def restrict_bytes(nnzb0, n0, npb, s, nfn, nf, sym=True, n1=0):
    """Level-0 residual + restriction L_e^T (b - A_rr x - A_off x): the
    off-diagonal values, indices and kinds, the diagonal blocks, the transfer
    data, b and x read, the restricted residual written."""
    off = nnzb0 - n0
    return (off * npb * nfn * s + 5 * n0 * nf + n0 * row_block(npb, sym) * s
            + transfer0_bytes(n0, n1, npb, s, nf) + 3 * n0 * npb * s)


def spmv_bytes(nnzb0, n0, npb, nfn, nf, sym=True):
    """Outer FP64 q = A_0 p with (p,q), (p,r): the diagonal blocks, the
    off-diagonal blocks' facet-trace values, indices and kinds, p, r read, q
    written."""
    off = nnzb0 - n0
    return n0 * row_block(npb, sym) * 8 + off * npb * nfn * 8 + 5 * n0 * nf + 3 * n0 * npb * 8


def iteration_bytes(sizes, nnzb, npb, nfn, nf, nu1=2, nu2=2, s=4, sym=True):
    """Algorithmic bytes of one FCG(1) iteration with a V(nu1, nu2) cycle in
    precision s (bytes) and the FP64 outer loop, per level: what each kernel
    must read and write once (operator blocks, indices, vectors), nothing for
    re-reads.  Level 0 runs on the facet-trace form with D^{-1} (per-row
    blocks as upper triangles when sym, the operator being symmetric) and forms
    its transfers L_e from the element maps and parent coefficients; the coarse
    levels on D^{-1}-prescaled strips.  The first pre-sweep of every level is
    fused with forming D^{-1} b (no operator read); the last post-sweep of
    level 0 also reads q for the fused (z, q) dot."""
    L = len(sizes) - 1
    n = [int(x) for x in sizes]
    nz = [int(x) for x in nnzb]
    p2 = npb * npb
    out = {}
    for l in range(L + 1):
        if l == L:  # coarsest: children sums, then the dense inverse product
            ld = -(-n[l] * npb // 64) * 64
            b = n[l - 1] * npb * s + 4 * n[l] + n[l] * npb * s if l > 0 else n[l] * npb * 8
            b += n[l] * npb * ld * s + ld * s + n[l] * npb * s
            out["level%d" % l] = b
            break
        prolong = n[l] * p2 * s + 2 * n[l] * npb * s + 4 * n[l] + n[l + 1] * npb * s
        if l == 0:
            prolong = transfer0_bytes(n[0], n[1], npb, s, nf) + 2 * n[0] * npb * s + n[1] * npb * s
            sweep = smoother_bytes(nz[0], n[0], npb, s, nfn, nf, sym)
            entry = n[0] * npb * 8 + n[0] * row_block(npb, sym) * s + 2 * n[0] * npb * s
            restrict = restrict_bytes(nz[0], n[0], npb, s, nfn, nf, sym, n[1]) + n[0] * npb * s
            b = entry + (nu1 - 1) * sweep + restrict + prolong + nu2 * sweep + n[0] * npb * 8
        else:
            off = nz[l] - n[l]
            sweep = off * p2 * s + 4 * off + 3 * n[l] * npb * s + 8 * n[l]
            entry = n[l - 1] * npb * s + 4 * n[l] + n[l] * p2 * s + 2 * n[l] * npb * s
            restrict = sweep + n[l] * p2 * s
            b = entry + (nu1 - 1) * sweep + restrict + prolong + nu2 * sweep
        out["level%d" % l] = b
    m = n[0] * npb
    out["outer"] = (m * s + 2 * m * 8) + spmv_bytes(nz[0], n[0], npb, nfn, nf, sym) + 6 * m * 8
    out["total"] = sum(out.values())
    return out
