// Symbolic plans of the flux-form coarsening (Sec. 4.1), host side.
//
// The flux form of level l has the block-diagonal mass M_l (one n_p block per
// element and component), the gradient G_l (d component matrices) and
// C_l = A_l - G_l^T M_l^{-1} G_l.  Galerkin coarsening of each block with
// L_q = I_d (x) L and the Schur complement give
//     A_{l+1} = L^T C_l L + G_{l+1}^T M_{l+1}^{-1} G_{l+1}
//             = L^T A_l L - X^T M_l^{-1} X + Y^T M_{l+1}^{-1} Y,
// with X = G_l L (level-l rows, level-(l+1) columns), Y = L_q^T X = G_{l+1} and
// M_{l+1} = L_q^T M_l L_q.  The second line needs no explicit C_l; it is the
// same matrix up to rounding.  This file builds, for each output block, the
// ordered list of terms P^T Q R that the device sums (fixed order).
#include <algorithm>
#include <map>

#include "internal.hpp"

namespace cdg {

namespace {
OpRef op(OpKind k, int64_t idx, int comp = 0) { return OpRef{(int8_t)k, (int8_t)comp, idx}; }
const OpRef NONE{OP_NONE, 0, 0};
}  // namespace

// G_0 pattern (self + neighbours across hosted interior facets, local facet
// order) and its block-major values, component-major.
void flux_g0(Problem& P) {
  const Topology& T = P.topo;
  const Level& L0 = P.lv[0];
  const int nf = P.nf, W0 = nf + 1, np2 = P.np * P.np, d = P.d;
  FluxPlan& F = P.fp[0];
  F.g_ptr.assign(P.N0 + 1, 0);
  F.g_col.clear();
  std::vector<int32_t> slot;
  for (int64_t k = 0; k < P.N0; ++k) {
    const int64_t e = L0.perm[k];
    F.g_col.push_back((int32_t)k);
    slot.push_back(0);
    for (int i = 0; i < nf; ++i) {
      const int32_t nb = T.nbr[e * nf + i];
      if (nb >= 0 && T.hosted[e * nf + i]) {
        F.g_col.push_back(L0.iperm[nb]);
        slot.push_back(i + 1);
      }
    }
    F.g_ptr[k + 1] = (int64_t)F.g_col.size();
  }
  const int64_t nG = (int64_t)F.g_col.size();
  P.G0.assign((size_t)d * nG * np2, 0.0);
  for (int c = 0; c < d; ++c)
    for (int64_t k = 0; k < P.N0; ++k)
      for (int64_t q = F.g_ptr[k]; q < F.g_ptr[k + 1]; ++q) {
        const double* src = &P.Gblk[(((size_t)c * P.N0 + k) * W0 + slot[q]) * np2];
        std::copy(src, src + np2, &P.G0[((size_t)c * nG + q) * np2]);
      }
}

// X, Y and M_{l+1} plans for level l -> l+1 and the Schur-term targets; adds
// the columns of the Schur terms to the coarse rows.
void flux_level_symbolic(Problem& P, int l, std::vector<std::vector<int32_t>>& rows,
                         std::vector<std::pair<std::pair<int32_t, int32_t>, TPTerm>>& sterms) {
  const Level &f = P.lv[l], &c = P.lv[l + 1];
  const int d = P.d;
  FluxPlan& F = P.fp[l];
  if (l > 0) {  // G_l = Y of the previous level
    const FluxPlan& Fp = P.fp[l - 1];
    F.g_ptr = Fp.y_ptr;
    F.g_col = Fp.y_col;
  }
  const int64_t nG = (int64_t)F.g_col.size();
  // X pattern
  F.x_ptr.assign(f.n + 1, 0);
  F.x_col.clear();
  for (int64_t k = 0; k < f.n; ++k) {
    std::vector<int32_t> cols;
    for (int64_t q = F.g_ptr[k]; q < F.g_ptr[k + 1]; ++q) cols.push_back(f.parent[F.g_col[q]]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    F.x_col.insert(F.x_col.end(), cols.begin(), cols.end());
    F.x_ptr[k + 1] = (int64_t)F.x_col.size();
  }
  const int64_t nX = (int64_t)F.x_col.size();
  // X^c(k, t) = sum_{w: parent(gcol) = xcol(t)} G^c(k, w) L_{gcol}
  F.xp_ptr.assign((size_t)d * nX + 1, 0);
  F.xp.clear();
  for (int cc = 0; cc < d; ++cc)
    for (int64_t k = 0; k < f.n; ++k)
      for (int64_t t = F.x_ptr[k]; t < F.x_ptr[k + 1]; ++t) {
        for (int64_t q = F.g_ptr[k]; q < F.g_ptr[k + 1]; ++q)
          if (f.parent[F.g_col[q]] == F.x_col[t])
            F.xp.push_back(TPTerm{NONE, op(OP_G, q, cc), op(OP_L, F.g_col[q]), 1.0});
        F.xp_ptr[(size_t)cc * nX + t + 1] = (int64_t)F.xp.size();
      }
  // Y pattern (coarse rows J): union of the children's X columns
  F.y_ptr.assign(c.n + 1, 0);
  F.y_col.clear();
  for (int64_t J = 0; J < c.n; ++J) {
    std::vector<int32_t> cols;
    for (int64_t k = c.child_start[J]; k < c.child_start[J + 1]; ++k)
      for (int64_t t = F.x_ptr[k]; t < F.x_ptr[k + 1]; ++t) cols.push_back(F.x_col[t]);
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
    F.y_col.insert(F.y_col.end(), cols.begin(), cols.end());
    F.y_ptr[J + 1] = (int64_t)F.y_col.size();
  }
  const int64_t nY = (int64_t)F.y_col.size();
  // Y^c(J, u) = sum_{k in J, t: xcol = ycol(u)} L_k^T X^c(k, t)
  F.yp_ptr.assign((size_t)d * nY + 1, 0);
  F.yp.clear();
  for (int cc = 0; cc < d; ++cc)
    for (int64_t J = 0; J < c.n; ++J)
      for (int64_t u = F.y_ptr[J]; u < F.y_ptr[J + 1]; ++u) {
        for (int64_t k = c.child_start[J]; k < c.child_start[J + 1]; ++k)
          for (int64_t t = F.x_ptr[k]; t < F.x_ptr[k + 1]; ++t)
            if (F.x_col[t] == F.y_col[u]) F.yp.push_back(TPTerm{op(OP_L, k), op(OP_X, t, cc), NONE, 1.0});
        F.yp_ptr[(size_t)cc * nY + u + 1] = (int64_t)F.yp.size();
      }
  // M_{l+1}(J) = sum_{k in J} L_k^T M_l(k) L_k
  F.mp_ptr.assign(c.n + 1, 0);
  F.mp.clear();
  for (int64_t J = 0; J < c.n; ++J) {
    for (int64_t k = c.child_start[J]; k < c.child_start[J + 1]; ++k)
      F.mp.push_back(TPTerm{op(OP_L, k), op(OP_M, k), op(OP_L, k), 1.0});
    F.mp_ptr[J + 1] = (int64_t)F.mp.size();
  }
  // Schur terms and their columns
  sterms.clear();
  for (int64_t k = 0; k < f.n; ++k)
    for (int cc = 0; cc < d; ++cc)
      for (int64_t a = F.x_ptr[k]; a < F.x_ptr[k + 1]; ++a)
        for (int64_t b = F.x_ptr[k]; b < F.x_ptr[k + 1]; ++b)
          sterms.push_back({{F.x_col[a], F.x_col[b]},
                            TPTerm{op(OP_X, a, cc), op(OP_MINV, k), op(OP_X, b, cc), -1.0}});
  for (int64_t J = 0; J < c.n; ++J)
    for (int cc = 0; cc < d; ++cc)
      for (int64_t a = F.y_ptr[J]; a < F.y_ptr[J + 1]; ++a)
        for (int64_t b = F.y_ptr[J]; b < F.y_ptr[J + 1]; ++b)
          sterms.push_back({{F.y_col[a], F.y_col[b]},
                            TPTerm{op(OP_Y, a, cc), op(OP_MINVC, J), op(OP_Y, b, cc), 1.0}});
  for (auto& st : sterms) rows[st.first.first].push_back(st.first.second);
  (void)nG;
}

// bucket the Schur terms by the final A_{l+1} block id (generation order kept)
void flux_level_schur(Problem& P, int l, const std::vector<std::vector<int32_t>>& rows,
                      std::vector<std::pair<std::pair<int32_t, int32_t>, TPTerm>>& sterms) {
  const Level& c = P.lv[l + 1];
  FluxPlan& F = P.fp[l];
  auto blk = [&](int32_t I, int32_t N) {
    const auto& row = rows[I];
    const int t = (N == I) ? 0 : (int)(std::lower_bound(row.begin() + 1, row.end(), N) - row.begin());
    return c.row_blk[I] + t;
  };
  F.sp_ptr.assign(c.nnzb + 1, 0);
  for (auto& st : sterms) F.sp_ptr[blk(st.first.first, st.first.second) + 1]++;
  for (int64_t b = 0; b < c.nnzb; ++b) F.sp_ptr[b + 1] += F.sp_ptr[b];
  std::vector<int64_t> fill(F.sp_ptr.begin(), F.sp_ptr.end() - 1);
  F.sp.resize(sterms.size());
  for (auto& st : sterms) F.sp[fill[blk(st.first.first, st.first.second)]++] = st.second;
  std::vector<std::pair<std::pair<int32_t, int32_t>, TPTerm>>().swap(sterms);
}

}  // namespace cdg
