// Host-only reference evaluation of the level operators from the library's own
// setup data (kappa-free blocks, ordering, transfer blocks, Galerkin plans).
// Used by CPU tests to check the host half of the setup without a GPU; the
// device path computes the same quantities with the setup kernels.
#include <algorithm>

#include "internal.hpp"

using namespace cdg;

namespace {
// dense helpers on row-major n x n blocks
void invert_spd_like(int n, double* a) {
  // Gauss-Jordan without pivoting (blocks are symmetric positive definite)
  for (int k = 0; k < n; ++k) {
    const double p = a[k * n + k];
    a[k * n + k] = 1.0;
    for (int j = 0; j < n; ++j) a[k * n + j] /= p;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = a[i * n + k];
      a[i * n + k] = 0.0;
      for (int j = 0; j < n; ++j) a[i * n + j] -= f * a[k * n + j];
    }
  }
}

// out += sign * P^T Q R with P, R possibly identity (nullptr)
void tp_acc(int n, const double* P, const double* Q, const double* R, double sign, double* out) {
  std::vector<double> T(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      if (R)
        for (int m = 0; m < n; ++m) s += Q[i * n + m] * R[m * n + j];
      else
        s = Q[i * n + j];
      T[i * n + j] = s;
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      if (P)
        for (int m = 0; m < n; ++m) s += P[m * n + i] * T[m * n + j];
      else
        s = T[i * n + j];
      out[i * n + j] += sign * s;
    }
}
}  // namespace

extern "C" int cdgmg_debug_host_operator(const cdgmg_mesh* mesh, int p, const double* kappa,
                                         const cdgmg_hierarchy* hier, const cdgmg_options* opts, int level,
                                         int64_t* nnzb, int64_t* row_ptr, int32_t* cols, double* blocks) {
  set_error("");
  if (!mesh || !hier || !kappa || !nnzb || level < 0 || level >= hier->n_levels) {
    set_error("debug_host_operator: invalid argument");
    return CDGMG_ERR_ARG;
  }
  cdgmg_options o;
  if (opts)
    o = *opts;
  else
    cdgmg_default_options(&o);
  int rc = check_options(o);
  if (rc) return rc;
  Problem P;
  rc = build_problem(*mesh, p, *hier, o, P);
  if (rc) return rc;
  const int np = P.np, np2 = np * np, W0 = P.nf + 1;
  const Level& H = P.lv[level];
  *nnzb = H.nnzb;
  if (!row_ptr || !cols || !blocks) return CDGMG_OK;
  // level 0 in row-major [row][slot] blocks, internal order
  const Level& H0 = P.lv[0];
  std::vector<double> k(P.N0);
  for (int64_t r = 0; r < P.N0; ++r) k[r] = kappa[H0.perm[r]];
  auto col0 = [&](int64_t r, int w) { return H0.cols[H0.slice_blk[r / SLICE] + SLICE * w + r % SLICE]; };
  std::vector<double> A((size_t)P.N0 * W0 * np2, 0.0);
  for (int64_t r = 0; r < P.N0; ++r)
    for (int w = 0; w < W0; ++w) {
      const int hf = P.hostflag[r * W0 + w];
      const int32_t c = col0(r, w);
      double* dst = &A[((size_t)r * W0 + w) * np2];
      const double* ua = &P.UA[((size_t)r * W0 + w) * np2];
      if (w == 0) {
        for (int ij = 0; ij < np2; ++ij) dst[ij] = k[r] * ua[ij];
        for (int v = 1; v < W0; ++v)
          if (P.hostflag[r * W0 + v] == 0) {
            const int32_t cv = col0(r, v);
            const double* uh = &P.UH[((size_t)cv * W0 + P.revslot[r * W0 + v]) * np2];
            for (int ij = 0; ij < np2; ++ij) dst[ij] += k[cv] * uh[ij];
          }
      } else {
        const double s = hf == 1 ? k[r] : (hf == 0 ? k[c] : 0.0);
        for (int ij = 0; ij < np2; ++ij) dst[ij] = s * ua[ij];
      }
      if (!P.UC.empty()) {
        const double* uc = &P.UC[((size_t)r * W0 + w) * np2];
        for (int ij = 0; ij < np2; ++ij) dst[ij] += uc[ij];
      }
    }
  // Galerkin products level by level, blocks stored row-major per (row, slot)
  std::vector<double> cur = A;
  std::vector<int> width(1, W0);
  // flux-form state: M_l blocks and G_l blocks (component-major)
  std::vector<double> Ml, Gl;
  if (P.flux) {
    Ml.assign((size_t)P.N0 * np2, 0.0);
    for (int64_t r = 0; r < P.N0; ++r)
      for (int ij = 0; ij < np2; ++ij) Ml[(size_t)r * np2 + ij] = P.Mblk[(size_t)r * np2 + ij] / k[r];
    Gl = P.G0;
  }
  for (int l = 1; l <= level; ++l) {
    const Level &f = P.lv[l - 1], &c = P.lv[l];
    const int Wf = width.back();
    std::vector<double> nxt((size_t)c.nnzb * np2, 0.0);
    std::vector<double> T(np2);
    for (int64_t kb = 0; kb < c.nnzb; ++kb) {
      double* dst = &nxt[kb * np2];
      for (int64_t q = c.plan_ptr[kb]; q < c.plan_ptr[kb + 1]; ++q) {
        const int32_t e = c.plan_e[q];
        const int w = c.plan_w[q];
        const int32_t cc = f.cols[f.slice_blk[e / SLICE] + SLICE * w + e % SLICE];
        const double* Ab = (l == 1) ? &cur[((size_t)e * Wf + w) * np2] : &cur[(f.row_blk[e] + w) * np2];
        const double* Le = &f.Lblk[(size_t)e * np2];
        const double* Lc = &f.Lblk[(size_t)cc * np2];
        for (int i = 0; i < np; ++i)
          for (int j = 0; j < np; ++j) {
            double s = 0.0;
            for (int m = 0; m < np; ++m) s += Ab[i * np + m] * Lc[m * np + j];
            T[i * np + j] = s;
          }
        for (int i = 0; i < np; ++i)
          for (int j = 0; j < np; ++j) {
            double s = 0.0;
            for (int m = 0; m < np; ++m) s += Le[m * np + i] * T[m * np + j];
            dst[i * np + j] += s;
          }
      }
    }
    if (P.flux) {
      const FluxPlan& F = P.fp[l - 1];
      const int d = P.d;
      const int64_t nX = (int64_t)F.x_col.size(), nY = (int64_t)F.y_col.size();
      std::vector<double> Minv(Ml), X((size_t)d * nX * np2, 0.0), Y((size_t)d * nY * np2, 0.0),
          Mc((size_t)c.n * np2, 0.0);
      for (int64_t r = 0; r < f.n; ++r) invert_spd_like(np, &Minv[(size_t)r * np2]);
      auto blk = [&](const OpRef& o) -> const double* {
        switch (o.kind) {
          case OP_L: return &f.Lblk[(size_t)o.idx * np2];
          case OP_G: return &Gl[((size_t)o.comp * F.g_col.size() + o.idx) * np2];
          case OP_X: return &X[((size_t)o.comp * nX + o.idx) * np2];
          case OP_Y: return &Y[((size_t)o.comp * nY + o.idx) * np2];
          case OP_MINV: return &Minv[(size_t)o.idx * np2];
          case OP_M: return &Ml[(size_t)o.idx * np2];
          default: return nullptr;
        }
      };
      for (int64_t o = 0; o < d * nX; ++o)
        for (int64_t q = F.xp_ptr[o]; q < F.xp_ptr[o + 1]; ++q)
          tp_acc(np, blk(F.xp[q].P), blk(F.xp[q].Q), blk(F.xp[q].R), F.xp[q].sign, &X[(size_t)o * np2]);
      for (int64_t o = 0; o < d * nY; ++o)
        for (int64_t q = F.yp_ptr[o]; q < F.yp_ptr[o + 1]; ++q)
          tp_acc(np, blk(F.yp[q].P), blk(F.yp[q].Q), blk(F.yp[q].R), F.yp[q].sign, &Y[(size_t)o * np2]);
      for (int64_t J = 0; J < c.n; ++J)
        for (int64_t q = F.mp_ptr[J]; q < F.mp_ptr[J + 1]; ++q)
          tp_acc(np, blk(F.mp[q].P), blk(F.mp[q].Q), blk(F.mp[q].R), F.mp[q].sign, &Mc[(size_t)J * np2]);
      std::vector<double> Minvc(Mc);
      for (int64_t J = 0; J < c.n; ++J) invert_spd_like(np, &Minvc[(size_t)J * np2]);
      auto blk2 = [&](const OpRef& o) -> const double* {
        if (o.kind == OP_MINVC) return &Minvc[(size_t)o.idx * np2];
        return blk(o);
      };
      for (int64_t kb = 0; kb < c.nnzb; ++kb)
        for (int64_t q = F.sp_ptr[kb]; q < F.sp_ptr[kb + 1]; ++q)
          tp_acc(np, blk2(F.sp[q].P), blk2(F.sp[q].Q), blk2(F.sp[q].R), F.sp[q].sign, &nxt[(size_t)kb * np2]);
      Ml.swap(Mc);
      Gl.swap(Y);
    }
    cur.swap(nxt);
    width.push_back(0);
  }
  // export in hierarchy numbering, columns ascending
  std::vector<int64_t> cnt(H.n + 1, 0);
  auto valid = [&](int64_t r, int w) {
    if (level == 0) return w == 0 || P.topo.nbr[(int64_t)H.perm[r] * P.nf + w - 1] >= 0;
    return w < H.row_len[r];
  };
  for (int64_t r = 0; r < H.n; ++r) {
    int n = 0;
    for (int w = 0; w < H.row_len[r]; ++w) n += valid(r, w);
    cnt[H.perm[r] + 1] = n;
  }
  for (int64_t i = 0; i < H.n; ++i) cnt[i + 1] += cnt[i];
  std::copy(cnt.begin(), cnt.end(), row_ptr);
  for (int64_t r = 0; r < H.n; ++r) {
    std::vector<std::pair<int32_t, int>> ent;
    for (int w = 0; w < H.row_len[r]; ++w)
      if (valid(r, w)) ent.push_back({H.perm[H.cols[H.slice_blk[r / SLICE] + SLICE * w + r % SLICE]], w});
    std::sort(ent.begin(), ent.end());
    int64_t kk = row_ptr[H.perm[r]];
    for (auto& e : ent) {
      cols[kk] = e.first;
      const double* src = (level == 0) ? &cur[((size_t)r * W0 + e.second) * np2] : &cur[(H.row_blk[r] + e.second) * np2];
      std::copy(src, src + np2, &blocks[kk * np2]);
      ++kk;
    }
  }
  return CDGMG_OK;
}
