// Reference simplex, kappa-free CDG element operators, internal ordering,
// agglomerate bases, transfer blocks and coarse sparsity (host).
#include <algorithm>
#include <cmath>
#include <numeric>

#include "internal.hpp"

namespace cdg {

// --------------------------------------------------------------- linear algebra
// Symmetric eigen-decomposition of a small dense matrix by cyclic Jacobi rotations.
static void sym_eig(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double vkp = V[k * n + p], vkq = V[k * n + q];
          V[k * n + p] = c * vkp - s * vkq;
          V[k * n + q] = s * vkp + c * vkq;
        }
      }
  }
}

// In-place inverse of a small dense matrix, Gauss-Jordan with partial pivoting.
static bool invert(int n, double* a) {
  std::vector<int> piv(n);
  std::vector<double> b(2 * n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) b[i * 2 * n + j] = a[i * n + j];
    b[i * 2 * n + n + i] = 1.0;
  }
  for (int k = 0; k < n; ++k) {
    int pr = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(b[i * 2 * n + k]) > std::fabs(b[pr * 2 * n + k])) pr = i;
    if (b[pr * 2 * n + k] == 0.0) return false;
    if (pr != k)
      for (int j = 0; j < 2 * n; ++j) std::swap(b[k * 2 * n + j], b[pr * 2 * n + j]);
    double d = 1.0 / b[k * 2 * n + k];
    for (int j = 0; j < 2 * n; ++j) b[k * 2 * n + j] *= d;
    for (int i = 0; i < n; ++i) {
      if (i == k) continue;
      double f = b[i * 2 * n + k];
      if (f == 0.0) continue;
      for (int j = 0; j < 2 * n; ++j) b[i * 2 * n + j] -= f * b[k * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[i * n + j] = b[i * 2 * n + n + j];
  return true;
}

// Lower Cholesky factor in place (row-major); false if not positive definite.
static bool cholesky(int n, double* a) {
  for (int j = 0; j < n; ++j) {
    double s = a[j * n + j];
    for (int k = 0; k < j; ++k) s -= a[j * n + k] * a[j * n + k];
    if (!(s > 0.0)) return false;
    double ljj = std::sqrt(s);
    a[j * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double t = a[i * n + j];
      for (int k = 0; k < j; ++k) t -= a[i * n + k] * a[j * n + k];
      a[i * n + j] = t / ljj;
    }
    for (int k = j + 1; k < n; ++k) a[j * n + k] = 0.0;
  }
  return true;
}

// ------------------------------------------------------------------ quadrature
// n-point Gauss-Jacobi rule on [0,1] for the weight (1-t)^alpha (Golub-Welsch).
void gauss_jacobi01(int n, int alpha, std::vector<double>& x, std::vector<double>& w) {
  const double a = alpha, b = 0.0;
  std::vector<double> T(n * n, 0.0), V;
  for (int k = 0; k < n; ++k) {
    double diag = (k == 0) ? (b - a) / (a + b + 2.0)
                           : (b * b - a * a) / ((2 * k + a + b) * (2 * k + a + b + 2.0));
    T[k * n + k] = diag;
    if (k + 1 < n) {
      double kk = k + 1;
      double s = 2 * kk + a + b;
      double off = std::sqrt(4.0 * kk * (kk + a) * (kk + b) * (kk + a + b) / (s * s * (s + 1.0) * (s - 1.0)));
      T[k * n + k + 1] = T[(k + 1) * n + k] = off;
    }
  }
  sym_eig(n, T, V);
  const double mu0 = std::pow(2.0, a + b + 1.0) / (a + b + 1.0);
  std::vector<std::pair<double, double>> nw(n);
  for (int i = 0; i < n; ++i) nw[i] = {T[i * n + i], mu0 * V[i] * V[i]};
  std::sort(nw.begin(), nw.end());
  x.resize(n);
  w.resize(n);
  const double scale = std::pow(2.0, a + 1.0);
  for (int i = 0; i < n; ++i) {
    x[i] = 0.5 * (1.0 + nw[i].first);
    w[i] = nw[i].second / scale;
  }
}

// Collapsed Gauss rule on the reference d-simplex (vertices 0, e_1, .., e_d):
// Gauss-Legendre in the first collapsed coordinate and Gauss-Jacobi with
// weight (1-t)^k for the k-th collapsed direction; exact to degree 2n-1.
void simplex_rule(int d, int n, std::vector<double>& x, std::vector<double>& w) {
  std::vector<double> g0, w0, g1, w1, g2, w2;
  gauss_jacobi01(n, 0, g0, w0);
  x.clear();
  w.clear();
  if (d == 1) {
    x = g0;
    w = w0;
    return;
  }
  gauss_jacobi01(n, 1, g1, w1);
  if (d == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        x.push_back(g0[i] * (1.0 - g1[j]));
        x.push_back(g1[j]);
        w.push_back(w0[i] * w1[j]);
      }
    return;
  }
  gauss_jacobi01(n, 2, g2, w2);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int k = 0; k < n; ++k) {
        x.push_back(g0[i] * (1.0 - g1[j]) * (1.0 - g2[k]));
        x.push_back(g1[j] * (1.0 - g2[k]));
        x.push_back(g2[k]);
        w.push_back(w0[i] * w1[j] * w2[k]);
      }
}

// ------------------------------------------------------------ reference element
static std::vector<std::array<int, 3>> graded_exponents(int d, int p) {
  std::vector<std::array<int, 3>> out;
  for (int deg = 0; deg <= p; ++deg) {
    if (d == 2) {
      for (int b = 0; b <= deg; ++b) out.push_back({deg - b, b, 0});
    } else {
      for (int c = 0; c <= deg; ++c)
        for (int b = 0; b <= deg - c; ++b) out.push_back({deg - b - c, b, c});
    }
  }
  return out;
}

void eval_monomials(int d, const std::vector<std::array<int, 3>>& exps, const double* x, double* m) {
  for (size_t k = 0; k < exps.size(); ++k) {
    double v = 1.0;
    for (int c = 0; c < d; ++c)
      for (int q = 0; q < exps[k][c]; ++q) v *= x[c];
    m[k] = v;
  }
}

void RefElem::init(int d_, int p_) {
  d = d_;
  p = p_;
  exps = graded_exponents(d, p);
  np = (int)exps.size();
  nodes.clear();
  bary.clear();
  if (d == 2) {
    for (int j = 0; j <= p; ++j)
      for (int i = 0; i <= p - j; ++i) {
        nodes.push_back((double)i / p);
        nodes.push_back((double)j / p);
        bary.push_back({p - i - j, i, j, 1});
      }
  } else {
    for (int k = 0; k <= p; ++k)
      for (int j = 0; j <= p - k; ++j)
        for (int i = 0; i <= p - j - k; ++i) {
          nodes.push_back((double)i / p);
          nodes.push_back((double)j / p);
          nodes.push_back((double)k / p);
          bary.push_back({p - i - j - k, i, j, k});
        }
  }
  std::vector<double> V(np * np);
  for (int i = 0; i < np; ++i) eval_monomials(d, exps, &nodes[i * d], &V[i * np]);
  invert(np, V.data());  // V^{-1}: coef[m][n]
  coef = V;
  simplex_rule(d, p + 1, qx, qw);
  simplex_rule(d - 1, p + 1, fx, fw);
  nq = (int)qw.size();
  nfq = (int)fw.size();
}

void RefElem::eval(const double* xi, double* phi) const {
  double m[32];
  eval_monomials(d, exps, xi, m);
  for (int n = 0; n < np; ++n) {
    double s = 0.0;
    for (int k = 0; k < np; ++k) s += m[k] * coef[k * np + n];
    phi[n] = s;
  }
}

void RefElem::eval_grad(const double* xi, double* g) const {
  double dm[32][3];
  for (int k = 0; k < np; ++k)
    for (int c = 0; c < d; ++c) {
      if (exps[k][c] == 0) {
        dm[k][c] = 0.0;
        continue;
      }
      double v = exps[k][c];
      for (int cc = 0; cc < d; ++cc) {
        int pw = exps[k][cc] - (cc == c ? 1 : 0);
        for (int q = 0; q < pw; ++q) v *= xi[cc];
      }
      dm[k][c] = v;
    }
  for (int n = 0; n < np; ++n)
    for (int c = 0; c < d; ++c) {
      double s = 0.0;
      for (int k = 0; k < np; ++k) s += dm[k][c] * coef[k * np + n];
      g[n * d + c] = s;
    }
}

// ------------------------------------------------------------------- geometry
namespace {
struct Geo {
  double v0[3], J[3][3], Ji[3][3], det;
};

Geo geometry(const cdgmg_mesh& m, int64_t e) {
  const int d = m.dim, nf = d + 1;
  Geo g{};
  const int32_t* v = m.e2v + e * nf;
  for (int c = 0; c < d; ++c) g.v0[c] = m.coords[v[0] * d + c];
  for (int k = 0; k < d; ++k)
    for (int c = 0; c < d; ++c) g.J[c][k] = m.coords[v[k + 1] * d + c] - g.v0[c];
  if (d == 2) {
    g.det = g.J[0][0] * g.J[1][1] - g.J[0][1] * g.J[1][0];
    g.Ji[0][0] = g.J[1][1] / g.det;
    g.Ji[0][1] = -g.J[0][1] / g.det;
    g.Ji[1][0] = -g.J[1][0] / g.det;
    g.Ji[1][1] = g.J[0][0] / g.det;
  } else {
    double(*J)[3] = g.J;
    g.det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
            J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double id = 1.0 / g.det;
    g.Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) * id;
    g.Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    g.Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    g.Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) * id;
    g.Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    g.Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    g.Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) * id;
    g.Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    g.Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
  }
  return g;
}

void to_ref(const Geo& g, int d, const double* x, double* xi) {
  for (int a = 0; a < d; ++a) {
    double s = 0.0;
    for (int c = 0; c < d; ++c) s += g.Ji[a][c] * (x[c] - g.v0[c]);
    xi[a] = s;
  }
}

void to_phys(const Geo& g, int d, const double* xi, double* x) {
  for (int c = 0; c < d; ++c) {
    double s = g.v0[c];
    for (int a = 0; a < d; ++a) s += g.J[c][a] * xi[a];
    x[c] = s;
  }
}

// Facet i of element e: quadrature points, weights, outward unit normal, measure.
struct Facet {
  std::vector<double> x, w;
  double n[3];
  double meas;
};

Facet facet(const cdgmg_mesh& m, const RefElem& R, int64_t e, int i) {
  const int d = m.dim, nf = d + 1;
  const int32_t* v = m.e2v + e * nf;
  double W[3][3];
  int c = 0;
  for (int k = 0; k < nf; ++k)
    if (k != i) {
      for (int a = 0; a < d; ++a) W[c][a] = m.coords[v[k] * d + a];
      ++c;
    }
  Facet F;
  double t1[3] = {0, 0, 0}, t2[3] = {0, 0, 0};
  for (int a = 0; a < d; ++a) {
    t1[a] = W[1][a] - W[0][a];
    if (d == 3) t2[a] = W[2][a] - W[0][a];
  }
  if (d == 2) {
    F.meas = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1]);
    F.n[0] = t1[1] / F.meas;
    F.n[1] = -t1[0] / F.meas;
    F.n[2] = 0.0;
  } else {
    double cr[3] = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2], t1[0] * t2[1] - t1[1] * t2[0]};
    double nn = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    F.meas = 0.5 * nn;
    for (int a = 0; a < 3; ++a) F.n[a] = cr[a] / nn;
  }
  double dot = 0.0;
  for (int a = 0; a < d; ++a) dot += (m.coords[v[i] * d + a] - W[0][a]) * F.n[a];
  if (dot > 0)
    for (int a = 0; a < d; ++a) F.n[a] = -F.n[a];
  const double refmeas = (d == 2) ? 1.0 : 0.5;
  F.x.resize(R.nfq * d);
  F.w.resize(R.nfq);
  for (int q = 0; q < R.nfq; ++q) {
    for (int a = 0; a < d; ++a) {
      double s = W[0][a];
      for (int k = 0; k < d - 1; ++k) s += R.fx[q * (d - 1) + k] * (W[k + 1][a] - W[0][a]);
      F.x[q * d + a] = s;
    }
    F.w[q] = R.fw[q] * F.meas / refmeas;
  }
  return F;
}

// small dense helpers (row-major)
inline void matTmulM(int n, const double* A, const double* Wd, const double* B, int nq, double* C) {
  // C[i][j] = sum_q A[q][i] * Wd[q] * B[q][j]   (A, B: [nq][n])
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double s = 0.0;
      for (int q = 0; q < nq; ++q) s += A[q * n + i] * Wd[q] * B[q * n + j];
      C[i * n + j] = s;
    }
}
}  // namespace

// ---------------------------------------------------------------- the problem
int build_problem(const cdgmg_mesh& m, int p, const cdgmg_hierarchy& h, const cdgmg_options& o, Problem& P) {
  if (p < 1 || p > 3) {
    set_error("setup: p must be 1, 2 or 3");
    return CDGMG_ERR_ARG;
  }
  int rc = build_topology(m, P.topo);
  if (rc) return rc;
  if (o.switch_mode == CDGMG_SWITCH_NATURAL)
    natural_switch(P.topo, m.face_bc, o.switch_seed);
  else
    consistent_switch(P.topo, m.face_bc);
  const Topology& T = P.topo;
  const int d = m.dim, nf = d + 1;
  const int64_t N0 = m.n_elem;
  P.d = d;
  P.p = p;
  P.nf = nf;
  P.N0 = N0;
  P.ref.init(d, p);
  const RefElem& R = P.ref;
  const int np = R.np;
  P.np = np;
  const int nb2 = np * np;

  // ---- hierarchy validation and internal orders
  if (h.n_levels < 1 || h.level_sizes[0] != N0) {
    set_error("hierarchy: level_sizes[0] must equal n_elem");
    return CDGMG_ERR_HIERARCHY;
  }
  const int L = h.n_levels - 1;
  P.L = L;
  P.lv.assign(L + 1, Level());
  std::vector<const int32_t*> par(L);
  {
    int64_t off = 0;
    for (int l = 0; l < L; ++l) {
      par[l] = h.parent + off;
      const int64_t nl = h.level_sizes[l], nc = h.level_sizes[l + 1];
      if (nc < 1 || nc > nl) {
        set_error("hierarchy: level sizes must be positive and non-increasing");
        return CDGMG_ERR_HIERARCHY;
      }
      std::vector<char> seen(nc, 0);
      for (int64_t e = 0; e < nl; ++e) {
        int32_t q = par[l][e];
        if (q < 0 || q >= nc) {
          set_error("hierarchy: parent index out of range at level " + std::to_string(l));
          return CDGMG_ERR_HIERARCHY;
        }
        seen[q] = 1;
      }
      for (int64_t c = 0; c < nc; ++c)
        if (!seen[c]) {
          set_error("hierarchy: empty aggregate at level " + std::to_string(l + 1));
          return CDGMG_ERR_HIERARCHY;
        }
      off += nl;
    }
  }
  for (int l = 0; l <= L; ++l) P.lv[l].n = h.level_sizes[l];
  {
    Level& c = P.lv[L];
    c.perm.resize(c.n);
    std::iota(c.perm.begin(), c.perm.end(), 0);
    c.iperm = c.perm;
  }
  for (int l = L - 1; l >= 0; --l) {
    Level &f = P.lv[l], &c = P.lv[l + 1];
    f.perm.resize(f.n);
    std::iota(f.perm.begin(), f.perm.end(), 0);
    std::stable_sort(f.perm.begin(), f.perm.end(), [&](int32_t a, int32_t b) {
      return c.iperm[par[l][a]] < c.iperm[par[l][b]];
    });
    f.iperm.resize(f.n);
    for (int64_t r = 0; r < f.n; ++r) f.iperm[f.perm[r]] = (int32_t)r;
    f.parent.resize(f.n);
    for (int64_t r = 0; r < f.n; ++r) f.parent[r] = c.iperm[par[l][f.perm[r]]];
    c.child_start.assign(c.n + 1, 0);
    for (int64_t r = 0; r < f.n; ++r) c.child_start[f.parent[r] + 1]++;
    for (int64_t I = 0; I < c.n; ++I) c.child_start[I + 1] += c.child_start[I];
  }
  P.lv[0].fine_begin.resize(N0 + 1);
  std::iota(P.lv[0].fine_begin.begin(), P.lv[0].fine_begin.end(), 0);
  for (int l = 1; l <= L; ++l) {
    Level &c = P.lv[l], &f = P.lv[l - 1];
    c.fine_begin.resize(c.n + 1);
    for (int64_t I = 0; I <= c.n; ++I) c.fine_begin[I] = f.fine_begin[c.child_start[I]];
  }
  const std::vector<int32_t>& perm0 = P.lv[0].perm;
  const std::vector<int32_t>& iperm0 = P.lv[0].iperm;

  // ---- Dirichlet penalty scale: h_avg = mean of d |K| / |f| over Dirichlet facets
  {
    double sum = 0.0;
    int64_t cnt = 0;
    for (int64_t e = 0; e < N0; ++e)
      for (int i = 0; i < nf; ++i)
        if (T.nbr[e * nf + i] < 0 && m.face_bc[e * nf + i] == 0) {
          Geo g = geometry(m, e);
          double vol = g.det / (d == 2 ? 2.0 : 6.0);
          Facet F = facet(m, R, e, i);
          sum += d * vol / F.meas;
          ++cnt;
        }
    P.h_avg = cnt ? sum / cnt : 1.0;
    P.gamma = o.gamma;
    P.CD = o.gamma / P.h_avg;
  }

  // ---- level-0 kappa-free blocks
  const int W0 = nf + 1;
  P.UA.assign((size_t)N0 * W0 * nb2, 0.0);
  P.UH.assign((size_t)N0 * W0 * nb2, 0.0);
  P.hostflag.assign((size_t)N0 * W0, -1);
  P.revslot.assign((size_t)N0 * W0, 0);
  P.Mblk.assign((size_t)N0 * nb2, 0.0);
  P.Gblk.assign((size_t)d * N0 * W0 * nb2, 0.0);
  P.nodes.assign((size_t)N0 * np * d, 0.0);
  std::vector<double> phiq(R.nq * np), gref(R.nq * np * d);
  for (int q = 0; q < R.nq; ++q) {
    R.eval(&R.qx[q * d], &phiq[q * np]);
    R.eval_grad(&R.qx[q * d], &gref[q * np * d]);
  }
  std::vector<int> bad(1, 0);
  parallel_for(N0, [&](int64_t e0, int64_t e1) {
    std::vector<double> M(nb2), Mi(nb2), S(nb2), Dc(3 * nb2), g(R.nq * np * d), wq(R.nq);
    std::vector<double> TK(R.nfq * np), TN(R.nfq * np), DnK(R.nfq * np), FK(nb2), FN(nb2), tmp(nb2);
    std::vector<double> Uown(nb2), UKN(nb2), UNN(nb2), GKK(3 * nb2), GKN(3 * nb2);
    double xi[3], phi[32], gr[32 * 3];
    for (int64_t e = e0; e < e1; ++e) {
      const int64_t r = iperm0[e];
      Geo G = geometry(m, e);
      for (int q = 0; q < R.nq; ++q) wq[q] = R.qw[q] * G.det;
      matTmulM(np, phiq.data(), wq.data(), phiq.data(), R.nq, M.data());
      Mi = M;
      if (!invert(np, Mi.data())) bad[0] = 1;
      for (int q = 0; q < R.nq; ++q)
        for (int n = 0; n < np; ++n)
          for (int c = 0; c < d; ++c) {
            double s = 0.0;
            for (int a = 0; a < d; ++a) s += gref[(q * np + n) * d + a] * G.Ji[a][c];
            g[(q * np + n) * d + c] = s;
          }
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
          double s = 0.0;
          for (int q = 0; q < R.nq; ++q)
            for (int c = 0; c < d; ++c) s += wq[q] * g[(q * np + i) * d + c] * g[(q * np + j) * d + c];
          S[i * np + j] = s;
          for (int c = 0; c < d; ++c) {
            double t = 0.0;
            for (int q = 0; q < R.nq; ++q) t += wq[q] * phiq[q * np + i] * g[(q * np + j) * d + c];
            Dc[c * nb2 + i * np + j] = t;
          }
        }
      Uown = S;
      for (int c = 0; c < d; ++c)
        for (int k = 0; k < nb2; ++k) GKK[c * nb2 + k] = Dc[c * nb2 + k];
      for (int i = 0; i < nf; ++i) {
        const int32_t nb = T.nbr[e * nf + i];
        const bool hosted = T.hosted[e * nf + i] != 0;
        if (!hosted) continue;  // unhosted interior facet or Neumann facet
        Facet F = facet(m, R, e, i);
        Geo GN{};
        int jn = 0;  // the facet's local index in the neighbour
        if (nb >= 0) {
          GN = geometry(m, nb);
          while (T.nbr[nb * nf + jn] != e) ++jn;
        }
        // traces on the facet: basis functions of nodes off the facet vanish
        // there identically, and are set to exact zeros (so every
        // off-diagonal block couples the neighbours through facet nodes only)
        for (int q = 0; q < R.nfq; ++q) {
          to_ref(G, d, &F.x[q * d], xi);
          R.eval(xi, phi);
          R.eval_grad(xi, gr);
          for (int n = 0; n < np; ++n) {
            TK[q * np + n] = R.on_facet(n, i) ? phi[n] : 0.0;
            double dn = 0.0;
            for (int c = 0; c < d; ++c) {
              double gc = 0.0;
              for (int a = 0; a < d; ++a) gc += gr[n * d + a] * G.Ji[a][c];
              dn += gc * F.n[c];
            }
            DnK[q * np + n] = dn;
          }
          if (nb >= 0) {
            to_ref(GN, d, &F.x[q * d], xi);
            R.eval(xi, phi);
            for (int n = 0; n < np; ++n) TN[q * np + n] = R.on_facet(n, jn) ? phi[n] : 0.0;
          }
        }
        // jump w = T_N u_N - T_K u_K;  F_K = -T_K^T W T_K, F_N = T_K^T W T_N
        matTmulM(np, TK.data(), F.w.data(), TK.data(), R.nfq, tmp.data());
        for (int k = 0; k < nb2; ++k) FK[k] = -tmp[k];
        // t1_KK = -DnK^T W TK
        matTmulM(np, DnK.data(), F.w.data(), TK.data(), R.nfq, tmp.data());
        for (int a = 0; a < np; ++a)
          for (int b = 0; b < np; ++b) Uown[a * np + b] += -tmp[a * np + b] - tmp[b * np + a];
        // lifting (K,K): F_K^T M^-1 F_K
        for (int a = 0; a < np; ++a)
          for (int b = 0; b < np; ++b) {
            double s = 0.0;
            for (int k = 0; k < np; ++k)
              for (int l = 0; l < np; ++l) s += FK[k * np + a] * Mi[k * np + l] * FK[l * np + b];
            Uown[a * np + b] += s;
          }
        for (int c = 0; c < d; ++c)
          for (int k = 0; k < nb2; ++k) GKK[c * nb2 + k] += F.n[c] * FK[k];
        if (nb < 0) {  // Dirichlet penalty
          matTmulM(np, TK.data(), F.w.data(), TK.data(), R.nfq, tmp.data());
          for (int k = 0; k < nb2; ++k) Uown[k] += P.CD * tmp[k];
          continue;
        }
        matTmulM(np, TK.data(), F.w.data(), TN.data(), R.nfq, FN.data());
        matTmulM(np, DnK.data(), F.w.data(), TN.data(), R.nfq, tmp.data());  // t1_KN
        for (int a = 0; a < np; ++a)
          for (int b = 0; b < np; ++b) {
            double s = 0.0, s2 = 0.0;
            for (int k = 0; k < np; ++k)
              for (int l = 0; l < np; ++l) {
                s += FK[k * np + a] * Mi[k * np + l] * FN[l * np + b];
                s2 += FN[k * np + a] * Mi[k * np + l] * FN[l * np + b];
              }
            UKN[a * np + b] = tmp[a * np + b] + s;
            UNN[a * np + b] = s2;
          }
        const int64_t rn = iperm0[nb];
        const int j = jn;
        double* ua = &P.UA[((size_t)r * W0 + i + 1) * nb2];
        double* uh = &P.UH[((size_t)r * W0 + i + 1) * nb2];
        double* ub = &P.UA[((size_t)rn * W0 + j + 1) * nb2];
        for (int a = 0; a < np; ++a)
          for (int b = 0; b < np; ++b) {
            ua[a * np + b] = UKN[a * np + b];
            uh[a * np + b] = UNN[a * np + b];
            ub[b * np + a] = UKN[a * np + b];
          }
        P.hostflag[(size_t)r * W0 + i + 1] = 1;
        P.hostflag[(size_t)rn * W0 + j + 1] = 0;
        for (int c = 0; c < d; ++c) {
          double* gd = &P.Gblk[(((size_t)c * N0 + r) * W0 + i + 1) * nb2];
          for (int k = 0; k < nb2; ++k) gd[k] = F.n[c] * FN[k];
        }
      }
      std::copy(Uown.begin(), Uown.end(), &P.UA[(size_t)r * W0 * nb2]);
      std::copy(M.begin(), M.end(), &P.Mblk[(size_t)r * nb2]);
      for (int c = 0; c < d; ++c)
        std::copy(&GKK[c * nb2], &GKK[c * nb2] + nb2, &P.Gblk[(((size_t)c * N0 + r) * W0) * nb2]);
      for (int n = 0; n < np; ++n) to_phys(G, d, &R.nodes[n * d], &P.nodes[((size_t)e * np + n) * d]);
    }
  });
  if (bad[0]) {
    set_error("setup: singular element mass matrix");
    return CDGMG_ERR_MESH;
  }
  // The diagonal contributions (an element's own block, and what a hosted
  // facet adds to the neighbour's diagonal block) are symmetric in exact
  // arithmetic; their rounding is made symmetric too, so that every
  // assembled diagonal block of the symmetric operator is symmetric bit for
  // bit and may be stored as its upper triangle.
  parallel_for(N0, [&](int64_t r0, int64_t r1) {
    for (int64_t r = r0; r < r1; ++r)
      for (int w = 0; w < W0; ++w) {
        double* B = w == 0 ? &P.UA[(size_t)r * W0 * nb2] : &P.UH[((size_t)r * W0 + w) * nb2];
        for (int a = 0; a < np; ++a)
          for (int c = a + 1; c < np; ++c) {
            const double v = 0.5 * (B[a * np + c] + B[c * np + a]);
            B[a * np + c] = v;
            B[c * np + a] = v;
          }
      }
  });
  // ---- upwind convection blocks of beta v . grad u (Sec. 5):
  //   (beta v . grad u_K, w_K)_K - sum over inflow facets (v . n_K < 0) of
  //   int_f beta (v . n_K) (u_K - u_ext) w_K,  u_ext = neighbour trace, 0 on
  //   Dirichlet facets, u_K on Neumann facets (no term)
  P.beta = o.beta;
  if (o.beta != 0.0) {
    P.UC.assign((size_t)N0 * W0 * nb2, 0.0);
    const double* v = o.velocity;
    parallel_for(N0, [&](int64_t e0, int64_t e1) {
      std::vector<double> g(R.nq * np * d), wq(R.nq), TK(R.nfq * np), TN(R.nfq * np), tmp(nb2);
      double xi[3], phi[32];
      for (int64_t e = e0; e < e1; ++e) {
        const int64_t r = iperm0[e];
        Geo G = geometry(m, e);
        for (int q = 0; q < R.nq; ++q) wq[q] = R.qw[q] * G.det;
        double* own = &P.UC[(size_t)r * W0 * nb2];
        for (int i = 0; i < np; ++i)
          for (int j = 0; j < np; ++j) {
            double s = 0.0;
            for (int q = 0; q < R.nq; ++q) {
              double vg = 0.0;
              for (int c = 0; c < d; ++c) {
                double gc = 0.0;
                for (int a = 0; a < d; ++a) gc += gref[(q * np + j) * d + a] * G.Ji[a][c];
                vg += v[c] * gc;
              }
              s += wq[q] * phiq[q * np + i] * vg;
            }
            own[i * np + j] = o.beta * s;
          }
        for (int i = 0; i < nf; ++i) {
          const int32_t nb = T.nbr[e * nf + i];
          if (nb < 0 && m.face_bc[e * nf + i] != 0) continue;
          Facet F = facet(m, R, e, i);
          double vn = 0.0;
          for (int c = 0; c < d; ++c) vn += v[c] * F.n[c];
          if (vn >= 0.0) continue;
          Geo GN{};
          int jn = 0;
          if (nb >= 0) {
            GN = geometry(m, nb);
            while (T.nbr[nb * nf + jn] != e) ++jn;
          }
          for (int q = 0; q < R.nfq; ++q) {
            to_ref(G, d, &F.x[q * d], xi);
            R.eval(xi, phi);
            for (int n = 0; n < np; ++n) TK[q * np + n] = R.on_facet(n, i) ? phi[n] : 0.0;
            if (nb >= 0) {
              to_ref(GN, d, &F.x[q * d], xi);
              R.eval(xi, phi);
              for (int n = 0; n < np; ++n) TN[q * np + n] = R.on_facet(n, jn) ? phi[n] : 0.0;
            }
          }
          matTmulM(np, TK.data(), F.w.data(), TK.data(), R.nfq, tmp.data());
          for (int k = 0; k < nb2; ++k) own[k] += -o.beta * vn * tmp[k];
          if (nb >= 0) {
            matTmulM(np, TK.data(), F.w.data(), TN.data(), R.nfq, tmp.data());
            double* off = &P.UC[((size_t)r * W0 + i + 1) * nb2];
            for (int k = 0; k < nb2; ++k) off[k] = o.beta * vn * tmp[k];
          }
        }
      }
    });
  }
  // reverse slots
  for (int64_t r = 0; r < N0; ++r) {
    const int64_t e = perm0[r];
    for (int i = 0; i < nf; ++i) {
      int32_t nb = T.nbr[e * nf + i];
      if (nb < 0) continue;
      int j = 0;
      while (T.nbr[nb * nf + j] != e) ++j;
      P.revslot[r * W0 + i + 1] = (int8_t)(j + 1);
    }
  }

  // ---- level-0 sliced-ELL pattern (uniform width nf+1; boundary slots padded)
  {
    Level& A = P.lv[0];
    const int64_t ns = A.slices();
    A.row_len.assign(N0, W0);
    A.slice_w.assign(ns, W0);
    A.slice_blk.resize(ns + 1);
    for (int64_t s = 0; s <= ns; ++s) A.slice_blk[s] = s * (int64_t)W0 * SLICE;
    A.cols.assign(ns * W0 * SLICE, 0);
    A.nnzb = 0;
    for (int64_t r = 0; r < ns * SLICE; ++r) {
      const int64_t s = r / SLICE, lane = r % SLICE;
      for (int w = 0; w < W0; ++w) {
        int32_t col = (r < N0) ? (int32_t)r : 0;
        if (r < N0 && w > 0) {
          int32_t nb = T.nbr[perm0[r] * nf + w - 1];
          if (nb >= 0) col = iperm0[nb];
        }
        A.cols[A.slice_blk[s] + w * SLICE + lane] = col;
      }
    }
    for (int64_t r = 0; r < N0; ++r) {
      A.nnzb += 1;
      for (int i = 0; i < nf; ++i) A.nnzb += T.nbr[perm0[r] * nf + i] >= 0;
    }
  }

  // ---- aggregate bases (levels >= 1): centroid, radius, two-pass Cholesky
  const int nm = np;
  for (int l = 1; l <= L; ++l) {
    Level& c = P.lv[l];
    c.center.assign(c.n * d, 0.0);
    c.scale.assign(c.n, 0.0);
    c.bcoef.assign((size_t)c.n * nm * np, 0.0);
    std::vector<int> fail(1, 0);
    parallel_for(c.n, [&](int64_t I0, int64_t I1) {
      std::vector<double> xq(R.nq * d), mono(nm), Gm(nm * nm), Cf(nm * np), G2(np * np), tmp(nm * np);
      for (int64_t I = I0; I < I1; ++I) {
        double cen[3] = {0, 0, 0}, vol = 0.0;
        for (int64_t fr = c.fine_begin[I]; fr < c.fine_begin[I + 1]; ++fr) {
          Geo G = geometry(m, perm0[fr]);
          for (int q = 0; q < R.nq; ++q) {
            double x[3];
            to_phys(G, d, &R.qx[q * d], x);
            double w = R.qw[q] * G.det;
            for (int a = 0; a < d; ++a) cen[a] += w * x[a];
            vol += w;
          }
        }
        for (int a = 0; a < d; ++a) cen[a] /= vol;
        double hmax = 0.0;
        for (int64_t fr = c.fine_begin[I]; fr < c.fine_begin[I + 1]; ++fr) {
          const int32_t* v = m.e2v + (int64_t)perm0[fr] * nf;
          for (int k = 0; k < nf; ++k) {
            double s = 0.0;
            for (int a = 0; a < d; ++a) {
              double t = m.coords[v[k] * d + a] - cen[a];
              s += t * t;
            }
            hmax = std::max(hmax, std::sqrt(s));
          }
        }
        std::fill(Gm.begin(), Gm.end(), 0.0);
        for (int64_t fr = c.fine_begin[I]; fr < c.fine_begin[I + 1]; ++fr) {
          Geo G = geometry(m, perm0[fr]);
          for (int q = 0; q < R.nq; ++q) {
            double x[3], xh[3];
            to_phys(G, d, &R.qx[q * d], x);
            for (int a = 0; a < d; ++a) xh[a] = (x[a] - cen[a]) / hmax;
            eval_monomials(d, R.exps, xh, mono.data());
            double w = R.qw[q] * G.det;
            for (int a = 0; a < nm; ++a)
              for (int b = 0; b < nm; ++b) Gm[a * nm + b] += w * mono[a] * mono[b];
          }
        }
        std::fill(Cf.begin(), Cf.end(), 0.0);
        for (int a = 0; a < nm; ++a) Cf[a * np + a] = 1.0;
        for (int pass = 0; pass < 2; ++pass) {
          // G2 = Cf^T Gm Cf ; Cf <- Cf chol(G2)^{-T}
          for (int a = 0; a < np; ++a)
            for (int b = 0; b < np; ++b) {
              double s = 0.0;
              for (int k = 0; k < nm; ++k)
                for (int l2 = 0; l2 < nm; ++l2) s += Cf[k * np + a] * Gm[k * nm + l2] * Cf[l2 * np + b];
              G2[a * np + b] = s;
            }
          if (!cholesky(np, G2.data())) {
            fail[0] = 1;
            break;
          }
          // solve Cf_new L^T = Cf  -> Cf_new = Cf L^{-T}: row-wise forward substitution
          for (int k = 0; k < nm; ++k) {
            for (int j = 0; j < np; ++j) {
              double s = Cf[k * np + j];
              for (int t = 0; t < j; ++t) s -= tmp[k * np + t] * G2[j * np + t];
              tmp[k * np + j] = s / G2[j * np + j];
            }
          }
          Cf = tmp;
        }
        for (int a = 0; a < d; ++a) c.center[I * d + a] = cen[a];
        c.scale[I] = hmax;
        std::copy(Cf.begin(), Cf.end(), &c.bcoef[(size_t)I * nm * np]);
      }
    });
    if (fail[0]) {
      set_error("setup: agglomerate Gram matrix is not positive definite");
      return CDGMG_ERR_SINGULAR;
    }
  }
  auto basis_eval = [&](const Level& c, int64_t I, const double* x, double* psi) {
    double xh[3], mono[32];
    for (int a = 0; a < d; ++a) xh[a] = (x[a] - c.center[I * d + a]) / c.scale[I];
    eval_monomials(d, R.exps, xh, mono);
    const double* C = &c.bcoef[(size_t)I * nm * np];
    for (int j = 0; j < np; ++j) {
      double s = 0.0;
      for (int k = 0; k < nm; ++k) s += mono[k] * C[k * np + j];
      psi[j] = s;
    }
  };

  // ---- level-0 affine maps into the parents' scaled coordinates
  if (L > 0) {
    const Level& c1 = P.lv[1];
    const int na = d + d * d;
    P.aff0.assign((size_t)N0 * na, 0.0);
    parallel_for(N0, [&](int64_t r0, int64_t r1) {
      for (int64_t r = r0; r < r1; ++r) {
        const int64_t I = P.lv[0].parent[r];
        Geo G = geometry(m, perm0[r]);
        double* u = &P.aff0[(size_t)r * na];
        const double h = c1.scale[I];
        for (int c = 0; c < d; ++c) {
          u[c] = (G.v0[c] - c1.center[I * d + c]) / h;
          for (int a = 0; a < d; ++a) u[d + c * d + a] = G.J[c][a] / h;
        }
      }
    });
  }

  // ---- transfer blocks L_e (row = child basis function, col = parent basis function)
  for (int l = 0; l < L; ++l) {
    Level &f = P.lv[l], &c = P.lv[l + 1];
    f.Lblk.assign((size_t)f.n * nb2, 0.0);
    parallel_for(f.n, [&](int64_t e0, int64_t e1) {
      double psiI[32], psie[32], x[3];
      for (int64_t e = e0; e < e1; ++e) {
        double* Lb = &f.Lblk[(size_t)e * nb2];
        const int64_t I = f.parent[e];
        if (l == 0) {
          const int64_t ue = perm0[e];
          for (int i = 0; i < np; ++i) {
            basis_eval(c, I, &P.nodes[((size_t)ue * np + i) * d], psiI);
            for (int j = 0; j < np; ++j) Lb[i * np + j] = psiI[j];
          }
        } else {
          for (int64_t fr = f.fine_begin[e]; fr < f.fine_begin[e + 1]; ++fr) {
            Geo G = geometry(m, perm0[fr]);
            for (int q = 0; q < R.nq; ++q) {
              to_phys(G, d, &R.qx[q * d], x);
              double w = R.qw[q] * G.det;
              basis_eval(f, e, x, psie);
              basis_eval(c, I, x, psiI);
              for (int i = 0; i < np; ++i)
                for (int j = 0; j < np; ++j) Lb[i * np + j] += w * psie[i] * psiI[j];
            }
          }
        }
      }
    });
  }

  // ---- coarse patterns (Galerkin: distance-1 on the coarse graph; flux form:
  //      plus the Schur-complement couplings) and K7 plans
  P.flux = (o.coarsening == CDGMG_COARSEN_FLUX);
  if (P.flux && L > 0) {
    P.fp.assign(L, FluxPlan());
    flux_g0(P);
  }
  std::vector<std::pair<std::pair<int32_t, int32_t>, TPTerm>> sterms;
  for (int l = 1; l <= L; ++l) {
    Level &f = P.lv[l - 1], &c = P.lv[l];
    std::vector<std::vector<int32_t>> rows(c.n);
    auto fcol = [&](int64_t e, int w) { return f.cols[f.slice_blk[e / SLICE] + w * SLICE + e % SLICE]; };
    auto fvalid = [&](int64_t e, int w) {
      if (l - 1 == 0) return w == 0 || T.nbr[(int64_t)perm0[e] * nf + w - 1] >= 0;
      return w < f.row_len[e];
    };
    for (int64_t I = 0; I < c.n; ++I) {
      auto& row = rows[I];
      row.push_back((int32_t)I);
      for (int64_t e = c.child_start[I]; e < c.child_start[I + 1]; ++e)
        for (int w = 0; w < f.row_len[e]; ++w)
          if (fvalid(e, w)) row.push_back(f.parent[fcol(e, w)]);
    }
    if (P.flux) flux_level_symbolic(P, l - 1, rows, sterms);
    for (int64_t I = 0; I < c.n; ++I) {
      auto& row = rows[I];
      std::sort(row.begin() + 1, row.end());
      row.erase(std::unique(row.begin() + 1, row.end()), row.end());
      row.erase(std::remove(row.begin() + 1, row.end(), (int32_t)I), row.end());
    }
    const int64_t ns = c.slices();
    c.row_len.resize(c.n);
    c.slice_w.assign(ns, 0);
    c.row_blk.assign(c.n + 1, 0);
    for (int64_t I = 0; I < c.n; ++I) {
      c.row_len[I] = (int32_t)rows[I].size();
      c.slice_w[I / SLICE] = std::max(c.slice_w[I / SLICE], c.row_len[I]);
      c.row_blk[I + 1] = c.row_blk[I] + c.row_len[I];
    }
    c.nnzb = c.row_blk[c.n];
    if (P.flux) flux_level_schur(P, l - 1, rows, sterms);
    c.slice_blk.assign(ns + 1, 0);
    for (int64_t s = 0; s < ns; ++s) c.slice_blk[s + 1] = c.slice_blk[s] + (int64_t)c.slice_w[s] * SLICE;
    c.cols.assign(c.slice_blk[ns], 0);
    for (int64_t r = 0; r < ns * SLICE; ++r) {
      const int64_t s = r / SLICE, lane = r % SLICE;
      for (int w = 0; w < c.slice_w[s]; ++w) {
        int32_t col = (r < c.n) ? (int32_t)r : 0;
        if (r < c.n && w < c.row_len[r]) col = rows[r][w];
        c.cols[c.slice_blk[s] + w * SLICE + lane] = col;
      }
    }
    // plan: for coarse block (I, t): all fine (e, w) with parent(col(e,w)) = rows[I][t]
    c.plan_ptr.assign(c.nnzb + 1, 0);
    c.plan_e.clear();
    c.plan_w.clear();
    for (int64_t I = 0; I < c.n; ++I) {
      const auto& row = rows[I];
      std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(row.size());
      for (int64_t e = c.child_start[I]; e < c.child_start[I + 1]; ++e)
        for (int w = 0; w < f.row_len[e]; ++w) {
          if (!fvalid(e, w)) continue;
          int32_t N = f.parent[fcol(e, w)];
          int t = (N == (int32_t)I) ? 0 : (int)(std::lower_bound(row.begin() + 1, row.end(), N) - row.begin());
          lists[t].push_back({(int32_t)e, w});
        }
      for (size_t t = 0; t < row.size(); ++t) {
        for (auto& pr : lists[t]) {
          c.plan_e.push_back(pr.first);
          c.plan_w.push_back(pr.second);
        }
        c.plan_ptr[c.row_blk[I] + t + 1] = (int64_t)c.plan_e.size();
      }
    }
  }
  return CDGMG_OK;
}

// validation of the options shared by setup and the host operator check
int check_options(const cdgmg_options& o) {
  if (o.nu1 < 0 || o.nu2 < 0 || o.nu1 + o.nu2 == 0 || !(o.omega > 0) || !(o.tol > 0) || o.max_iter < 1 ||
      !(o.gamma > 0)) {
    set_error("setup: invalid options");
    return CDGMG_ERR_ARG;
  }
  if (o.outer != CDGMG_OUTER_FCG && o.outer != CDGMG_OUTER_PCG && o.outer != CDGMG_OUTER_GMRES) {
    set_error("setup: unknown outer solver");
    return CDGMG_ERR_ARG;
  }
  if (o.outer == CDGMG_OUTER_GMRES && (o.restart < 1 || o.restart > 200)) {
    set_error("setup: GMRES restart must lie in 1..200");
    return CDGMG_ERR_ARG;
  }
  if (!std::isfinite(o.beta) || !std::isfinite(o.velocity[0]) || !std::isfinite(o.velocity[1]) ||
      !std::isfinite(o.velocity[2])) {
    set_error("setup: beta and velocity must be finite");
    return CDGMG_ERR_ARG;
  }
  if (o.beta != 0.0 && (o.outer != CDGMG_OUTER_GMRES || o.coarsening != CDGMG_COARSEN_PRIMAL)) {
    set_error("setup: convection (beta != 0) makes A nonsymmetric: it needs outer GMRES and primal coarsening");
    return CDGMG_ERR_ARG;
  }
  if (o.coarsening != CDGMG_COARSEN_PRIMAL && o.coarsening != CDGMG_COARSEN_FLUX) {
    set_error("setup: unknown coarsening");
    return CDGMG_ERR_ARG;
  }
  if ((o.p_coarse != 0 && o.p_coarse != 1) || (o.p_jump != 0 && o.p_jump != 1)) {
    set_error("setup: p_coarse and p_jump must be 0 or 1");
    return CDGMG_ERR_ARG;
  }
  if (o.p_coarse == 1 && (o.coarsening != CDGMG_COARSEN_PRIMAL || o.beta != 0.0)) {
    set_error("setup: the hp front end needs primal coarsening and beta = 0");
    return CDGMG_ERR_ARG;
  }
  if (o.coarse_group != 0 && o.coarse_group != 8 && o.coarse_group != 16 && o.coarse_group != 32 &&
      o.coarse_group != 64) {
    set_error("setup: coarse_group must be 0, 8, 16, 32 or 64");
    return CDGMG_ERR_ARG;
  }
  if (o.coarse_fp64 != 0 && o.coarse_fp64 != 1) {
    set_error("setup: coarse_fp64 must be 0 or 1");
    return CDGMG_ERR_ARG;
  }
  if (o.row_threads != 0 && o.row_threads != 64 && o.row_threads != 256) {
    set_error("setup: row_threads must be 0, 64 or 256");
    return CDGMG_ERR_ARG;
  }
  return CDGMG_OK;
}

}  // namespace cdg
