// Mesh topology, CDG switch functions and greedy agglomeration (host).
#include <algorithm>
#include <cmath>
#include <queue>
#include <thread>
#include <tuple>

#include "internal.hpp"

namespace cdg {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body) {
  unsigned hw = std::thread::hardware_concurrency();
  int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 16));
  if (n < 256 || nt == 1) {
    body(0, n);
    return;
  }
  nt = std::min<int64_t>(nt, n);
  std::vector<std::thread> th;
  for (int64_t t = 0; t < nt; ++t) {
    int64_t a = n * t / nt, b = n * (t + 1) / nt;
    th.emplace_back([&body, a, b] { body(a, b); });
  }
  for (auto& x : th) x.join();
}

// ------------------------------------------------------------------ topology
int build_topology(const cdgmg_mesh& m, Topology& t) {
  const int d = m.dim;
  if (d != 2 && d != 3) {
    set_error("mesh: dim must be 2 or 3");
    return CDGMG_ERR_ARG;
  }
  const int nf = d + 1;
  const int64_t N = m.n_elem;
  t.d = d;
  t.nf = nf;
  t.N = N;
  for (int64_t e = 0; e < N * nf; ++e) {
    if (m.e2v[e] < 0 || m.e2v[e] >= m.n_vert) {
      set_error("mesh: vertex index out of range");
      return CDGMG_ERR_MESH;
    }
  }
  // positive orientation
  for (int64_t e = 0; e < N; ++e) {
    const int32_t* v = m.e2v + e * nf;
    double J[3][3];
    for (int k = 0; k < d; ++k)
      for (int c = 0; c < d; ++c) J[c][k] = m.coords[v[k + 1] * d + c] - m.coords[v[0] * d + c];
    double det = (d == 2) ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                          : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    // degenerate too: a volume below 1e-12 of the cube of the longest edge
    // makes the element's mass matrix singular in FP64
    double h2 = 0.0;
    for (int k = 0; k < d; ++k) {
      double l2 = 0.0;
      for (int c = 0; c < d; ++c) l2 += J[c][k] * J[c][k];
      h2 = std::max(h2, l2);
    }
    const double hd = d == 2 ? h2 : h2 * std::sqrt(h2);
    if (!(det > 1e-12 * hd)) {
      set_error("mesh: element " + std::to_string(e) + " has non-positive or near-zero volume");
      return CDGMG_ERR_MESH;
    }
  }
  struct Key {
    int32_t v[3];
    int32_t e;
    int32_t i;
  };
  std::vector<Key> keys(N * nf);
  for (int64_t e = 0; e < N; ++e)
    for (int i = 0; i < nf; ++i) {
      Key k{{0, 0, 0}, (int32_t)e, i};
      int c = 0;
      for (int j = 0; j < nf; ++j)
        if (j != i) k.v[c++] = m.e2v[e * nf + j];
      std::sort(k.v, k.v + d);
      keys[e * nf + i] = k;
    }
  std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
    if (a.v[0] != b.v[0]) return a.v[0] < b.v[0];
    if (a.v[1] != b.v[1]) return a.v[1] < b.v[1];
    if (a.v[2] != b.v[2]) return a.v[2] < b.v[2];
    if (a.e != b.e) return a.e < b.e;
    return a.i < b.i;
  });
  t.nbr.assign(N * nf, -1);
  t.fid.assign(N * nf, -1);
  std::vector<std::array<int32_t, 4>> faces;
  auto same = [&](const Key& a, const Key& b) {
    return a.v[0] == b.v[0] && a.v[1] == b.v[1] && a.v[2] == b.v[2];
  };
  for (size_t k = 0; k < keys.size();) {
    size_t j = k + 1;
    while (j < keys.size() && same(keys[k], keys[j])) ++j;
    if (j - k > 2) {
      set_error("mesh: non-manifold facet shared by more than two elements");
      return CDGMG_ERR_MESH;
    }
    if (j - k == 2) {
      const Key &a = keys[k], &b = keys[k + 1];
      if (a.e == b.e) {
        set_error("mesh: degenerate element with a repeated facet");
        return CDGMG_ERR_MESH;
      }
      t.nbr[a.e * nf + a.i] = b.e;
      t.nbr[b.e * nf + b.i] = a.e;
      faces.push_back({a.e, a.i, b.e, b.i});  // a.e < b.e from the sort
    }
    k = j;
  }
  std::sort(faces.begin(), faces.end(), [](const std::array<int32_t, 4>& x, const std::array<int32_t, 4>& y) {
    return std::make_pair(x[0], x[2]) < std::make_pair(y[0], y[2]);
  });
  const size_t F = faces.size();
  t.face_a.resize(F);
  t.face_ia.resize(F);
  t.face_b.resize(F);
  t.face_ib.resize(F);
  for (size_t f = 0; f < F; ++f) {
    t.face_a[f] = faces[f][0];
    t.face_ia[f] = faces[f][1];
    t.face_b[f] = faces[f][2];
    t.face_ib[f] = faces[f][3];
    t.fid[faces[f][0] * nf + faces[f][1]] = (int32_t)f;
    t.fid[faces[f][2] * nf + faces[f][3]] = (int32_t)f;
  }
  t.hosted.assign(N * nf, 0);
  return CDGMG_OK;
}

static void set_hosts(Topology& t, const int8_t* face_bc, const std::vector<int32_t>& host) {
  const int nf = t.nf;
  std::fill(t.hosted.begin(), t.hosted.end(), 0);
  for (size_t f = 0; f < host.size(); ++f) {
    if (host[f] == t.face_a[f])
      t.hosted[t.face_a[f] * nf + t.face_ia[f]] = 1;
    else
      t.hosted[t.face_b[f] * nf + t.face_ib[f]] = 1;
  }
  for (int64_t e = 0; e < t.N; ++e)
    for (int i = 0; i < nf; ++i)
      if (t.nbr[e * nf + i] < 0 && face_bc[e * nf + i] == 0) t.hosted[e * nf + i] = 1;
}

// Balanced orientation of the dual graph by Hierholzer walks.
void consistent_switch(Topology& t, const int8_t* face_bc) {
  const int64_t N = t.N;
  const int64_t F = (int64_t)t.face_a.size();
  std::vector<int32_t> ea(t.face_a), eb(t.face_b);
  std::vector<int32_t> deg(N + 1, 0);
  for (int64_t f = 0; f < F; ++f) {
    deg[ea[f]]++;
    deg[eb[f]]++;
  }
  const int32_t V = (int32_t)N;
  for (int64_t e = 0; e < N; ++e)
    if (deg[e] & 1) {
      ea.push_back((int32_t)e);
      eb.push_back(V);
    }
  const int64_t E = (int64_t)ea.size();
  // adjacency in CSR, edge ids ascending per vertex
  std::vector<int64_t> ptr(N + 2, 0);
  for (int64_t k = 0; k < E; ++k) {
    ptr[ea[k] + 1]++;
    ptr[eb[k] + 1]++;
  }
  for (int64_t v = 0; v <= N; ++v) ptr[v + 1] += ptr[v];
  std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
  std::vector<int32_t> adj(ptr[N + 1]);
  for (int64_t k = 0; k < E; ++k) {  // k ascending -> lists sorted
    adj[fill[ea[k]]++] = (int32_t)k;
    adj[fill[eb[k]]++] = (int32_t)k;
  }
  std::vector<char> used(E, 0);
  std::vector<int64_t> cur(ptr.begin(), ptr.end() - 1);
  std::vector<int32_t> host(F, -1);
  std::vector<int32_t> stack;
  for (int32_t s = 0; s < (int32_t)N; ++s) {
    stack.assign(1, s);
    while (!stack.empty()) {
      int32_t v = stack.back();
      while (cur[v] < ptr[v + 1] && used[adj[cur[v]]]) ++cur[v];
      if (cur[v] == ptr[v + 1]) {
        stack.pop_back();
        continue;
      }
      int32_t k = adj[cur[v]];
      used[k] = 1;
      int32_t w = (ea[k] == v) ? eb[k] : ea[k];
      if (k < F) host[k] = w;
      stack.push_back(w);
    }
  }
  set_hosts(t, face_bc, host);
}

void natural_switch(Topology& t, const int8_t* face_bc, uint64_t seed) {
  const int64_t F = (int64_t)t.face_a.size();
  std::vector<int32_t> host(F);
  for (int64_t f = 0; f < F; ++f) {
    int32_t a = t.face_a[f], b = t.face_b[f];
    uint64_t na = splitmix64(seed ^ (uint64_t)a), nb = splitmix64(seed ^ (uint64_t)b);
    host[f] = (std::make_pair(na, a) < std::make_pair(nb, b)) ? a : b;
  }
  set_hosts(t, face_bc, host);
}

// ------------------------------------------------------------- agglomeration
namespace {
struct AggLevel {
  int64_t n;
  std::vector<std::vector<int32_t>> verts;  // sorted unique vertex ids per element
  std::vector<std::vector<int32_t>> nbrs;   // sorted unique face neighbours
};

std::vector<int32_t> greedy(const AggLevel& g, int64_t n_vert, uint64_t seed, int level) {
  const int64_t n = g.n;
  const uint64_t base = seed ^ ((uint64_t)level << 32);
  std::vector<uint64_t> rank(n);
  for (int64_t e = 0; e < n; ++e) rank[e] = splitmix64(base ^ (uint64_t)e);
  // vertex -> elements touching it (CSR)
  std::vector<int64_t> vptr(n_vert + 1, 0);
  for (int64_t e = 0; e < n; ++e)
    for (int32_t v : g.verts[e]) vptr[v + 1]++;
  for (int64_t v = 0; v < n_vert; ++v) vptr[v + 1] += vptr[v];
  std::vector<int32_t> velem(vptr[n_vert]);
  {
    std::vector<int64_t> f(vptr.begin(), vptr.end() - 1);
    for (int64_t e = 0; e < n; ++e)
      for (int32_t v : g.verts[e]) velem[f[v]++] = (int32_t)e;
  }
  std::vector<char> inP(n, 1);
  std::vector<int32_t> N(n);
  typedef std::tuple<int32_t, uint64_t, int32_t> QKey;
  std::priority_queue<QKey, std::vector<QKey>, std::greater<QKey>> heap;
  for (int64_t e = 0; e < n; ++e) {
    N[e] = (int32_t)g.nbrs[e].size();
    heap.emplace(N[e], rank[e], (int32_t)e);
  }
  std::vector<int32_t> parent(n, -1);
  std::vector<int64_t> size;
  auto remove = [&](const std::vector<int32_t>& members) {
    for (int32_t e : members) inP[e] = 0;
    for (int32_t e : members)
      for (int32_t k : g.nbrs[e])
        if (inP[k]) {
          N[k] -= 1;
          heap.emplace(N[k], rank[k], k);
        }
  };
  std::vector<int32_t> members, adjacent;
  while (!heap.empty()) {
    auto [key, rk, e] = heap.top();
    heap.pop();
    if (!inP[e] || key != N[e]) continue;
    adjacent.clear();
    for (int32_t k : g.nbrs[e])
      if (parent[k] >= 0) adjacent.push_back(parent[k]);
    std::sort(adjacent.begin(), adjacent.end());
    adjacent.erase(std::unique(adjacent.begin(), adjacent.end()), adjacent.end());
    if (N[e] >= 2 || adjacent.empty()) {
      inP[e] = 0;
      bool have = false;
      std::tuple<int64_t, uint64_t, int32_t> best;
      for (int32_t v : g.verts[e]) {
        int64_t cnt = 0;
        for (int64_t q = vptr[v]; q < vptr[v + 1]; ++q) cnt += inP[velem[q]];
        auto cand = std::make_tuple(-cnt, splitmix64(base ^ (1ull << 62) ^ (uint64_t)v), v);
        if (!have || cand < best) {
          best = cand;
          have = true;
        }
      }
      int32_t vmax = std::get<2>(best);
      members.assign(1, e);
      for (int64_t q = vptr[vmax]; q < vptr[vmax + 1]; ++q)
        if (inP[velem[q]]) members.push_back(velem[q]);
      std::sort(members.begin(), members.end());
      members.erase(std::unique(members.begin(), members.end()), members.end());
      inP[e] = 1;
      int32_t bid = (int32_t)size.size();
      size.push_back((int64_t)members.size());
      for (int32_t k : members) parent[k] = bid;
      remove(members);
    } else {
      int32_t bid = adjacent[0];
      for (int32_t b : adjacent)
        if (std::make_pair(size[b], b) < std::make_pair(size[bid], bid)) bid = b;
      parent[e] = bid;
      size[bid] += 1;
      members.assign(1, e);
      remove(members);
    }
  }
  return parent;
}

void coarsen(const AggLevel& g, const std::vector<int32_t>& parent, AggLevel& out) {
  int64_t nb = 0;
  for (int32_t p : parent) nb = std::max<int64_t>(nb, p + 1);
  out.n = nb;
  out.verts.assign(nb, {});
  out.nbrs.assign(nb, {});
  for (int64_t e = 0; e < g.n; ++e) {
    auto& dst = out.verts[parent[e]];
    dst.insert(dst.end(), g.verts[e].begin(), g.verts[e].end());
    for (int32_t k : g.nbrs[e])
      if (parent[k] != parent[e]) out.nbrs[parent[e]].push_back(parent[k]);
  }
  for (int64_t b = 0; b < nb; ++b) {
    auto& v = out.verts[b];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    auto& w = out.nbrs[b];
    std::sort(w.begin(), w.end());
    w.erase(std::unique(w.begin(), w.end()), w.end());
  }
}
}  // namespace

int agglomerate(const cdgmg_mesh& m, const Topology& t, int max_levels, int64_t coarse_dofs, int np,
                uint64_t seed, std::vector<int32_t>& parents, std::vector<int32_t>& sizes) {
  const int nf = t.nf;
  AggLevel g;
  g.n = t.N;
  g.verts.resize(t.N);
  g.nbrs.resize(t.N);
  for (int64_t e = 0; e < t.N; ++e) {
    g.verts[e].assign(m.e2v + e * nf, m.e2v + (e + 1) * nf);
    std::sort(g.verts[e].begin(), g.verts[e].end());
    g.verts[e].erase(std::unique(g.verts[e].begin(), g.verts[e].end()), g.verts[e].end());
    for (int i = 0; i < nf; ++i)
      if (t.nbr[e * nf + i] >= 0) g.nbrs[e].push_back(t.nbr[e * nf + i]);
    std::sort(g.nbrs[e].begin(), g.nbrs[e].end());
    g.nbrs[e].erase(std::unique(g.nbrs[e].begin(), g.nbrs[e].end()), g.nbrs[e].end());
  }
  parents.clear();
  sizes.assign(1, (int32_t)t.N);
  int level = 0;
  while (true) {
    if (g.n <= 1) break;
    if (level + 1 >= max_levels) break;
    if (coarse_dofs > 0 && g.n * (int64_t)np <= coarse_dofs) break;
    std::vector<int32_t> par = greedy(g, m.n_vert, seed, level);
    parents.insert(parents.end(), par.begin(), par.end());
    AggLevel next;
    coarsen(g, par, next);
    g = std::move(next);
    sizes.push_back((int32_t)g.n);
    ++level;
  }
  return level + 1;
}

}  // namespace cdg
