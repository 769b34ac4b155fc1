// Driver of the host half of the library for sanitizer builds (AddressSanitizer,
// UndefinedBehaviorSanitizer): no GPU, no HIP.  Each argument is a case file
// (little-endian):
//   int32 dim, p, levels, coarsening, switch_mode, p_coarse; uint64 seed;
//   int64 n_vert, n_elem; float64 coords[n_vert][dim]; int32 e2v[n_elem][dim+1];
//   int8 face_bc[n_elem][dim+1]; float64 kappa[n_elem]
// For each case it runs the switch, the greedy agglomeration and, per level,
// the host-formed level operator, and prints summaries the caller compares
// with the regular build's.
#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/cdgmg.h"

namespace {

template <typename T>
bool read_n(FILE* f, T* dst, size_t n) {
  return n == 0 || std::fread(dst, sizeof(T), n, f) == n;
}

int run_case(const char* path) {
  FILE* f = std::fopen(path, "rb");
  if (!f) return 2;
  int32_t hdr[6];
  uint64_t seed = 0;
  int64_t nv = 0, ne = 0;
  bool ok = read_n(f, hdr, 6) && read_n(f, &seed, 1) && read_n(f, &nv, 1) && read_n(f, &ne, 1);
  const int dim = hdr[0], p = hdr[1], levels = hdr[2];
  std::vector<double> coords, kappa;
  std::vector<int32_t> e2v;
  std::vector<int8_t> bc;
  if (ok) {
    coords.resize((size_t)nv * dim);
    e2v.resize((size_t)ne * (dim + 1));
    bc.resize((size_t)ne * (dim + 1));
    kappa.resize((size_t)ne);
    ok = read_n(f, coords.data(), coords.size()) && read_n(f, e2v.data(), e2v.size()) &&
         read_n(f, bc.data(), bc.size()) && read_n(f, kappa.data(), kappa.size());
  }
  std::fclose(f);
  if (!ok) return 3;
  cdgmg_mesh m{dim, nv, coords.data(), ne, e2v.data(), bc.data()};
  cdgmg_options o;
  cdgmg_default_options(&o);
  o.coarsening = hdr[3];
  o.switch_mode = hdr[4];
  o.switch_seed = seed;
  o.p_coarse = hdr[5];
  std::vector<int8_t> hosted(e2v.size());
  int rc = cdgmg_switch(&m, o.switch_mode, seed, hosted.data());
  if (rc) return 10 - rc;
  long long hs = 0;
  for (size_t k = 0; k < hosted.size(); ++k) hs += (long long)hosted[k] * (long long)(k % 9973 + 1);
  std::printf("switch %lld\n", hs);
  std::vector<int32_t> parents((size_t)ne * levels), sizes(levels);
  int nl = 0;
  rc = cdgmg_agglomerate(&m, levels, 0, p, seed, parents.data(), sizes.data(), &nl);
  if (rc) return 20 - rc;
  std::printf("levels");
  for (int l = 0; l < nl; ++l) std::printf(" %d", sizes[l]);
  std::printf("\n");
  cdgmg_hierarchy h{nl, sizes.data(), parents.data()};
  const int np = dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
  for (int l = 0; l < nl; ++l) {
    int64_t nnzb = 0;
    rc = cdgmg_debug_host_operator(&m, p, kappa.data(), &h, &o, l, &nnzb, nullptr, nullptr, nullptr);
    if (rc) return 30 - rc;
    std::vector<int64_t> rp(sizes[l] + 1);
    std::vector<int32_t> cols(nnzb);
    const int npl = (o.p_coarse == 1 && l >= 1) ? (dim == 2 ? 3 : 4) : np;
    std::vector<double> blk((size_t)nnzb * npl * npl);
    rc = cdgmg_debug_host_operator(&m, p, kappa.data(), &h, &o, l, &nnzb, rp.data(), cols.data(), blk.data());
    if (rc) return 40 - rc;
    double s1 = 0.0, s2 = 0.0;
    for (size_t k = 0; k < blk.size(); ++k) {
      s1 += std::fabs(blk[k]);
      s2 += blk[k] * (double)(k % 101 + 1);
    }
    long long cs = 0;
    for (int64_t k = 0; k < nnzb; ++k) cs += (long long)cols[k] * (k % 7 + 1);
    std::printf("level %d nnzb %lld cols %lld abs %.17g weighted %.17g\n", l, (long long)nnzb, cs, s1, s2);
  }
  return 0;
}

}  // namespace

int main(int argc, char** argv) {
  for (int a = 1; a < argc; ++a) {
    std::printf("case %s\n", argv[a]);
    const int rc = run_case(argv[a]);
    if (rc) {
      std::printf("failed %d: %s\n", rc, cdgmg_last_error());
      return rc;
    }
  }
  return 0;
}
