// Host-only entry points of the C ABI: version, error text, default options,
// greedy agglomeration (Alg. 1/2) and the switch (Sec. 2.2, Sec. 4.2).  They
// need no GPU; the sanitizer build of the host code links them as well.
#include <algorithm>
#include <cstring>

#include "internal.hpp"

namespace cdg {
const char* last_error_cstr();
}

using namespace cdg;

extern "C" {

int cdgmg_version(void) { return 10100; }

const char* cdgmg_last_error(void) { return cdg::last_error_cstr(); }

void cdgmg_default_options(cdgmg_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->gamma = 1e4;
  o->omega = 0.7;
  o->nu1 = 2;
  o->nu2 = 2;
  o->mg_precision = CDGMG_MG_FP32;
  o->outer = CDGMG_OUTER_FCG;
  o->coarsening = CDGMG_COARSEN_PRIMAL;
  o->switch_mode = CDGMG_SWITCH_CONSISTENT;
  o->switch_seed = 0;
  o->tol = 1e-10;
  o->max_iter = 500;
  o->profile = 0;
  o->kernel_variant = 0;
  o->restart = 50;
  o->beta = 0.0;
  o->velocity[0] = 1.0;
  o->p_coarse = 0;
  o->p_jump = 0;
  o->coarse_group = 0;
  o->row_threads = 0;
  o->coarse_fp64 = 0;
}

int cdgmg_agglomerate(const cdgmg_mesh* mesh, int max_levels, int64_t coarse_dofs_max, int p, uint64_t seed,
                      int32_t* parent_out, int32_t* level_sizes_out, int* n_levels_out) {
  set_error("");
  if (!mesh || !parent_out || !level_sizes_out || !n_levels_out || max_levels < 1 || p < 1 || p > 3) {
    set_error("agglomerate: invalid argument");
    return CDGMG_ERR_ARG;
  }
  try {
    Topology t;
    int rc = build_topology(*mesh, t);
    if (rc) return rc;
    const int np = mesh->dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
    std::vector<int32_t> parents, sizes;
    int nl = agglomerate(*mesh, t, max_levels, coarse_dofs_max, np, seed, parents, sizes);
    std::copy(parents.begin(), parents.end(), parent_out);
    std::copy(sizes.begin(), sizes.end(), level_sizes_out);
    *n_levels_out = nl;
  } catch (const std::exception& e) {
    set_error(std::string("agglomerate: ") + e.what());
    return CDGMG_ERR_NOMEM;
  }
  return CDGMG_OK;
}

int cdgmg_switch(const cdgmg_mesh* mesh, int mode, uint64_t seed, int8_t* hosted_out) {
  set_error("");
  if (!mesh || !hosted_out) {
    set_error("switch: invalid argument");
    return CDGMG_ERR_ARG;
  }
  Topology t;
  int rc = build_topology(*mesh, t);
  if (rc) return rc;
  if (mode == CDGMG_SWITCH_NATURAL)
    natural_switch(t, mesh->face_bc, seed);
  else
    consistent_switch(t, mesh->face_bc);
  std::copy(t.hosted.begin(), t.hosted.end(), hosted_out);
  return CDGMG_OK;
}

}  // extern "C"
