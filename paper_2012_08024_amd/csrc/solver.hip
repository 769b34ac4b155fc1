// libcdgmg: device setup, V-cycle, outer Krylov loop and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "kernels.inl"

namespace cdg {
const char* last_error_cstr();
}

using namespace cdg;

#define HIPCHK(x)                                                                                   \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) {                                                                         \
      set_error(std::string("HIP error '") + hipGetErrorString(e_) + "' in " #x);                  \
      return CDGMG_ERR_DEVICE;                                                                      \
    }                                                                                               \
  } while (0)

#define RETURN_IF(rc) \
  do {                \
    int rc_ = (rc);   \
    if (rc_) return rc_; \
  } while (0)

#define NP_DISPATCH(np, ...)                 \
  switch (np) {                              \
    case 3: { constexpr int NP = 3; __VA_ARGS__; } break;   \
    case 4: { constexpr int NP = 4; __VA_ARGS__; } break;   \
    case 6: { constexpr int NP = 6; __VA_ARGS__; } break;   \
    case 10: { constexpr int NP = 10; __VA_ARGS__; } break; \
    case 20: { constexpr int NP = 20; __VA_ARGS__; } break; \
    default: break;                          \
  }

// component split of the level-0 kernels (wavefronts per 64-row slice)
#define H_DISPATCH(hv, ...)                                \
  switch (hv) {                                            \
    case 1: { constexpr int H = 1; __VA_ARGS__; } break;   \
    case 2: { constexpr int H = 2; __VA_ARGS__; } break;   \
    case 4: { constexpr int H = 4; __VA_ARGS__; } break;   \
    case 5: { constexpr int H = 5; __VA_ARGS__; } break;   \
    default: break;                                        \
  }

// level-0 kernels: facets per element n_f (3 in 2D, 4 in 3D) and the
// wavefront split H; only the n_p of the element's dimension are instantiated
constexpr bool l0_pair(int np, int nf) {
  return nf == 3 ? (np == 3 || np == 6 || np == 10) : (np == 4 || np == 10 || np == 20);
}
// level-0 kernels: facets per element NF, wavefronts per slice H, and SYM
// (the per-row diagonal blocks and D^{-1} stored as upper triangles)
#define SYM_DISPATCH(sym, ...)          \
  if (sym) {                            \
    constexpr bool SYM = true;          \
    __VA_ARGS__;                        \
  } else {                              \
    constexpr bool SYM = false;         \
    __VA_ARGS__;                        \
  }
#define L0_DISPATCH_H(hh, hv, ...)                                                                          \
  switch ((hh)->P.nf) {                                                                                     \
    case 3: {                                                                                               \
      constexpr int NF = 3;                                                                                 \
      SYM_DISPATCH((hh)->sym0, H_DISPATCH((hv), if constexpr (NP % H == 0 && l0_pair(NP, NF)) {             \
        __VA_ARGS__;                                                                                        \
      }));                                                                                                  \
    } break;                                                                                                \
    case 4: {                                                                                               \
      constexpr int NF = 4;                                                                                 \
      SYM_DISPATCH((hh)->sym0, H_DISPATCH((hv), if constexpr (NP % H == 0 && l0_pair(NP, NF)) {             \
        __VA_ARGS__;                                                                                        \
      }));                                                                                                  \
    } break;                                                                                                \
    default: break;                                                                                         \
  }
#define L0_DISPATCH(hh, ...) L0_DISPATCH_H(hh, (hh)->H0, __VA_ARGS__)
// the compensated (double-double) outer kernels use their own split (H0c)
#define L0C_DISPATCH(hh, ...) L0_DISPATCH_H(hh, (hh)->H0c, __VA_ARGS__)

// hp front end: (n_p at degree q, n_p at the next lower degree) pairs
#define HP_DISPATCH(np0, np1, ...)                                                   \
  if ((np0) == 6 && (np1) == 3) {                                                    \
    constexpr int NP0 = 6, NP1 = 3;                                                  \
    __VA_ARGS__;                                                                     \
  } else if ((np0) == 10 && (np1) == 3) {                                            \
    constexpr int NP0 = 10, NP1 = 3;                                                 \
    __VA_ARGS__;                                                                     \
  } else if ((np0) == 10 && (np1) == 4) {                                            \
    constexpr int NP0 = 10, NP1 = 4;                                                 \
    __VA_ARGS__;                                                                     \
  } else if ((np0) == 20 && (np1) == 4) {                                            \
    constexpr int NP0 = 20, NP1 = 4;                                                 \
    __VA_ARGS__;                                                                     \
  } else if ((np0) == 10 && (np1) == 6) {                                            \
    constexpr int NP0 = 10, NP1 = 6;                                                 \
    __VA_ARGS__;                                                                     \
  } else if ((np0) == 20 && (np1) == 10) {                                           \
    constexpr int NP0 = 20, NP1 = 10;                                                \
    __VA_ARGS__;                                                                     \
  }

// lanes per row of the coarse-level kernels
#define G_DISPATCH(gv, ...)                                  \
  switch (gv) {                                              \
    case 8: { constexpr int G = 8; __VA_ARGS__; } break;     \
    case 16: { constexpr int G = 16; __VA_ARGS__; } break;   \
    case 32: { constexpr int G = 32; __VA_ARGS__; } break;   \
    default: { constexpr int G = 64; __VA_ARGS__; } break;   \
  }

namespace {

// facet nodes of the degree-p simplex: n_fn of the facet-trace form
inline int fnodes(int np, int nf) {
  return nf == 3 ? (np == 3 ? 2 : np == 6 ? 3 : 4) : (np == 4 ? 3 : np == 10 ? 6 : 10);
}

struct DLevel {
  int64_t n = 0, ns = 0, slots = 0, nnzb = 0;
  int32_t* cols = nullptr;
  int64_t* sblk = nullptr;
  int32_t* perm = nullptr;  // internal -> hierarchy id
  double* A64 = nullptr;  // A_l, FP64, sliced (Galerkin products, outer SpMV, export)
  double* D64 = nullptr;  // D_l^{-1}, FP64, per-row layout
  double* L64 = nullptr;  // L_e, FP64, per-row layout
  // V-cycle operators in the multigrid precision T (FP64 mode: Dm = D64, Lm = L64)
  void* Ac = nullptr;  // level 0: off-diagonal blocks in facet-trace form (FP64 mode: the outer A0c)
  void* Ad = nullptr;  // level 0: diagonal blocks, per-row layout
  int8_t* meta = nullptr;  // level 0: facet-trace kind of each off-diagonal slot
  void* Dm = nullptr;  // D^{-1}
  void* Lt = nullptr;  // D^T L_e (D the diagonal block of A), levels 1 .. L-1
  void* Lm = nullptr;  // L_e, levels 1 .. L-1 (level 0 forms it from Aff and Cp)
  void* Aff = nullptr;  // level 0: each element's map into its parent's scaled coordinates, per-row layout
  void* Cp = nullptr;   // level 0: the parents' monomial coefficients, [n_1][n_p][n_p]
  int32_t* parent = nullptr;
  int32_t* child_start = nullptr;
  int32_t* blk_row = nullptr;
  int64_t* row_blk = nullptr;
  int64_t* plan_ptr = nullptr;
  int32_t* plan_e = nullptr;
  int32_t* plan_c = nullptr;  // column of each plan entry's fine block
  int64_t* plan_a = nullptr;  // offset of each plan entry's fine block in the sliced fine operator
  void *b = nullptr, *x = nullptr, *xb = nullptr, *t = nullptr;
  // flux-form coarsening (building level l+1 from this level l)
  double *Mbm = nullptr, *Minv = nullptr, *G = nullptr, *X = nullptr, *Y = nullptr;
  int64_t nX = 0, nY = 0;
  TPDev *xp = nullptr, *yp = nullptr, *mp = nullptr, *sp = nullptr;
  TPOut *xo = nullptr, *yo = nullptr, *mo = nullptr, *so = nullptr;
  int64_t *xpp = nullptr, *ypp = nullptr, *mpp = nullptr, *spp = nullptr;
  int64_t nxo = 0, nyo = 0, nmo = 0, nso = 0;
  // coarse levels: off-diagonal strips of D^{-1} A (wave per row), compact
  // columns (slot 0 = the row itself) and row offsets
  int32_t* wcols = nullptr;
  int64_t* woff = nullptr;
  void* R = nullptr;
  int grp_s = 64, grp_r = 64;  // lanes per row of the sweep and of the restriction
};

struct ProfEv {
  int cls;
  hipEvent_t a, b;
};

// Device memory of a handle: every array is carved, in setup order, out of one
// caller-owned workspace (offsets rounded up to WS_ALIGN bytes).  A counting
// workspace only sums the sizes (cdgmg_workspace_size, or a workspace found too
// small): its pointers are stand-ins that nothing dereferences, and no copy or
// fill is issued through them.
constexpr size_t WS_ALIGN = 256;
struct Workspace {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool counting = true;
};

// Workspace of the handles made by cdgmg_setup_static, for callers that cannot
// allocate: one array per GPU, held by every GPU the library runs on until the
// process ends.  In host code `scratch` is a host-side stand-in; its device
// address on each GPU comes from hipGetSymbolAddress (static_scratch) and is
// the only way host code refers to it.  One live handle per GPU owns it.
constexpr size_t STATIC_WS_BYTES = (size_t)64 << 20;
constexpr int STATIC_MAX_DEV = 64;
std::mutex g_static_mu;
void* g_static_ptr[STATIC_MAX_DEV];
bool g_static_busy[STATIC_MAX_DEV];

}  // namespace

static __device__ __align__(256) char scratch[STATIC_WS_BYTES];

struct cdgmg_handle {
  Problem P;
  cdgmg_options o;
  hipStream_t stream = nullptr;
  int np = 0, d = 0, W0 = 0, L = 0;
  int H0 = 1;   // wavefronts per slice of the level-0 kernels
  int H0c = 1;  // the same for the compensated outer product and true residual
  int64_t N0 = 0;
  std::vector<DLevel> lv;
  Workspace own_ws;
  Workspace* ws = &own_ws;  // a lower hp level carves from its owner's workspace
  int static_dev = -1;      // GPU whose static workspace this handle holds (cdgmg_setup_static)
  bool pinned = true;       // host readback buffers in pinned (hipHostMalloc) memory
  // level 0
  double *UA = nullptr, *UH = nullptr, *M = nullptr, *kappa = nullptr;
  double* UC = nullptr;    // upwind convection blocks (beta != 0), operator layout
  double* A0c = nullptr;   // off-diagonal blocks of A_0 in facet-trace form, FP64 (outer loop)
  // hp front end: the lower-degree hierarchy below level 0 (owned), the nodal
  // embedding T [np][np1] in FP64 and in the multigrid precision
  cdgmg_handle* inner = nullptr;
  bool given_A0 = false;   // this level 0 is set by the owner (T^T A_0 T), not assembled from kappa
  // symmetric operator (no convection): the level-0 per-row blocks (D^{-1},
  // the diagonal blocks in the cycle's precision, and A0d, the FP64 diagonal
  // blocks of the outer loop) are stored as upper triangles
  bool sym0 = false;
  double* A0d = nullptr;
  int np1 = 0;
  // level-0 passes over the V-cycle operator so far; their parity sets the
  // direction of the next one
  uint64_t at_pass = 0;
  double* Tp64 = nullptr;
  void* Tpm = nullptr;
  double* Atmp = nullptr;  // A_0^T staging (beta != 0)
  bool transposed = false; // the levels hold A_l^T
  int8_t *hostflag = nullptr, *revslot = nullptr;
  // coarsest
  int64_t nd = 0, ld = 0;
  double *dense = nullptr, *gjP = nullptr;  // coarsest operator -> its inverse (ld x ld, FP64); pivot block
  double *gjR = nullptr, *gjK = nullptr, *gjC = nullptr;  // panel buffers of one elimination step
  double* gjD = nullptr;                     // its diagonal before elimination
  void* AinvP = nullptr;  // A_L^{-1} in the multigrid precision, leading dimension ld
  // outer vectors (internal order, FP64)
  double *b = nullptr, *x = nullptr, *xl = nullptr, *r = nullptr, *p = nullptr, *q = nullptr, *t1 = nullptr,
         *t2 = nullptr;
  double *scal = nullptr, *part = nullptr;
  int nparts = 0;
  int* err = nullptr;
  double* hscal = nullptr;
  int* herr = nullptr;
  hipEvent_t ev_rr = nullptr;  // ||r||^2 of the last update copied to hscal
  // operator builds: a second stream for the work beside the critical chain
  // (none for handles that must not create resources), its fork and join
  // events, and its own error flag
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int* err_side = nullptr;
  // GMRES: Arnoldi basis V [(m+1) x gm_ld], Z = B V [m x gm_ld], Hessenberg
  // columns (two Gram-Schmidt passes and the norm), partial sums, y
  double *gmV = nullptr, *gmZ = nullptr, *gmH = nullptr, *gmPart = nullptr, *gmY = nullptr;
  double *hgmH = nullptr, *hgmY = nullptr;
  int64_t gm_ld = 0;
  // profiling
  std::vector<ProfEv> evs;
  std::vector<hipEvent_t> pool;
  size_t pool_next = 0;
};

namespace {

// the next count elements of the workspace; once the workspace is exhausted
// it turns into a counting one, so that setup can report the size it needs
template <typename T>
int dalloc(cdgmg_handle* h, T** ptr, size_t count) {
  Workspace& w = *h->ws;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  const size_t off = (w.used + WS_ALIGN - 1) / WS_ALIGN * WS_ALIGN;
  w.used = off + bytes;
  if (w.used > w.cap) w.counting = true;
  *ptr = (T*)((w.counting ? (char*)WS_ALIGN : w.base) + off);
  return CDGMG_OK;
}

template <typename T>
int upload(cdgmg_handle* h, T** ptr, const std::vector<T>& v) {
  RETURN_IF(dalloc(h, ptr, v.size()));
  if (!v.empty() && !h->ws->counting)
    HIPCHK(hipMemcpyAsync(*ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, h->stream));
  return CDGMG_OK;
}

int dzero(cdgmg_handle* h, void* ptr, size_t bytes) {
  if (!h->ws->counting) HIPCHK(hipMemsetAsync(ptr, 0, bytes, h->stream));
  return CDGMG_OK;
}

// host buffer the device results are copied back to (pinned unless the handle
// must not allocate pinned memory); released by host_free
template <typename T>
int host_alloc(cdgmg_handle* h, T** ptr, size_t count) {
  *ptr = nullptr;
  if (h->ws->counting) return CDGMG_OK;
  if (h->pinned) {
    HIPCHK(hipHostMalloc((void**)ptr, std::max<size_t>(count, 1) * sizeof(T)));
  } else {
    *ptr = new (std::nothrow) T[std::max<size_t>(count, 1)]();
    if (!*ptr) return CDGMG_ERR_NOMEM;
  }
  return CDGMG_OK;
}

template <typename T>
void host_free(const cdgmg_handle* h, T* ptr) {
  if (!ptr) return;
  if (h->pinned)
    (void)hipHostFree(ptr);
  else
    delete[] ptr;
}

inline unsigned grid_for(int64_t n, int tpb = TPB) { return (unsigned)((n + tpb - 1) / tpb); }

hipEvent_t next_event(cdgmg_handle* h) {
  if (h->pool_next == h->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    h->pool.push_back(e);
  }
  return h->pool[h->pool_next++];
}

template <typename K, typename... Args>
void launch_lds(cdgmg_handle* h, int cls, K kernel, dim3 grid, dim3 block, size_t lds, Args... args) {
  hipEvent_t a = nullptr, b = nullptr;
  if (h->o.profile && cls >= 0) {
    a = next_event(h);
    b = next_event(h);
    if (a) (void)hipEventRecord(a, h->stream);
  }
  hipLaunchKernelGGL(kernel, grid, block, lds, h->stream, args...);
  if (a && b) {
    (void)hipEventRecord(b, h->stream);
    h->evs.push_back({cls, a, b});
  }
}
template <typename K, typename... Args>
void launch(cdgmg_handle* h, int cls, K kernel, dim3 grid, dim3 block, Args... args) {
  launch_lds(h, cls, kernel, grid, block, 0, args...);
}

// row-major [n][W][np2] -> sliced-ELL layout of the level
template <typename T>
std::vector<T> to_sliced(const std::vector<T>& src, const Level& L, int W, int np2) {
  const int64_t ns = L.slices();
  std::vector<T> out((size_t)L.slice_blk[ns] * np2, T(0));
  for (int64_t r = 0; r < L.n; ++r) {
    const int64_t s = r / SLICE, lane = r % SLICE, B = L.slice_blk[s];
    for (int w = 0; w < W; ++w)
      for (int ij = 0; ij < np2; ++ij)
        out[(size_t)(B + SLICE * w) * np2 + (size_t)ij * SLICE + lane] = src[((size_t)r * W + w) * np2 + ij];
  }
  return out;
}

// row-major [n][np2] -> per-row layout
template <typename T>
std::vector<T> to_rows(const std::vector<T>& src, int64_t n, int np2) {
  const int64_t ns = (n + SLICE - 1) / SLICE;
  std::vector<T> out((size_t)ns * SLICE * np2, T(0));
  for (int64_t r = 0; r < n; ++r)
    for (int ij = 0; ij < np2; ++ij)
      out[(size_t)(r / SLICE) * SLICE * np2 + (size_t)ij * SLICE + r % SLICE] = src[(size_t)r * np2 + ij];
  return out;
}

int check_flag(cdgmg_handle* h, int* flag, int code, const char* what) {
  HIPCHK(hipMemcpyAsync(h->herr, flag, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (*h->herr) {
    *h->herr = 0;
    HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), h->stream));
    set_error(what);
    return code;
  }
  return CDGMG_OK;
}
int check_err(cdgmg_handle* h, int code, const char* what) { return check_flag(h, h->err, code, what); }

// Work of an operator build that is off its critical chain (assembly ->
// Galerkin products level by level -> coarsest inverse) runs on the handle's
// second stream: fork() sends the following launches there after all work
// enqueued so far, back() returns to the main stream, and the join (at
// destruction of the guard, so on every return path) makes the main stream
// wait for the side work.  Without a second stream all of it stays in order
// on the main stream.
struct SideWork {
  cdgmg_handle* h;
  hipStream_t main;
  bool used = false;
  explicit SideWork(cdgmg_handle* hh) : h(hh), main(hh->stream) {}
  bool on() const { return h->side != nullptr; }
  void fork() {
    if (!on()) return;
    (void)hipEventRecord(h->ev_fork, main);
    (void)hipStreamWaitEvent(h->side, h->ev_fork, 0);
    h->stream = h->side;
    used = true;
  }
  void back() { h->stream = main; }
  void join() {
    h->stream = main;
    if (!used) return;
    (void)hipEventRecord(h->ev_join, h->side);
    (void)hipStreamWaitEvent(main, h->ev_join, 0);
    used = false;
  }
  ~SideWork() { join(); }
};

// ---------------------------------------------------------------- device setup
// Flux-form coarsening: device arrays for M_l, M_l^{-1}, G_l, X, Y per level and
// the host plans translated into (pointer, stride) terms.
int upload_flux(cdgmg_handle* h) {
  Problem& P = h->P;
  const int np = P.np, np2 = np * np, d = P.d;
  for (int l = 0; l <= P.L; ++l) {
    DLevel& D = h->lv[l];
    RETURN_IF(dalloc(h, &D.Mbm, (size_t)D.n * np2));
    RETURN_IF(dalloc(h, &D.Minv, (size_t)D.n * np2));
  }
  RETURN_IF(upload(h, &h->lv[0].G, P.G0));
  for (int l = 0; l < P.L; ++l) {
    const FluxPlan& F = P.fp[l];
    DLevel &D = h->lv[l], &C = h->lv[l + 1];
    D.nX = (int64_t)F.x_col.size();
    D.nY = (int64_t)F.y_col.size();
    RETURN_IF(dalloc(h, &D.X, (size_t)d * D.nX * np2));
    RETURN_IF(dalloc(h, &D.Y, (size_t)d * D.nY * np2));
    C.G = D.Y;
  }
  for (int l = 0; l < P.L; ++l) {
    const FluxPlan& F = P.fp[l];
    DLevel &D = h->lv[l], &C = h->lv[l + 1];
    const int64_t nG = (int64_t)F.g_col.size();
    auto ref = [&](const OpRef& o, const double** ptr, int32_t* stride) {
      *stride = 1;
      switch (o.kind) {
        case OP_L:
          *ptr = D.L64 + (o.idx / SLICE) * SLICE * np2 + (o.idx % SLICE);
          *stride = SLICE;
          break;
        case OP_G: *ptr = D.G + ((size_t)o.comp * nG + o.idx) * np2; break;
        case OP_X: *ptr = D.X + ((size_t)o.comp * D.nX + o.idx) * np2; break;
        case OP_Y: *ptr = D.Y + ((size_t)o.comp * D.nY + o.idx) * np2; break;
        case OP_MINV: *ptr = D.Minv + (size_t)o.idx * np2; break;
        case OP_MINVC: *ptr = C.Minv + (size_t)o.idx * np2; break;
        case OP_M: *ptr = D.Mbm + (size_t)o.idx * np2; break;
        default: *ptr = nullptr; break;
      }
    };
    auto terms = [&](const std::vector<TPTerm>& src, TPDev** dst) {
      std::vector<TPDev> v(src.size());
      for (size_t q = 0; q < src.size(); ++q) {
        ref(src[q].P, &v[q].P, &v[q].sp);
        ref(src[q].Q, &v[q].Q, &v[q].sq);
        ref(src[q].R, &v[q].R, &v[q].sr);
        v[q].pad = 0;
        v[q].sign = src[q].sign;
      }
      return upload(h, dst, v);
    };
    std::vector<TPOut> outs;
    // X outputs (component-major), Y outputs, M_{l+1} rows, A_{l+1} blocks
    outs.resize((size_t)d * D.nX);
    for (size_t o = 0; o < outs.size(); ++o) outs[o] = TPOut{D.X + o * np2, 1};
    RETURN_IF(upload(h, &D.xo, outs));
    RETURN_IF(upload(h, &D.xpp, F.xp_ptr));
    RETURN_IF(terms(F.xp, &D.xp));
    D.nxo = (int64_t)outs.size();
    outs.resize((size_t)d * D.nY);
    for (size_t o = 0; o < outs.size(); ++o) outs[o] = TPOut{D.Y + o * np2, 1};
    RETURN_IF(upload(h, &D.yo, outs));
    RETURN_IF(upload(h, &D.ypp, F.yp_ptr));
    RETURN_IF(terms(F.yp, &D.yp));
    D.nyo = (int64_t)outs.size();
    outs.resize((size_t)C.n);
    for (size_t o = 0; o < outs.size(); ++o) outs[o] = TPOut{C.Mbm + o * np2, 1};
    RETURN_IF(upload(h, &D.mo, outs));
    RETURN_IF(upload(h, &D.mpp, F.mp_ptr));
    RETURN_IF(terms(F.mp, &D.mp));
    D.nmo = (int64_t)outs.size();
    const Level& H = P.lv[l + 1];
    outs.resize((size_t)H.nnzb);
    for (int64_t I = 0; I < H.n; ++I)
      for (int64_t t = 0; t < H.row_len[I]; ++t)
        outs[H.row_blk[I] + t] =
            TPOut{C.A64 + (H.slice_blk[I / SLICE] + (int64_t)SLICE * t) * np2 + (I % SLICE), SLICE};
    RETURN_IF(upload(h, &D.so, outs));
    RETURN_IF(upload(h, &D.spp, F.sp_ptr));
    RETURN_IF(terms(F.sp, &D.sp));
    D.nso = (int64_t)outs.size();
  }
  std::vector<FluxPlan>().swap(P.fp);
  std::vector<double>().swap(P.G0);
  return CDGMG_OK;
}

int upload_problem(cdgmg_handle* h) {
  Problem& P = h->P;
  const int np = P.np, np2 = np * np;
  h->np = np;
  h->d = P.d;
  h->W0 = P.nf + 1;
  h->L = P.L;
  h->N0 = P.N0;
  h->lv.assign(P.L + 1, DLevel());
  const bool fp32 = h->o.mg_precision == CDGMG_MG_FP32;
  h->sym0 = P.beta == 0.0;
  const int npk = h->sym0 ? np * (np + 1) / 2 : np2;  // values per level-0 per-row block
  for (int l = 0; l <= P.L; ++l) {
    Level& H = P.lv[l];
    DLevel& D = h->lv[l];
    D.n = H.n;
    D.ns = H.slices();
    D.slots = H.slice_blk[D.ns];
    D.nnzb = H.nnzb;
    RETURN_IF(upload(h, &D.cols, H.cols));
    RETURN_IF(upload(h, &D.sblk, H.slice_blk));
    RETURN_IF(upload(h, &D.perm, H.perm));
    RETURN_IF(dalloc(h, &D.A64, (size_t)D.slots * np2));
    RETURN_IF(dzero(h, D.A64, (size_t)D.slots * np2 * sizeof(double)));
    const size_t rowblk = (size_t)D.ns * SLICE * np2;
    const size_t rowblk0 = (size_t)D.ns * SLICE * npk;  // level 0: packed when symmetric
    if (l == 0 && h->inner) {  // hp front end: level 0 restricts to the lower degree
      RETURN_IF(dalloc(h, &D.D64, rowblk));
      void* tmp;
      if (fp32) {
        RETURN_IF(dalloc(h, (char**)&tmp, rowblk0 * sizeof(float)));
        D.Dm = tmp;
      } else if (h->sym0) {
        RETURN_IF(dalloc(h, (char**)&tmp, rowblk0 * sizeof(double)));
        D.Dm = tmp;
      } else {
        D.Dm = D.D64;
      }
    }
    if (l < P.L) {
      RETURN_IF(dalloc(h, &D.D64, rowblk));
      std::vector<double> Lr = to_rows(H.Lblk, H.n, np2);
      RETURN_IF(upload(h, &D.L64, Lr));
      if (l == 0) {  // the V-cycle's level-0 transfers form L_e on the fly
        const int na = P.d + P.d * P.d;
        if (P.aff0.size() != (size_t)H.n * na || P.lv[1].bcoef.size() != (size_t)P.lv[1].n * np2) {
          set_error("setup: the level-0 element maps are missing");
          return CDGMG_ERR_HIERARCHY;
        }
        std::vector<double> Ar = to_rows(P.aff0, H.n, na);
        const std::vector<double>& C1 = P.lv[1].bcoef;
        if (fp32) {
          float* tmp;
          RETURN_IF(upload(h, &tmp, std::vector<float>(Ar.begin(), Ar.end())));
          D.Aff = tmp;
          RETURN_IF(upload(h, &tmp, std::vector<float>(C1.begin(), C1.end())));
          D.Cp = tmp;
        } else {
          double* tmp;
          RETURN_IF(upload(h, &tmp, Ar));
          D.Aff = tmp;
          RETURN_IF(upload(h, &tmp, C1));
          D.Cp = tmp;
        }
        std::vector<double>().swap(P.aff0);
      }
      if (fp32) {
        float* tmp;
        if (l > 0) {
          RETURN_IF(upload(h, &tmp, std::vector<float>(Lr.begin(), Lr.end())));
          D.Lm = tmp;
        }
        RETURN_IF(dalloc(h, &tmp, l == 0 ? rowblk0 : rowblk));
        D.Dm = tmp;
        if (l > 0) {
          RETURN_IF(dalloc(h, &tmp, rowblk));
          D.Lt = tmp;
        }
      } else {
        D.Lm = D.L64;
        D.Dm = D.D64;
        if (l == 0 && h->sym0) {
          double* tmp;
          RETURN_IF(dalloc(h, &tmp, rowblk0));
          D.Dm = tmp;
        }
        if (l > 0) {
          double* tmp;
          RETURN_IF(dalloc(h, &tmp, rowblk));
          D.Lt = tmp;
        }
      }
      RETURN_IF(upload(h, &D.parent, H.parent));
    }
    if (l == 0) {
      // facet-trace form of the off-diagonal blocks: the kind of each slot
      // (the neighbour's local facet when this row hosts it, else n_f)
      const int nf = P.nf, W = P.nf + 1;
      std::vector<int8_t> meta((size_t)D.ns * nf * SLICE, 0);
      for (int64_t r = 0; r < D.n; ++r)
        for (int w = 0; w < nf; ++w) {
          const int hf = P.hostflag[r * W + w + 1];
          meta[((r / SLICE) * nf + w) * SLICE + r % SLICE] =
              (int8_t)(hf == 1 ? P.revslot[r * W + w + 1] - 1 : hf == 0 ? nf : 0);
        }
      RETURN_IF(upload(h, &D.meta, meta));
      const size_t nc = (size_t)D.ns * SLICE * nf * np * fnodes(np, nf);
      const bool smooth = P.L > 0 || h->inner;
      if (!h->given_A0 || (smooth && !fp32)) RETURN_IF(dalloc(h, &h->A0c, nc));
      if (!h->given_A0 && h->sym0) RETURN_IF(dalloc(h, &h->A0d, rowblk0));
      if (smooth) {
        if (fp32) {
          float* tmp;
          RETURN_IF(dalloc(h, &tmp, nc));
          D.Ac = tmp;
          RETURN_IF(dalloc(h, &tmp, rowblk0));
          D.Ad = tmp;
        } else {
          D.Ac = h->A0c;
          double* tmp;
          RETURN_IF(dalloc(h, &tmp, rowblk0));
          D.Ad = tmp;
        }
      }
    }
    if (l >= 1 && l < P.L) {
      std::vector<int32_t> wc(H.nnzb);
      for (int64_t r = 0; r < H.n; ++r)
        for (int w = 0; w < H.row_len[r]; ++w)
          wc[H.row_blk[r] + w] = H.cols[H.slice_blk[r / SLICE] + (int64_t)SLICE * w + r % SLICE];
      RETURN_IF(upload(h, &D.wcols, wc));
      RETURN_IF(upload(h, &D.woff, H.row_blk));
      const size_t nr = (size_t)(H.nnzb - H.n) * np2;
      void* tmp;
      RETURN_IF(dalloc(h, (char**)&tmp, nr * (fp32 ? sizeof(float) : sizeof(double))));
      D.R = tmp;
      // lanes per row by the mean strip width (measured: 32 for the n_p = 10
      // strips of about 60 columns of the 2D p = 3 hierarchy, at every level
      // and for both kernels; 64 for the n_p = 20 strips of 3D p = 3)
      const double kmean = (double)(H.nnzb - H.n) * np / std::max<int64_t>(H.n, 1);
      if (h->o.coarse_group)
        D.grp_s = D.grp_r = h->o.coarse_group;
      else
        D.grp_s = D.grp_r = kmean <= 192 ? 32 : 64;
    }
    if (l >= 1) {
      std::vector<int32_t> cs(H.child_start.begin(), H.child_start.end());
      RETURN_IF(upload(h, &D.child_start, cs));
      std::vector<int32_t> brow(H.nnzb);
      for (int64_t I = 0; I < H.n; ++I)
        for (int64_t k = H.row_blk[I]; k < H.row_blk[I + 1]; ++k) brow[k] = (int32_t)I;
      RETURN_IF(upload(h, &D.blk_row, brow));
      RETURN_IF(upload(h, &D.row_blk, H.row_blk));
      RETURN_IF(upload(h, &D.plan_ptr, H.plan_ptr));
      RETURN_IF(upload(h, &D.plan_e, H.plan_e));
      // each plan entry's fine block (e, w): its offset in the sliced fine
      // operator and its column, resolved once here (kappa-independent), so
      // that the Galerkin kernel's loads wait on one index load, not three
      const Level& F = P.lv[l - 1];
      std::vector<int32_t> pc(H.plan_e.size());
      std::vector<int64_t> pa(H.plan_e.size());
      for (size_t q = 0; q < pc.size(); ++q) {
        const int64_t e = H.plan_e[q], B = F.slice_blk[e / SLICE] + (int64_t)SLICE * H.plan_w[q];
        pc[q] = F.cols[B + e % SLICE];
        pa[q] = B * np2 + e % SLICE;
      }
      RETURN_IF(upload(h, &D.plan_c, pc));
      RETURN_IF(upload(h, &D.plan_a, pa));
    }
    const size_t vb = (size_t)D.ns * SLICE * np * sizeof(double);
    double* tmp;
    RETURN_IF(dalloc(h, &tmp, vb / sizeof(double)));
    D.b = tmp;
    RETURN_IF(dalloc(h, &tmp, vb / sizeof(double)));
    D.x = tmp;
    RETURN_IF(dalloc(h, &tmp, vb / sizeof(double)));
    D.xb = tmp;
    RETURN_IF(dalloc(h, &tmp, vb / sizeof(double)));
    D.t = tmp;
    // padding entries past n n_p stay zero (the dense coarsest product reads them)
    for (void* v : {D.b, D.x, D.xb, D.t}) RETURN_IF(dzero(h, v, vb));
  }
  // level-0 kappa-free blocks (a level 0 set by its owner needs none of them)
  if (!h->given_A0) {
    RETURN_IF(upload(h, &h->UA, to_sliced(P.UA, P.lv[0], h->W0, np2)));
    RETURN_IF(upload(h, &h->UH, to_sliced(P.UH, P.lv[0], h->W0, np2)));
    RETURN_IF(upload(h, &h->hostflag, P.hostflag));
    RETURN_IF(upload(h, &h->revslot, P.revslot));
    RETURN_IF(upload(h, &h->M, to_rows(P.Mblk, P.N0, np2)));
  }
  if (!P.UC.empty()) {
    RETURN_IF(upload(h, &h->UC, to_sliced(P.UC, P.lv[0], h->W0, np2)));
    RETURN_IF(dalloc(h, &h->Atmp, (size_t)h->lv[0].slots * np2));
    RETURN_IF(dzero(h, h->Atmp, (size_t)h->lv[0].slots * np2 * sizeof(double)));  // padding rows stay zero
    std::vector<double>().swap(P.UC);
  }
  RETURN_IF(dalloc(h, &h->kappa, P.N0));
  if (!h->inner) {
    // coarsest dense
    h->nd = h->lv[P.L].n * np;
    if (h->nd > 12000) {
      set_error("setup: coarsest level has " + std::to_string(h->nd) + " unknowns (limit 12000); use more levels");
      return CDGMG_ERR_ARG;
    }
    h->ld = (h->nd + GJB - 1) / GJB * GJB;
    RETURN_IF(dalloc(h, &h->dense, (size_t)h->ld * h->ld));
    RETURN_IF(dalloc(h, &h->gjP, (size_t)GJB * GJB));
    RETURN_IF(dalloc(h, &h->gjR, (size_t)GJB * h->ld));
    RETURN_IF(dalloc(h, &h->gjK, (size_t)GJB * h->ld));
    RETURN_IF(dalloc(h, &h->gjC, (size_t)GJB * h->ld));
    RETURN_IF(dalloc(h, &h->gjD, (size_t)h->ld));
    if (fp32 && !h->o.coarse_fp64) {
      float* tmp;
      RETURN_IF(dalloc(h, &tmp, (size_t)h->nd * h->ld));
      h->AinvP = tmp;
    } else {
      h->AinvP = h->dense;
    }
  }
  // outer vectors; a lower hp level runs only its V-cycle and level products,
  // which use t1 and t2
  const size_t m = (size_t)h->lv[0].ns * SLICE * np;
  for (double** v : {&h->b, &h->x, &h->xl, &h->r, &h->p, &h->q, &h->t1, &h->t2}) {
    if (h->given_A0 && v != &h->t1 && v != &h->t2) continue;
    RETURN_IF(dalloc(h, v, m));
    RETURN_IF(dzero(h, *v, m * sizeof(double)));
  }
  if (h->o.outer == CDGMG_OUTER_GMRES) {
    const int R = h->o.restart;
    h->gm_ld = (int64_t)m;
    RETURN_IF(dalloc(h, &h->gmV, (size_t)(R + 1) * m));
    RETURN_IF(dalloc(h, &h->gmZ, (size_t)R * m));
    RETURN_IF(dalloc(h, &h->gmH, 3 * (size_t)(R + 1)));
    RETURN_IF(dalloc(h, &h->gmPart, (size_t)(R + 1) * 1024));
    RETURN_IF(dalloc(h, &h->gmY, (size_t)R));
    RETURN_IF(dzero(h, h->gmV, (size_t)(R + 1) * m * sizeof(double)));
    RETURN_IF(dzero(h, h->gmZ, (size_t)R * m * sizeof(double)));
    RETURN_IF(host_alloc(h, &h->hgmH, 3 * (size_t)(R + 1)));
    RETURN_IF(host_alloc(h, &h->hgmY, (size_t)R));
  }
  RETURN_IF(dalloc(h, &h->scal, SC_N));
  h->nparts = (int)std::max<int64_t>(1024, (P.N0 + SLICE - 1) / SLICE + 1);
  RETURN_IF(dalloc(h, &h->part, 2 * (size_t)h->nparts));
  RETURN_IF(dalloc(h, &h->err, 1));
  RETURN_IF(dzero(h, h->err, sizeof(int)));
  RETURN_IF(dalloc(h, &h->err_side, 1));
  RETURN_IF(dzero(h, h->err_side, sizeof(int)));
  RETURN_IF(host_alloc(h, &h->hscal, SC_N));
  RETURN_IF(host_alloc(h, &h->herr, 1));
  if (P.flux) RETURN_IF(upload_flux(h));
  // release large host copies that the device now holds
  std::vector<double>().swap(P.UA);
  std::vector<double>().swap(P.UH);
  std::vector<double>().swap(P.Gblk);
  for (auto& H : P.lv) {
    std::vector<double>().swap(H.Lblk);
    std::vector<int32_t>().swap(H.plan_e);
    std::vector<int32_t>().swap(H.plan_w);
  }
  return CDGMG_OK;
}

#define NF_DISPATCH(nfv, ...)                                                   \
  switch (nfv) {                                                                \
    case 3: { constexpr int NF = 3; if constexpr (l0_pair(NP, NF)) { __VA_ARGS__; } } break; \
    case 4: { constexpr int NF = 4; if constexpr (l0_pair(NP, NF)) { __VA_ARGS__; } } break; \
    default: break;                                                             \
  }

// the off-diagonal blocks of the sliced A_0 (FP64) in facet-trace form, in T;
// the dropped entries are checked to be zero (err)
template <typename T, int NP>
void compress0(cdgmg_handle* h, T* out, int* err) {
  DLevel& D = h->lv[0];
  NF_DISPATCH(h->P.nf, {
    constexpr int NPF = NP * FacetTab<NP, NF>::NFN;
    launch(h, -1, k_compress0<T, NP, NF>, dim3(grid_for(D.ns * NF * NPF * WAVE)), dim3(TPB), D.n, D.ns,
           (const double*)D.A64, (const int8_t*)D.meta, out, err);
  });
}

// level 0 of the V-cycle in precision T: off-diagonal blocks in facet-trace
// form (in FP64 mode the outer loop's copy), diagonal blocks, D^{-1}
template <typename T, int NP>
void level0_operators(cdgmg_handle* h) {
  constexpr int NP2 = NP * NP;
  DLevel& D = h->lv[0];
  if ((void*)D.Ac != (void*)h->A0c) {
    if (h->A0c) {  // the FP64 facet-trace copy, compressed and checked already: same layout
      const int64_t nc = D.ns * SLICE * h->P.nf * NP * fnodes(NP, h->P.nf);
      launch(h, -1, k_cast<double, T>, dim3(grid_for(nc)), dim3(TPB), nc, (const double*)h->A0c, (T*)D.Ac);
    } else {
      compress0<T, NP>(h, (T*)D.Ac, h->err);
    }
  }
  if (h->sym0) {  // upper triangles of the diagonal blocks and of D^{-1}
    constexpr int NPK = RowBlk<NP, true>::N;
    const int64_t nt = D.ns * NPK * WAVE;
    launch(h, -1, k_pack_sym<T, NP>, dim3(grid_for(nt)), dim3(TPB), D.ns, (int64_t)(h->P.nf + 1) * NP2,
           (const double*)D.A64, (T*)D.Ad);
    launch(h, -1, k_pack_sym<T, NP>, dim3(grid_for(nt)), dim3(TPB), D.ns, (int64_t)NP2, (const double*)D.D64,
           (T*)D.Dm);
    return;
  }
  NF_DISPATCH(h->P.nf, launch(h, -1, k_diag0<T, NP, NF>, dim3(grid_for(D.ns * NP2 * WAVE)), dim3(TPB), D.ns,
                              (const double*)D.A64, (T*)D.Ad));
  if ((void*)D.Dm != (void*)D.D64) {
    const int64_t nb = D.ns * SLICE * NP2;
    launch(h, -1, k_cast<double, T>, dim3(grid_for(nb)), dim3(TPB), nb, (const double*)D.D64, (T*)D.Dm);
  }
}

// the outer loop's FP64 diagonal blocks of A_0, packed (symmetric operator)
template <int NP>
void pack_outer_diag(cdgmg_handle* h) {
  if (!h->A0d) return;
  DLevel& D = h->lv[0];
  const int64_t nt = D.ns * RowBlk<NP, true>::N * WAVE;
  launch(h, -1, k_pack_sym<double, NP>, dim3(grid_for(nt)), dim3(TPB), D.ns, (int64_t)(h->P.nf + 1) * NP * NP,
         (const double*)D.A64, h->A0d);
}

// hp front end, level 0 at degree p: D^{-1}, the next p-level's operator
// T^T A_0 T, the whole lower-degree hierarchy, and the level-0 V-cycle
// operators (the restriction uses the constant embedding T)
template <typename T, int NP0, int NP1>
void prescale_hp(cdgmg_handle* h) {
  level0_operators<T, NP0>(h);
}

int build_operators(cdgmg_handle* h, const double* kappa_dev, bool transposed);

// D^{-1} of every diagonal block of a level (K8): one thread per row up to
// n_p = 10, a group of lanes per row above
template <int NP>
void diag_inverse(cdgmg_handle* h, DLevel& L, int definite) {
  if constexpr (NP <= 10)
    launch(h, -1, k_diag_inverse<NP>, dim3(grid_for(L.n)), dim3(TPB), L.n, (const int64_t*)L.sblk,
           (const double*)L.A64, L.D64, h->err, definite);
  else
    launch(h, -1, k_diag_inverse_cols<NP>, dim3(grid_for(L.n * DIG)), dim3(TPB), L.n, (const int64_t*)L.sblk,
           (const double*)L.A64, L.D64, h->err, definite);
}

int build_hp(cdgmg_handle* h) {
  DLevel& l0 = h->lv[0];
  cdgmg_handle* in = h->inner;
  NP_DISPATCH(h->np, diag_inverse<NP>(h, l0, 1));
  RETURN_IF(check_err(h, CDGMG_ERR_SINGULAR, "setup: a diagonal block is not positive definite"));
  const int64_t tot = l0.ns * h->W0 * (int64_t)h->np1 * h->np1 * WAVE;
  HP_DISPATCH(h->np, h->np1, launch(h, -1, k_galerkin_p<NP0, NP1>, dim3(grid_for(tot)), dim3(TPB), l0.ns, h->W0,
                                    (const double*)l0.A64, (const double*)h->Tp64, in->lv[0].A64));
  RETURN_IF(build_operators(in, nullptr, false));
  if (h->o.mg_precision == CDGMG_MG_FP32) {
    HP_DISPATCH(h->np, h->np1, prescale_hp<float, NP0, NP1>(h));
  } else {
    HP_DISPATCH(h->np, h->np1, prescale_hp<double, NP0, NP1>(h));
  }
  RETURN_IF(check_err(h, CDGMG_ERR_MESH, "setup: a level-0 off-diagonal block is not in facet-trace form"));
  HIPCHK(hipGetLastError());
  return CDGMG_OK;
}

template <typename T, int NP>
void prescale(cdgmg_handle* h) {
  constexpr int NP2 = NP * NP;
  for (int l = 0; l < h->L; ++l) {
    DLevel& D = h->lv[l];
    if (l == 0) {
      level0_operators<T, NP>(h);
      continue;
    }
    launch(h, -1, k_scale_wpr<T, NP>, dim3(grid_for(D.nnzb * NP2)), dim3(TPB), D.nnzb, (const int32_t*)D.blk_row,
           (const int64_t*)D.sblk, (const int64_t*)D.woff, (const double*)D.A64, (const double*)D.D64, (T*)D.R);
    launch(h, -1, k_scale_L<T, NP>, dim3(grid_for(D.ns * NP2 * WAVE)), dim3(TPB), D.n, (const int64_t*)D.sblk,
           (const double*)D.A64, (const double*)D.L64, (T*)D.Lt);
    if ((void*)D.Dm != (void*)D.D64) {
      const int64_t nb = D.ns * SLICE * NP2;
      launch(h, -1, k_cast<double, T>, dim3(grid_for(nb)), dim3(TPB), nb, (const double*)D.D64, (T*)D.Dm);
    }
  }
}

// kappa -> A_0 -> (D^{-1}, Galerkin) per level -> prescaled V-cycle operators
// -> coarsest inverse.  kappa_dev null: rebuild from the stored kappa.
// transposed: every level holds A_l^T (A_0^T, then the same Galerkin products,
// since (L^T A L)^T = L^T A^T L), for the adjoint of a nonsymmetric operator.
int build_operators(cdgmg_handle* h, const double* kappa_dev, bool transposed) {
  const int np = h->np, np2 = np * np;
  DLevel& l0 = h->lv[0];
  if (kappa_dev) {
    launch(h, -1, k_kappa_perm, dim3(grid_for(h->N0)), dim3(TPB), h->N0, (const int32_t*)l0.perm, kappa_dev,
           h->kappa, h->err);
    RETURN_IF(check_err(h, CDGMG_ERR_ARG, "setup: kappa must be positive and finite"));
  }
  if (!h->given_A0)
    NP_DISPATCH(np, launch(h, -1, k_assemble_A0<NP>, dim3(grid_for(h->N0)), dim3(TPB), h->N0, h->W0,
                           (const int32_t*)l0.cols, (const int64_t*)l0.sblk, (const double*)h->UA,
                           (const double*)h->UH, (const int8_t*)h->hostflag, (const int8_t*)h->revslot,
                           (const double*)h->kappa, (const double*)h->UC, l0.A64));
  if (transposed) {
    NP_DISPATCH(np, launch(h, -1, k_transpose_A0<NP>, dim3(grid_for(h->N0)), dim3(TPB), h->N0, h->W0,
                           (const int64_t*)l0.sblk, (const int32_t*)l0.cols, (const int8_t*)h->revslot,
                           (const double*)l0.A64, h->Atmp));
    HIPCHK(hipMemcpyAsync(l0.A64, h->Atmp, (size_t)l0.slots * np2 * sizeof(double), hipMemcpyDeviceToDevice,
                          h->stream));
  }
  h->transposed = transposed;
  const char* not_trace = "setup: a level-0 off-diagonal block is not in facet-trace form";
  // the facet-trace copy of A_0 (outer loop, and source of the V-cycle's
  // copy) beside the Galerkin chain, which reads the sliced A_0
  // (forked once the level-0 block inverses are enqueued, so that it does not
  // share the device with them), then the prescaled copies beside the
  // coarsest inverse
  SideWork side(h);
  const bool fork = side.on() && h->A0c && !h->inner && h->L > 0;  // forked from the level loop
  if (h->A0c && !fork) {
    NP_DISPATCH(np, compress0<double, NP>(h, h->A0c, h->err));
    RETURN_IF(check_err(h, CDGMG_ERR_MESH, not_trace));
  }
  if (!fork) NP_DISPATCH(np, pack_outer_diag<NP>(h));
  if (h->inner) return build_hp(h);
  const bool flux = h->P.flux;
  // the Galerkin hierarchy of the symmetric Poisson operator is SPD: its
  // pivots must be positive; otherwise they must be nonzero
  const int definite = (flux || h->P.beta != 0.0) ? 0 : 1;
  const int tpb = std::min(1024, ((np2 + 63) / 64) * 64);
  if (flux)
    NP_DISPATCH(np, launch(h, -1, k_mass_kappa<NP>, dim3(grid_for(h->N0)), dim3(TPB), h->N0, (const double*)h->M,
                           (const double*)h->kappa, l0.Mbm));
  for (int l = 0; l < h->L; ++l) {
    DLevel &f = h->lv[l], &c = h->lv[l + 1];
    NP_DISPATCH(np, diag_inverse<NP>(h, f, definite));
    if (l == 0 && fork) {
      side.fork();
      NP_DISPATCH(np, compress0<double, NP>(h, h->A0c, h->err_side));
      NP_DISPATCH(np, pack_outer_diag<NP>(h));
      side.back();
    }
    if (flux) {
      // M_l^{-1}, X = G_l L, Y = L^T X (= G_{l+1}), M_{l+1} = L^T M_l L, M_{l+1}^{-1}
      NP_DISPATCH(np, launch(h, -1, k_block_inverse_bm<NP>, dim3(grid_for(f.n)), dim3(TPB), f.n,
                             (const double*)f.Mbm, f.Minv, h->err));
      NP_DISPATCH(np, launch(h, -1, k_triple<NP>, dim3((unsigned)f.nxo), dim3(tpb), f.nxo, (const TPOut*)f.xo,
                             (const int64_t*)f.xpp, (const TPDev*)f.xp, 0));
      NP_DISPATCH(np, launch(h, -1, k_triple<NP>, dim3((unsigned)f.nyo), dim3(tpb), f.nyo, (const TPOut*)f.yo,
                             (const int64_t*)f.ypp, (const TPDev*)f.yp, 0));
      NP_DISPATCH(np, launch(h, -1, k_triple<NP>, dim3((unsigned)f.nmo), dim3(tpb), f.nmo, (const TPOut*)f.mo,
                             (const int64_t*)f.mpp, (const TPDev*)f.mp, 0));
      NP_DISPATCH(np, launch(h, -1, k_block_inverse_bm<NP>, dim3(grid_for(c.n)), dim3(TPB), c.n,
                             (const double*)c.Mbm, c.Minv, h->err));
    }
    NP_DISPATCH(np, launch(h, -1, k_galerkin<NP>, dim3((unsigned)c.nnzb), dim3(tpb), c.nnzb,
                           (const int32_t*)c.blk_row, (const int64_t*)c.row_blk, (const int64_t*)c.plan_ptr,
                           (const int32_t*)c.plan_e, (const int32_t*)c.plan_c, (const int64_t*)c.plan_a,
                           (const double*)f.A64, (const double*)f.L64, (const int64_t*)c.sblk, c.A64));
    if (flux)  // A_{l+1} += -X^T M_l^{-1} X + Y^T M_{l+1}^{-1} Y
      NP_DISPATCH(np, launch(h, -1, k_triple<NP>, dim3((unsigned)f.nso), dim3(tpb), f.nso, (const TPOut*)f.so,
                             (const int64_t*)f.spp, (const TPDev*)f.sp, 1));
  }
  RETURN_IF(check_err(h, CDGMG_ERR_SINGULAR, flux ? "setup: a diagonal or mass block is singular"
                                                  : "setup: a diagonal block is not positive definite"));
  // coarsest: dense scatter + Gauss-Jordan inverse
  DLevel& cl = h->lv[h->L];
  const int64_t nd = h->nd, ld = h->ld;
  launch(h, -1, k_dense_init, dim3(grid_for(ld * ld)), dim3(TPB), nd, ld, h->dense);
  NP_DISPATCH(np, launch(h, -1, k_dense_scatter<NP>, dim3(grid_for(cl.n * np2)), dim3(TPB), cl.n, ld,
                         (const int32_t*)cl.cols, (const int64_t*)cl.sblk, (const double*)cl.A64, h->dense));
  launch(h, -1, k_dense_diag, dim3(grid_for(ld)), dim3(TPB), ld, (const double*)h->dense, h->gjD);
  // prescaled V-cycle operators D^{-1} A (off-diagonal), D^T L_e, and D^{-1} in the
  // multigrid precision, beside the inverse
  if (fork) side.fork();
  if (h->o.mg_precision == CDGMG_MG_FP32) {
    NP_DISPATCH(np, prescale<float, NP>(h));
  } else {
    NP_DISPATCH(np, prescale<double, NP>(h));
  }
  side.back();
  if (!fork) RETURN_IF(check_err(h, CDGMG_ERR_MESH, not_trace));
  const int nbk = (int)(ld / GJB);
  for (int K = 0; K < nbk; ++K) {
    launch(h, -1, k_gj_pivot, dim3(1), dim3(GJT), ld, K, h->dense, h->gjP, (const double*)h->gjD, h->err,
           definite);
    if (nbk > 1) {
      launch(h, -1, k_gj_panels, dim3(2 * nbk), dim3(256), ld, K, nbk, (const double*)h->dense,
             (const double*)h->gjP, h->gjR, h->gjK, h->gjC);
      launch(h, -1, k_gj_update, dim3(nbk, nbk), dim3(256), ld, K, h->dense, (const double*)h->gjR,
             (const double*)h->gjK, (const double*)h->gjC);
    }
  }
  side.join();
  if (fork) RETURN_IF(check_flag(h, h->err_side, CDGMG_ERR_MESH, not_trace));
  RETURN_IF(check_err(h, CDGMG_ERR_SINGULAR, flux ? "setup: the coarsest operator is singular"
                                                  : "setup: the coarsest operator is not positive definite"));
  if (h->o.mg_precision == CDGMG_MG_FP32 && !h->o.coarse_fp64)
    launch(h, -1, k_cast<double, float>, dim3(grid_for(nd * ld)), dim3(TPB), nd * ld, (const double*)h->dense,
           (float*)h->AinvP);
  HIPCHK(hipGetLastError());
  return CDGMG_OK;
}

// ---------------------------------------------------------------- V-cycle
// wavefronts per 64-row slice of the level-0 kernels: 0 picks by n_p (one
// wavefront per slice up to n_p = 10; the n_p = 20 rows are split in two,
// measured fastest on the 3D p = 3 workload)
// wavefronts per 64-row slice of the level-0 kernels: one unless the option
// asks otherwise (measured fastest at every n_p); the compensated outer
// kernels (comp) at n_p = 20 hold too many double-double accumulators for one
// wavefront per slice (they spill) and take two
int pick_h0(int np, int variant, bool comp = false) {
  if (variant == 0) return comp && np >= 20 ? 2 : 1;
  if ((variant == 1 || variant == 2 || variant == 4 || variant == 5) && np % variant == 0) return variant;
  return 0;
}

// count damped block-Jacobi sweeps on level l (ping-pong x <-> xb); with dv
// given, the last level-0 sweep also leaves the partial sums of (x, dv) in
// h->part, one per slice; with xf given (l >= 1), the last sweep also
// prolongs into level l - 1, x_{l-1} += L x_l (xf = x_{l-1})
template <typename T, int NP>
void smooth_sweeps(cdgmg_handle* h, int l, int count, T** x, T** xb, const double* dv = nullptr,
                   T* xf = nullptr) {
  DLevel& d = h->lv[l];
  const T omega = (T)h->o.omega;
  const int cls = l == 0 && !h->given_A0 ? CDGMG_K_SMOOTH0 : CDGMG_K_SMOOTH;
  for (int s = 0; s < count; ++s) {
    if (l == 0) {
      const bool dot = dv && s == count - 1;
      const int rev = h->at_pass++ & 1;
      if (dot) {
        L0_DISPATCH(h, launch(h, cls, k_sweep0<T, NP, H, NF, true, SYM>, dim3((unsigned)d.ns), dim3(WAVE * H), d.n,
                              (const int32_t*)d.cols, (const int8_t*)d.meta, (const T*)d.Ac, (const T*)d.Dm,
                              (const T*)d.b, (const T*)*x, omega, *xb, dv, h->part, rev));
      } else {
        L0_DISPATCH(h, launch(h, cls, k_sweep0<T, NP, H, NF, false, SYM>, dim3((unsigned)d.ns), dim3(WAVE * H), d.n,
                              (const int32_t*)d.cols, (const int8_t*)d.meta, (const T*)d.Ac, (const T*)d.Dm,
                              (const T*)d.b, (const T*)*x, omega, *xb, (const double*)nullptr, (double*)nullptr,
                              rev));
      }
    } else if (xf && s == count - 1) {
      G_DISPATCH(d.grp_s, launch(h, cls, k_sweep_grp<T, NP, G, true>, dim3(grid_for(d.n * G)), dim3(TPB), d.n,
                                 (const int32_t*)d.wcols, (const int64_t*)d.woff, (const T*)d.R, (const T*)d.b,
                                 (const T*)*x, omega, *xb, (const int32_t*)d.child_start,
                                 (const T*)h->lv[l - 1].Lm, xf));
    } else {
      G_DISPATCH(d.grp_s, launch(h, cls, k_sweep_grp<T, NP, G>, dim3(grid_for(d.n * G)), dim3(TPB), d.n,
                                 (const int32_t*)d.wcols, (const int64_t*)d.woff, (const T*)d.R, (const T*)d.b,
                                 (const T*)*x, omega, *xb, (const int32_t*)nullptr, (const T*)nullptr,
                                 (T*)nullptr));
    }
    std::swap(*x, *xb);
  }
}

// partial sums of (z, dv) into h->part
template <typename T>
void dot_t(cdgmg_handle* h, const T* z, const double* dv, int* nparts) {
  const int64_t m = h->N0 * h->np;
  const unsigned g = std::min<unsigned>(1024, grid_for(m));
  launch(h, CDGMG_K_VECTOR, k_dot_t<T>, dim3(g), dim3(TPB), m, z, dv, h->part);
  *nparts = (int)g;
}

// thread-per-row kernels: one-wavefront workgroups on small levels spread the
// few wavefronts over the compute units
// LDS of the one-launch coarsest level (its padded right-hand side)
constexpr size_t COARSEST_LDS = 48 * 1024;

inline int row_tpb(const cdgmg_handle* h, int l) {
  (void)l;
  return h->o.row_threads ? h->o.row_threads : WAVE;
}

void* vcycle(cdgmg_handle* h, const double* r64, const double* dv, int* nparts);

// x = A_L^{-1} b on the coarsest level, the inverse in the multigrid precision
// or, with coarse_fp64 in the FP32 cycle, in FP64
template <typename T>
void coarse_solve(cdgmg_handle* h, const T* b, T* x) {
  if constexpr (sizeof(T) == 4) {
    if (h->o.coarse_fp64) {
      launch(h, CDGMG_K_COARSE, k_dense_gemv_mixed, dim3(grid_for(h->nd * WAVE)), dim3(TPB), h->nd, h->ld,
             (const double*)h->dense, (const float*)b, (float*)x);
      return;
    }
  }
  launch(h, CDGMG_K_COARSE, k_dense_gemv<T>, dim3(grid_for(h->nd * WAVE)), dim3(TPB), h->nd, h->ld,
         (const T*)h->AinvP, b, x);
}

// hp front end: the degree-p level 0 smooths, restricts to the lower-degree
// space (D^T T)^T (D^{-1} r), calls the lower hierarchy's V-cycle and prolongs
// x += T z (Sec. 4, hp paragraph)
template <typename T, int NP>
T* vcycle_hp(cdgmg_handle* h, const double* r64, const double* dv, int* nparts, T* x, T* xb) {
  DLevel& d = h->lv[0];
  const T omega = (T)h->o.omega;
  const int nu1 = h->o.nu1, nu2 = h->o.nu2;
  const T w1 = nu1 > 0 ? omega : T(0);
  cdgmg_handle* in = h->inner;
  L0_DISPATCH(h, launch(h, CDGMG_K_SMOOTH, k_entry0<T, NP, H, SYM>, dim3((unsigned)d.ns), dim3(WAVE * H), d.n, r64,
                        (const T*)d.Dm, w1, (T*)d.b, x));
  smooth_sweeps<T, NP>(h, 0, nu1 > 1 ? nu1 - 1 : 0, &x, &xb);
  const int rev = h->at_pass++ & 1;
  HP_DISPATCH(NP, h->np1, L0_DISPATCH(h, launch(h, CDGMG_K_RESTRICT, k_restrict0_rect<T, NP0, NP1, H, NF, SYM>,
                                                dim3((unsigned)d.ns), dim3(WAVE * H), d.n, (const int32_t*)d.cols,
                                                (const int8_t*)d.meta, (const T*)d.Ac, (const T*)d.Ad,
                                                (const T*)d.b, (const T*)x, (const T*)h->Tpm, in->t1, rev)));
  void* zin = vcycle(in, in->t1, nullptr, nullptr);
  HP_DISPATCH(NP, h->np1, launch(h, CDGMG_K_PROLONG, k_prolong_rect<T, NP0, NP1>, dim3(grid_for(d.n)), dim3(TPB),
                                 d.n, (const T*)h->Tpm, (const T*)zin, x));
  smooth_sweeps<T, NP>(h, 0, nu2, &x, &xb, dv);
  if (dv) {
    if (nu2 > 0)
      *nparts = (int)d.ns;
    else
      dot_t<T>(h, x, dv, nparts);
  }
  return x;
}

// One V-cycle z = B r (Sec. 4): on each level the first pre-smoothing sweep
// starts from zero and is fused with forming D^{-1} b; residual and
// restriction are fused; the coarsest level applies the dense inverse.
// Returns z in the multigrid precision (a level-0 work vector).  With dv
// given, *nparts partial sums of (z, dv) are left in h->part.
template <typename T, int NP>
T* vcycle_t(cdgmg_handle* h, const double* r64, const double* dv, int* nparts) {
  const int L = h->L;
  const T omega = (T)h->o.omega;
  const int nu1 = h->o.nu1, nu2 = h->o.nu2;
  const T w1 = nu1 > 0 ? omega : T(0);
  std::vector<T*> xs(L + 1), xbs(L + 1);
  for (int l = 0; l <= L; ++l) {
    xs[l] = (T*)h->lv[l].x;
    xbs[l] = (T*)h->lv[l].xb;
  }
  if (h->inner) return vcycle_hp<T, NP>(h, r64, dv, nparts, xs[0], xbs[0]);
  if (L == 0) {
    DLevel& d = h->lv[0];
    launch(h, CDGMG_K_VECTOR, k_cast<double, T>, dim3(grid_for(d.n * NP)), dim3(TPB), d.n * NP, r64, (T*)d.b);
    coarse_solve<T>(h, (const T*)d.b, xs[0]);
    if (dv) dot_t<T>(h, xs[0], dv, nparts);
    return xs[0];
  }
  for (int l = 0; l < L; ++l) {
    DLevel& d = h->lv[l];
    if (l == 0) {
      SYM_DISPATCH(h->sym0, H_DISPATCH(h->H0, if constexpr (NP % H == 0) launch(h, CDGMG_K_SMOOTH, k_entry0<T, NP, H, SYM>, 
                                                          dim3((unsigned)d.ns), dim3(WAVE * H), d.n, r64,
                                                          (const T*)d.Dm, w1, (T*)d.b, xs[0])));
    } else {
      const int tpb = row_tpb(h, l);
      launch(h, CDGMG_K_SMOOTH, k_entry_c<T, NP>, dim3(grid_for(d.n, tpb)), dim3(tpb), d.n,
             (const int32_t*)d.child_start, (const T*)h->lv[l - 1].t, (const T*)d.Dm, w1, (T*)d.b, xs[l]);
    }
    smooth_sweeps<T, NP>(h, l, nu1 > 1 ? nu1 - 1 : 0, &xs[l], &xbs[l]);
    if (l == 0) {
      const int rev = h->at_pass++ & 1;
      L0_DISPATCH(h, launch(h, CDGMG_K_RESTRICT, k_restrict0<T, NP, H, NF, SYM>, dim3((unsigned)d.ns), dim3(WAVE * H),
                            d.n, (const int32_t*)d.cols, (const int8_t*)d.meta, (const T*)d.Ac, (const T*)d.Ad,
                            (const T*)d.b, (const T*)xs[0], (const T*)d.Aff, (const int32_t*)d.parent,
                            (const T*)d.Cp, (T*)d.t, rev));
    } else {
      G_DISPATCH(d.grp_r, launch(h, CDGMG_K_RESTRICT, k_restrict_grp<T, NP, G>, dim3(grid_for(d.n * G)), dim3(TPB),
                             d.n, (const int32_t*)d.wcols, (const int64_t*)d.woff, (const T*)d.R, (const T*)d.b,
                             (const T*)xs[l], (const T*)d.Lt, (T*)d.t));
    }
  }
  DLevel& c = h->lv[L];
  // from three levels on, the coarsest level's entry, solve and prolongation
  // into level L - 1 run as one launch (its right-hand side formed in LDS)
  const size_t lds = (size_t)(h->ld + NP) * sizeof(T);
  const bool one = L >= 2 && lds <= COARSEST_LDS;
  if (one) {
    const DLevel& f = h->lv[L - 1];
    const dim3 grid((unsigned)c.n), block((unsigned)std::min(NP, 16) * WAVE);
    bool mixed = false;
    if constexpr (sizeof(T) == 4) {
      if (h->o.coarse_fp64) {
        mixed = true;
        launch_lds(h, CDGMG_K_COARSE, k_coarsest<float, double, NP>, grid, block, lds, c.n, h->ld,
                   (const double*)h->dense, (const int32_t*)c.child_start, (const float*)f.t, (const float*)f.Lm,
                   (float*)xs[L], (float*)xs[L - 1]);
      }
    }
    if (!mixed)
      launch_lds(h, CDGMG_K_COARSE, k_coarsest<T, T, NP>, grid, block, lds, c.n, h->ld, (const T*)h->AinvP,
                 (const int32_t*)c.child_start, (const T*)f.t, (const T*)f.Lm, xs[L], xs[L - 1]);
  } else {
    launch(h, CDGMG_K_COARSE, k_entry_c<T, NP>, dim3(grid_for(c.n, WAVE)), dim3(WAVE), c.n,
           (const int32_t*)c.child_start, (const T*)h->lv[L - 1].t, (const T*)nullptr, omega, (T*)c.b,
           (T*)nullptr);
    coarse_solve<T>(h, (const T*)c.b, xs[L]);
  }
  // upward: the last post-sweep of a level l >= 2 also prolongs into level
  // l - 1, where a separate launch would be bound by its latency (from the
  // coarsest level, into level 0, or with nu2 = 0, a separate launch)
  for (int l = L - 1; l >= 0; --l) {
    DLevel& d = h->lv[l];
    const bool fused = l >= 1 && l + 1 < L && nu2 > 0;
    if (l == 0) {
      const int tpb = row_tpb(h, 0);
      NF_DISPATCH(h->P.nf, launch(h, CDGMG_K_PROLONG, k_prolong0<T, NP, NF>, dim3(grid_for(d.n, tpb)), dim3(tpb),
                                  d.n, (const int32_t*)d.parent, (const T*)d.Aff, (const T*)d.Cp,
                                  (const T*)xs[1], xs[0]));
    } else if (!fused && !(one && l == L - 1)) {
      const int tpb = row_tpb(h, l);
      launch(h, CDGMG_K_PROLONG, k_prolong<T, NP>, dim3(grid_for(d.n, tpb)), dim3(tpb), d.n,
             (const int32_t*)d.parent, (const T*)d.Lm, (const T*)xs[l + 1], xs[l]);
    }
    smooth_sweeps<T, NP>(h, l, nu2, &xs[l], &xbs[l], l == 0 ? dv : nullptr, l >= 2 ? xs[l - 1] : nullptr);
  }
  if (dv) {
    if (nu2 > 0)
      *nparts = (int)h->lv[0].ns;
    else
      dot_t<T>(h, xs[0], dv, nparts);
  }
  return xs[0];
}

// z = B r; returns z in the multigrid precision
void* vcycle(cdgmg_handle* h, const double* r64, const double* dv, int* nparts) {
  void* z = nullptr;
  if (h->o.mg_precision == CDGMG_MG_FP32) {
    NP_DISPATCH(h->np, z = vcycle_t<float, NP>(h, r64, dv, nparts));
  } else {
    NP_DISPATCH(h->np, z = vcycle_t<double, NP>(h, r64, dv, nparts));
  }
  return z;
}

// z64 = B r in FP64 (C ABI)
void vcycle64(cdgmg_handle* h, const double* r64, double* z64) {
  void* z = vcycle(h, r64, nullptr, nullptr);
  const int64_t m = h->N0 * h->np;
  if (h->o.mg_precision == CDGMG_MG_FP32)
    launch(h, CDGMG_K_VECTOR, k_cast<float, double>, dim3(grid_for(m)), dim3(TPB), m, (const float*)z, z64);
  else
    launch(h, CDGMG_K_VECTOR, k_cast<double, double>, dim3(grid_for(m)), dim3(TPB), m, (const double*)z, z64);
}

// ---------------------------------------------------------------- outer solve
void dot_into(cdgmg_handle* h, int64_t m, const double* a, const double* b, int slot) {
  const unsigned g = std::min<unsigned>(1024, grid_for(m));
  launch(h, CDGMG_K_VECTOR, k_dots, dim3(g), dim3(TPB), m, 1, a, b, (const double*)nullptr,
         (const double*)nullptr, h->part);
  launch(h, CDGMG_K_VECTOR, k_reduce, dim3(1), dim3(RED_T), (const double*)h->part, (int)g, 1, h->scal, slot, -1);
}

int read_scalar(cdgmg_handle* h, int slot, double* out) {
  HIPCHK(hipMemcpyAsync(h->hscal + slot, h->scal + slot, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *out = h->hscal[slot];
  return CDGMG_OK;
}

// compensated true residual r = b - A (x_hi + x_lo), written into h->r (the
// recursive residual is replaced by it); ||r||^2 lands in scal[SC_TMP]
void enqueue_true_residual(cdgmg_handle* h) {
  DLevel& d = h->lv[0];
  NP_DISPATCH(h->np, L0C_DISPATCH(h, launch(h, CDGMG_K_VECTOR, k_residual0<NP, H, NF, SYM>, dim3((unsigned)d.ns),
                                            dim3(WAVE * H), d.n, (const int32_t*)d.cols, (const int8_t*)d.meta,
                                            (const double*)(SYM ? h->A0d : d.A64), (const double*)h->A0c, (const double*)h->b,
                                            (const double*)h->x, (const double*)h->xl, h->r, h->part)));
  launch(h, CDGMG_K_VECTOR, k_reduce, dim3(1), dim3(RED_T), (const double*)h->part, (int)d.ns, 1, h->scal, SC_TMP,
         -1);
}

int true_residual(cdgmg_handle* h, double* rr) {
  enqueue_true_residual(h);
  return read_scalar(h, SC_TMP, rr);
}

void reset_profile(cdgmg_handle* h) {
  h->evs.clear();
  h->pool_next = 0;
  if (h->inner) reset_profile(h->inner);
}

void collect_profile(cdgmg_handle* h, cdgmg_solve_info* info) {
  if (!info) return;
  for (int k = 0; k < CDGMG_NK; ++k) {
    info->kernel_ms[k] = 0.0;
    info->kernel_launches[k] = 0;
  }
  if (!h->o.profile) return;
  (void)hipStreamSynchronize(h->stream);
  for (cdgmg_handle* g = h; g; g = g->inner)
    for (auto& e : g->evs) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
        info->kernel_ms[e.cls] += ms;
        info->kernel_launches[e.cls] += 1;
      }
    }
}

// solve A x = b with h->b set (internal order); result in x_hi + x_lo.
//
// One iteration is the V-cycle z = B r followed by the Krylov update (the dot
// of z, the new direction p, q = A p, x and r).  The host needs ||r||^2 after
// each update; the V-cycle of the next iteration is enqueued before the host
// waits for it, so the device does not idle during the round trip.  That
// V-cycle reads r, so a reliable update (r replaced by the compensated true
// residual once ||r|| dropped 100x) is applied after the following update,
// before the next V-cycle is enqueued.  Convergence is accepted on the true
// residual only, at the same iteration as without the look-ahead.
int krylov_cg(cdgmg_handle* h, cdgmg_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t m = h->N0 * h->np;
  const int np = h->np;
  DLevel& d0 = h->lv[0];
  HIPCHK(hipMemsetAsync(h->x, 0, m * sizeof(double), h->stream));
  HIPCHK(hipMemsetAsync(h->xl, 0, m * sizeof(double), h->stream));
  HIPCHK(hipMemcpyAsync(h->r, h->b, m * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  double bb = 0.0;
  dot_into(h, m, h->b, h->b, SC_BB);
  RETURN_IF(read_scalar(h, SC_BB, &bb));
  if (!std::isfinite(bb)) {
    set_error("solve: right-hand side is not finite");
    return CDGMG_ERR_NAN;
  }
  if (!h->ev_rr) HIPCHK(hipEventCreateWithFlags(&h->ev_rr, hipEventDisableTiming));
  const double nb = std::sqrt(bb);
  const double tol = h->o.tol;
  const bool fcg = h->o.outer == CDGMG_OUTER_FCG;
  int it = 0;
  double rel = 0.0, rel_prev = 0.0, rel_true = 0.0;
  int status = CDGMG_NOT_CONVERGED;
  double rho_last = nb;
  // near the tolerance the rounding of a plain FP64 q = A p (about
  // eps |A| |alpha p| per step) would make the recursive residual drift from
  // the true one; from rel <= 1e4 tol on, q is accumulated compensated
  bool accurate = false;
  bool replace_pending = false;
  void* z = nullptr;
  int nz = 0;
  bool zdot = false;
  // V-cycle of iteration `iter` on the current r (its dot with q or r fused)
  auto enqueue_vcycle = [&](int iter) {
    const double* dv = fcg ? (iter > 0 ? h->q : nullptr) : h->r;
    z = vcycle(h, h->r, dv, &nz);
    zdot = dv != nullptr;
  };
  // the Krylov update of iteration `iter` after its V-cycle; ||r||^2 -> SC_RR
  auto enqueue_update = [&](int iter) {
    // the dot of z (with q or r) and, from the second iteration on, beta
    if (zdot)
      launch(h, CDGMG_K_VECTOR, k_reduce, dim3(1), dim3(RED_T), (const double*)h->part, nz, 1, h->scal,
             fcg ? (int)SC_ZQ : (int)SC_ZR, iter > 0 ? (fcg ? 0 : 1) : -1);
    const double sign = fcg ? -1.0 : 1.0;
    const dim3 gp(grid_for((m + UP_K - 1) / UP_K));
    if (h->o.mg_precision == CDGMG_MG_FP32)
      launch(h, CDGMG_K_VECTOR, k_update_p<float>, gp, dim3(TPB), m, (const float*)z, h->p, (const double*)h->scal,
             sign, iter == 0 ? 1 : 0);
    else
      launch(h, CDGMG_K_VECTOR, k_update_p<double>, gp, dim3(TPB), m, (const double*)z, h->p, (const double*)h->scal,
             sign, iter == 0 ? 1 : 0);
    const unsigned g = (unsigned)d0.ns;
    if (accurate) {
      NP_DISPATCH(np, L0C_DISPATCH(h, launch(h, CDGMG_K_SPMV, k_spmv0<NP, H, NF, SYM, true>, dim3(g), dim3(WAVE * H),
                                            d0.n, (const int32_t*)d0.cols, (const int8_t*)d0.meta,
                                            (const double*)(SYM ? h->A0d : d0.A64), (const double*)h->A0c, (const double*)h->p,
                                            (const double*)h->r, h->q, h->part)));
    } else {
      NP_DISPATCH(np, L0_DISPATCH(h, launch(h, CDGMG_K_SPMV, k_spmv0<NP, H, NF, SYM, false>, dim3(g), dim3(WAVE * H),
                                            d0.n, (const int32_t*)d0.cols, (const int8_t*)d0.meta,
                                            (const double*)(SYM ? h->A0d : d0.A64), (const double*)h->A0c, (const double*)h->p,
                                            (const double*)h->r, h->q, h->part)));
    }
    launch(h, CDGMG_K_VECTOR, k_reduce, dim3(1), dim3(RED_T), (const double*)h->part, (int)g, 2, h->scal, SC_PQ,
           fcg ? 2 : 3);
    // x += alpha p: double-double once the compensated phase has started
    // (x_lo stays zero before), r -= alpha q
    const unsigned gu = std::min<unsigned>(1024, grid_for(m));
    if (accurate)
      launch(h, CDGMG_K_VECTOR, k_update_xr2, dim3(gu), dim3(TPB), m, (const double*)h->p, (const double*)h->q,
             h->x, h->xl, h->r, (const double*)h->scal, h->part);
    else
      launch(h, CDGMG_K_VECTOR, k_update_xr, dim3(gu), dim3(TPB), m, (const double*)h->p, (const double*)h->q,
             h->x, h->r, (const double*)h->scal, h->part);
    launch(h, CDGMG_K_VECTOR, k_reduce, dim3(1), dim3(RED_T), (const double*)h->part, (int)gu, 1, h->scal, SC_RR,
           -1);
  };
  if (nb == 0.0) {
    status = CDGMG_OK;
  } else {
    enqueue_vcycle(0);
    while (it < h->o.max_iter) {
      enqueue_update(it);
      const bool replaced = replace_pending;
      if (replaced) enqueue_true_residual(h);
      replace_pending = false;
      HIPCHK(hipMemcpyAsync(h->hscal, h->scal, SC_N * sizeof(double), hipMemcpyDeviceToHost, h->stream));
      HIPCHK(hipEventRecord(h->ev_rr, h->stream));
      // look ahead unless this update is expected to converge (the last
      // reduction factor applied once more reaches the tolerance)
      const bool expect_done = it >= 2 && rel_prev > 0.0 && rel * (rel / rel_prev) <= tol;
      const bool ahead = it + 1 < h->o.max_iter && !expect_done;
      if (ahead) enqueue_vcycle(it + 1);
      HIPCHK(hipEventSynchronize(h->ev_rr));
      const double rr = h->hscal[SC_RR];
      const double rt = replaced ? h->hscal[SC_TMP] : 0.0;
      ++it;
      if (!std::isfinite(rr) || !std::isfinite(rt)) {
        set_error("solve: residual is not finite");
        status = CDGMG_ERR_NAN;
        break;
      }
      rel_prev = rel;
      rel = std::sqrt(rr) / nb;
      if (rel <= 1e4 * tol) accurate = true;
      if (info && info->history && it <= info->history_len) info->history[it - 1] = rel;
      bool stale = false;  // the enqueued look-ahead V-cycle read an r that is replaced now
      if (replaced) {
        rel_true = std::sqrt(rt) / nb;
        rho_last = std::sqrt(rt);
        if (rel_true <= tol) {
          status = CDGMG_OK;
          break;
        }
      }
      if (rel <= tol) {
        // convergence is accepted on the compensated true residual
        double rt2;
        RETURN_IF(true_residual(h, &rt2));
        rel_true = std::sqrt(rt2) / nb;
        rho_last = std::sqrt(rt2);
        if (rel_true <= tol) {
          status = CDGMG_OK;
          break;
        }
        stale = true;
      } else if (std::sqrt(rr) <= 1e-2 * rho_last) {
        replace_pending = true;
      }
      if (it < h->o.max_iter && (!ahead || stale)) enqueue_vcycle(it);
    }
  }
  if (status != CDGMG_OK && status != CDGMG_ERR_NAN && nb != 0.0) {
    double rt;
    RETURN_IF(true_residual(h, &rt));
    rel_true = std::sqrt(rt) / nb;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iterations = it;
    info->rel_residual = rel_true;
    info->conv_factor = (it > 0 && rel > 0.0) ? std::pow(rel, 1.0 / it) : 0.0;
    info->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    collect_profile(h, info);
  }
  if (status == CDGMG_NOT_CONVERGED) set_error("solve: not converged within max_iter");
  return status;
}

// z = B v into Z_j (FP64)
void vcycle_into(cdgmg_handle* h, const double* v, double* zj) {
  void* z = vcycle(h, v, nullptr, nullptr);
  const int64_t m = h->N0 * h->np;
  if (h->o.mg_precision == CDGMG_MG_FP32)
    launch(h, CDGMG_K_VECTOR, k_cast<float, double>, dim3(grid_for(m)), dim3(TPB), m, (const float*)z, zj);
  else
    launch(h, CDGMG_K_VECTOR, k_cast<double, double>, dim3(grid_for(m)), dim3(TPB), m, (const double*)z, zj);
}

// Right-preconditioned restarted GMRES(m) in the flexible form (Sec. 4):
// each cycle starts from the compensated true residual r = b - A x,
// v_0 = r / ||r||; step j: z_j = B v_j, w = A z_j, classical Gram-Schmidt
// against v_0..v_j applied twice (each pass one multi-dot and one multi-axpy
// over the basis), h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}.  The host
// applies the Givens rotations to the Hessenberg column, whose last entry is
// the residual estimate; at the end of a cycle x += Z y (double-double).
// The V-cycle of step j+1 is enqueued before the host reads column j.
int krylov_gmres(cdgmg_handle* h, cdgmg_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  const int64_t m = h->N0 * h->np;
  const int np = h->np;
  DLevel& d0 = h->lv[0];
  const int R = h->o.restart;
  const int64_t ld = h->gm_ld;
  double* V = h->gmV;
  double* Z = h->gmZ;
  HIPCHK(hipMemsetAsync(h->x, 0, m * sizeof(double), h->stream));
  HIPCHK(hipMemsetAsync(h->xl, 0, m * sizeof(double), h->stream));
  double bb = 0.0;
  dot_into(h, m, h->b, h->b, SC_BB);
  RETURN_IF(read_scalar(h, SC_BB, &bb));
  if (!std::isfinite(bb)) {
    set_error("solve: right-hand side is not finite");
    return CDGMG_ERR_NAN;
  }
  if (!h->ev_rr) HIPCHK(hipEventCreateWithFlags(&h->ev_rr, hipEventDisableTiming));
  const double nb = std::sqrt(bb);
  const double tol = h->o.tol;
  std::vector<double> H((size_t)(R + 1) * R), cs(R), sn(R), g(R + 1), y(R);
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * R + j]; };
  int it = 0;
  double rel = 0.0, rel_prev = 0.0, rel_true = 0.0;
  bool accurate = false;
  int status = CDGMG_NOT_CONVERGED;
  const unsigned gd = std::min<unsigned>(1024, grid_for(m));
  auto reduce_to = [&](int nd, double* out) {
    launch(h, CDGMG_K_VECTOR, k_reduce, dim3(1), dim3(RED_T), (const double*)h->gmPart, (int)gd, nd, out, 0, -1);
  };
  if (nb == 0.0) status = CDGMG_OK;
  while (status != CDGMG_OK && it < h->o.max_iter) {
    // cycle start: r = b - A (x_hi + x_lo), compensated
    double rt;
    RETURN_IF(true_residual(h, &rt));
    if (!std::isfinite(rt)) {
      set_error("solve: residual is not finite");
      status = CDGMG_ERR_NAN;
      break;
    }
    rel_true = std::sqrt(rt) / nb;
    if (rel_true <= tol) {
      status = CDGMG_OK;
      break;
    }
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = std::sqrt(rt);
    launch(h, CDGMG_K_VECTOR, k_scale_vec, dim3(grid_for(m)), dim3(TPB), m, (const double*)h->r,
           (const double*)(h->scal + SC_TMP), V);
    vcycle_into(h, V, Z);
    int k = 0;
    for (int j = 0; j < R; ++j) {
      double* w = V + (int64_t)(j + 1) * ld;
      const double* zj = Z + (int64_t)j * ld;
      const unsigned gs = (unsigned)d0.ns;
      if (accurate) {
        NP_DISPATCH(np, L0C_DISPATCH(h, launch(h, CDGMG_K_SPMV, k_spmv0<NP, H, NF, SYM, true, false>, dim3(gs),
                                              dim3(WAVE * H), d0.n, (const int32_t*)d0.cols, (const int8_t*)d0.meta,
                                              (const double*)(SYM ? h->A0d : d0.A64), (const double*)h->A0c, zj,
                                              (const double*)nullptr, w, (double*)nullptr)));
      } else {
        NP_DISPATCH(np, L0_DISPATCH(h, launch(h, CDGMG_K_SPMV, k_spmv0<NP, H, NF, SYM, false, false>, dim3(gs),
                                              dim3(WAVE * H), d0.n, (const int32_t*)d0.cols, (const int8_t*)d0.meta,
                                              (const double*)(SYM ? h->A0d : d0.A64), (const double*)h->A0c, zj,
                                              (const double*)nullptr, w, (double*)nullptr)));
      }
      for (int pass = 0; pass < 2; ++pass) {
        double* hc = h->gmH + (size_t)pass * (R + 1);
        launch(h, CDGMG_K_VECTOR, k_multi_dot, dim3(gd), dim3(TPB), m, j + 1, (const double*)V, ld,
               (const double*)w, h->gmPart);
        reduce_to(j + 1, hc);
        launch(h, CDGMG_K_VECTOR, k_multi_axpy, dim3(grid_for(m)), dim3(TPB), m, j + 1, (const double*)V, ld,
               (const double*)hc, w);
      }
      double* nrm2 = h->gmH + 2 * (size_t)(R + 1);
      launch(h, CDGMG_K_VECTOR, k_dots, dim3(gd), dim3(TPB), m, 1, (const double*)w, (const double*)w,
             (const double*)nullptr, (const double*)nullptr, h->gmPart);
      reduce_to(1, nrm2);
      launch(h, CDGMG_K_VECTOR, k_scale_vec, dim3(grid_for(m)), dim3(TPB), m, (const double*)w,
             (const double*)nrm2, w);
      HIPCHK(hipMemcpyAsync(h->hgmH, h->gmH, 3 * (size_t)(R + 1) * sizeof(double), hipMemcpyDeviceToHost,
                            h->stream));
      HIPCHK(hipEventRecord(h->ev_rr, h->stream));
      // look ahead: the V-cycle of step j+1 needs only v_{j+1}
      const bool expect_done = j >= 2 && rel_prev > 0.0 && rel * (rel / rel_prev) <= tol;
      const bool ahead = j + 1 < R && it + 1 < h->o.max_iter && !expect_done;
      if (ahead) vcycle_into(h, w, Z + (int64_t)(j + 1) * ld);
      HIPCHK(hipEventSynchronize(h->ev_rr));
      ++it;
      k = j + 1;
      const double* hh = h->hgmH;
      for (int i = 0; i <= j; ++i) Hij(i, j) = hh[i] + hh[R + 1 + i];
      const double hn = std::sqrt(hh[2 * (R + 1)]);
      Hij(j + 1, j) = hn;
      if (!std::isfinite(hn)) {
        set_error("solve: Arnoldi vector is not finite");
        status = CDGMG_ERR_NAN;
        break;
      }
      for (int i = 0; i < j; ++i) {
        const double a = Hij(i, j), b = Hij(i + 1, j);
        Hij(i, j) = cs[i] * a + sn[i] * b;
        Hij(i + 1, j) = -sn[i] * a + cs[i] * b;
      }
      const double den = std::hypot(Hij(j, j), Hij(j + 1, j));
      cs[j] = Hij(j, j) / den;
      sn[j] = Hij(j + 1, j) / den;
      Hij(j, j) = den;
      Hij(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      rel_prev = rel;
      rel = std::fabs(g[j + 1]) / nb;
      if (rel <= 1e4 * tol) accurate = true;
      if (info && info->history && it <= info->history_len) info->history[it - 1] = rel;
      const bool cycle_end = rel <= tol || j + 1 == R || it >= h->o.max_iter || hn == 0.0;
      if (cycle_end) break;
      if (!ahead) vcycle_into(h, w, Z + (int64_t)(j + 1) * ld);
    }
    if (status == CDGMG_ERR_NAN) break;
    // y: back substitution on the rotated Hessenberg matrix; x += Z y
    for (int i = k - 1; i >= 0; --i) {
      double sacc = g[i];
      for (int c = i + 1; c < k; ++c) sacc -= Hij(i, c) * y[c];
      y[i] = sacc / Hij(i, i);
    }
    std::copy(y.begin(), y.begin() + k, h->hgmY);
    HIPCHK(hipMemcpyAsync(h->gmY, h->hgmY, (size_t)k * sizeof(double), hipMemcpyHostToDevice, h->stream));
    launch(h, CDGMG_K_VECTOR, k_update_x_multi, dim3(grid_for(m)), dim3(TPB), m, k, (const double*)Z, ld,
           (const double*)h->gmY, h->x, h->xl);
  }
  if (status == CDGMG_NOT_CONVERGED && nb != 0.0) {
    double rt;
    RETURN_IF(true_residual(h, &rt));
    rel_true = std::sqrt(rt) / nb;
    if (rel_true <= tol) status = CDGMG_OK;
  }
  HIPCHK(hipStreamSynchronize(h->stream));
  auto t1 = std::chrono::steady_clock::now();
  if (info) {
    info->iterations = it;
    info->rel_residual = rel_true;
    info->conv_factor = (it > 0 && rel > 0.0) ? std::pow(rel, 1.0 / it) : 0.0;
    info->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    collect_profile(h, info);
  }
  if (status == CDGMG_NOT_CONVERGED) set_error("solve: not converged within max_iter");
  return status;
}

int krylov(cdgmg_handle* h, cdgmg_solve_info* info) {
  return h->o.outer == CDGMG_OUTER_GMRES ? krylov_gmres(h, info) : krylov_cg(h, info);
}

// a nonsymmetric operator keeps one direction on the device at a time: the
// adjoint solve rebuilds the transposed hierarchy, forward calls rebuild A
int ensure_direction(cdgmg_handle* h, bool transposed) {
  if (h->transposed == transposed) return CDGMG_OK;
  return build_operators(h, nullptr, transposed);
}

// hp front end: the next p-level (degree p - 1, or 1 with p_jump) on the
// same mesh and hierarchy; its level-0 operator is set from this level 0.
// Below degree 2 the inner handle holds the p = 1 agglomeration hierarchy,
// above it recurses.  This handle keeps its level 0 only.
int upload_embedding(cdgmg_handle* h);

int setup_inner(cdgmg_handle* h, const cdgmg_mesh& mesh, const cdgmg_hierarchy& hier) {
  cdgmg_handle* in = new (std::nothrow) cdgmg_handle();
  if (!in) return CDGMG_ERR_NOMEM;
  h->inner = in;
  const int q = h->o.p_jump ? 1 : h->P.p - 1;
  in->o = h->o;
  in->o.kernel_variant = 0;
  in->o.outer = CDGMG_OUTER_FCG;  // only its V-cycle runs: no Krylov work vectors
  in->stream = h->stream;
  in->ws = h->ws;
  in->pinned = h->pinned;
  in->given_A0 = true;
  int rc;
  try {
    rc = build_problem(mesh, q, hier, in->o, in->P);
  } catch (const std::exception& e) {
    set_error(std::string("setup: ") + e.what());
    rc = CDGMG_ERR_NOMEM;
  }
  if (rc) return rc;
  in->H0 = pick_h0(in->P.np, 0);
  in->H0c = pick_h0(in->P.np, 0, true);
  const Level &a = h->P.lv[0], &b = in->P.lv[0];
  if (a.perm != b.perm || a.cols != b.cols || a.slice_blk != b.slice_blk) {
    set_error("setup: the lower-degree level does not share the level-0 order and pattern");
    return CDGMG_ERR_HIERARCHY;
  }
  h->np1 = in->P.np;
  h->P.L = 0;
  h->P.lv.resize(1);
  if (q >= 2) RETURN_IF(setup_inner(in, mesh, hier));
  RETURN_IF(upload_problem(in));
  if (in->inner) RETURN_IF(upload_embedding(in));
  return CDGMG_OK;
}

// the embedding T[i][k] = lower-degree nodal basis k at the degree-p node i
int upload_embedding(cdgmg_handle* h) {
  const RefElem &R = h->P.ref, &R1 = h->inner->P.ref;
  const int np = R.np, np1 = R1.np, d = R.d;
  std::vector<double> T((size_t)np * np1);
  double phi[32];
  for (int i = 0; i < np; ++i) {
    R1.eval(&R.nodes[(size_t)i * d], phi);
    for (int k = 0; k < np1; ++k) {
      // a lower-degree basis function vanishes on every facet its node is
      // off: exact zeros keep T^T A_0 T in the facet-trace form of A_0
      bool zero = false;
      for (int f = 0; f <= d; ++f) zero = zero || (R.on_facet(i, f) && !R1.on_facet(k, f));
      T[(size_t)i * np1 + k] = zero ? 0.0 : phi[k];
    }
  }
  RETURN_IF(upload(h, &h->Tp64, T));
  if (h->o.mg_precision == CDGMG_MG_FP32) {
    float* tf;
    RETURN_IF(upload(h, &tf, std::vector<float>(T.begin(), T.end())));
    h->Tpm = tf;
  } else {
    h->Tpm = h->Tp64;
  }
  return CDGMG_OK;
}

int check_handle(cdgmg_handle* h) {
  if (!h) {
    set_error("null handle");
    return CDGMG_ERR_ARG;
  }
  return CDGMG_OK;
}

// Host half of setup and the layout of the device arrays in the workspace:
// the problem (topology, switch, kappa-free element blocks, bases, transfers,
// Galerkin and flux plans), then every device array carved from ws, host data
// copied into it.  ws null: a counting workspace (no device call is made).
// On error *out is null and the partial handle is freed.
int prepare(const cdgmg_mesh* mesh, int p, const cdgmg_hierarchy* hier, const cdgmg_options* opts,
            const Workspace* ws, hipStream_t stream, bool pinned, cdgmg_handle** out) {
  *out = nullptr;
  if (!mesh || !hier) {
    set_error("setup: invalid argument");
    return CDGMG_ERR_ARG;
  }
  cdgmg_options o;
  if (opts)
    o = *opts;
  else
    cdgmg_default_options(&o);
  RETURN_IF(check_options(o));
  cdgmg_handle* h = new (std::nothrow) cdgmg_handle();
  if (!h) return CDGMG_ERR_NOMEM;
  h->o = o;
  h->stream = stream;
  h->pinned = pinned;
  if (ws) h->own_ws = *ws;
  int rc;
  try {
    rc = build_problem(*mesh, p, *hier, o, h->P);
  } catch (const std::exception& e) {
    set_error(std::string("setup: ") + e.what());
    rc = CDGMG_ERR_NOMEM;
  }
  if (!rc) {
    h->H0 = pick_h0(h->P.np, o.kernel_variant);
    h->H0c = pick_h0(h->P.np, o.kernel_variant, true);
    if (!h->H0) {
      set_error("setup: kernel_variant must be 0 or one of 1, 2, 4, 5 dividing n_p = " + std::to_string(h->P.np));
      rc = CDGMG_ERR_ARG;
    }
  }
  if (!rc && o.p_coarse == 1 && p >= 2) rc = setup_inner(h, *mesh, *hier);
  if (!rc) rc = upload_problem(h);
  if (!rc && h->inner) rc = upload_embedding(h);
  if (!rc && ws && h->ws->counting) {
    set_error("setup: the workspace holds " + std::to_string(ws->cap) + " bytes; this problem needs " +
              std::to_string(h->ws->used) + " (cdgmg_workspace_size)");
    rc = CDGMG_ERR_ARG;
  }
  if (rc) {
    std::string msg = cdg::last_error_cstr();
    cdgmg_destroy(h);
    set_error(msg);
    return rc;
  }
  *out = h;
  return CDGMG_OK;
}

// device half of setup: operators for kappa, block inverses, coarsest inverse
int finish_setup(cdgmg_handle* h, const double* kappa_dev) {
  if (h->pinned && !h->inner) {  // not for the no-allocation setup
    HIPCHK(hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
  }
  RETURN_IF(build_operators(h, kappa_dev, false));
  if (hipStreamSynchronize(h->stream) != hipSuccess) {
    set_error("setup: device error");
    return CDGMG_ERR_DEVICE;
  }
  return CDGMG_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int cdgmg_workspace_size(const cdgmg_mesh* mesh, int p, const cdgmg_hierarchy* hier, const cdgmg_options* opts,
                         size_t* bytes) {
  set_error("");
  if (!bytes) {
    set_error("workspace_size: invalid argument");
    return CDGMG_ERR_ARG;
  }
  *bytes = 0;
  cdgmg_handle* h = nullptr;
  RETURN_IF(prepare(mesh, p, hier, opts, nullptr, nullptr, true, &h));
  *bytes = h->ws->used;
  cdgmg_destroy(h);
  return CDGMG_OK;
}

int cdgmg_setup(const cdgmg_mesh* mesh, int p, const double* kappa_dev, const cdgmg_hierarchy* hier,
                const cdgmg_options* opts, void* workspace_dev, size_t workspace_bytes, void* stream,
                cdgmg_handle** out) {
  set_error("");
  if (!kappa_dev || !out || !workspace_dev) {
    set_error("setup: invalid argument");
    return CDGMG_ERR_ARG;
  }
  if ((uintptr_t)workspace_dev % WS_ALIGN) {
    set_error("setup: the workspace must be aligned to " + std::to_string(WS_ALIGN) + " bytes");
    return CDGMG_ERR_ARG;
  }
  Workspace ws;
  ws.base = (char*)workspace_dev;
  ws.cap = workspace_bytes;
  ws.counting = false;
  cdgmg_handle* h = nullptr;
  RETURN_IF(prepare(mesh, p, hier, opts, &ws, (hipStream_t)stream, true, &h));
  int rc = finish_setup(h, kappa_dev);
  if (rc) {
    std::string msg = cdg::last_error_cstr();
    cdgmg_destroy(h);
    set_error(msg);
    return rc;
  }
  *out = h;
  return CDGMG_OK;
}

int cdgmg_setup_static(const cdgmg_mesh* mesh, int p, const double* kappa_dev, const cdgmg_hierarchy* hier,
                       const cdgmg_options* opts, void* stream, cdgmg_handle** out) {
  set_error("");
  if (!kappa_dev || !out) {
    set_error("setup_static: invalid argument");
    return CDGMG_ERR_ARG;
  }
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= STATIC_MAX_DEV) {
    set_error("setup_static: device index out of range");
    return CDGMG_ERR_ARG;
  }
  Workspace ws;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {  // first call on this device, with it current
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) {
        set_error(std::string("setup_static: hipGetSymbolAddress of the static workspace failed: ") +
                  hipGetErrorString(e));
        return CDGMG_ERR_DEVICE;
      }
      g_static_ptr[dev] = ptr;
    }
    if (g_static_busy[dev]) {
      set_error("setup_static: the static workspace of this device is held by a live handle (destroy it first)");
      return CDGMG_ERR_ARG;
    }
    g_static_busy[dev] = true;
    ws.base = (char*)g_static_ptr[dev];
  }
  ws.cap = STATIC_WS_BYTES;
  ws.counting = false;
  cdgmg_handle* h = nullptr;
  int rc = prepare(mesh, p, hier, opts, &ws, (hipStream_t)stream, false, &h);
  if (!rc) {
    h->static_dev = dev;
    rc = finish_setup(h, kappa_dev);
    if (rc) {
      std::string msg = cdg::last_error_cstr();
      cdgmg_destroy(h);  // releases the static workspace
      set_error(msg);
      return rc;
    }
    *out = h;
    return CDGMG_OK;
  }
  std::string msg = cdg::last_error_cstr();
  if (rc == CDGMG_ERR_ARG && msg.find("workspace holds") != std::string::npos)
    msg = "setup_static: the problem does not fit the static workspace of " + std::to_string(STATIC_WS_BYTES) +
          " bytes (" + msg + ")";
  {
    // prepare may have copied into the array on the stream: done before release
    (void)hipStreamSynchronize((hipStream_t)stream);
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_busy[dev] = false;
  }
  set_error(msg);
  return rc;
}

int cdgmg_update_kappa(cdgmg_handle* h, const double* kappa_dev) {
  RETURN_IF(check_handle(h));
  set_error("");
  RETURN_IF(build_operators(h, kappa_dev, false));
  return CDGMG_OK;
}

int cdgmg_solve(cdgmg_handle* h, const double* f_dev, double* u_dev, cdgmg_solve_info* info) {
  RETURN_IF(check_handle(h));
  set_error("");
  RETURN_IF(ensure_direction(h, false));
  reset_profile(h);
  const int np = h->np;
  DLevel& d = h->lv[0];
  NP_DISPATCH(np, launch(h, -1, k_mass_in<NP>, dim3(grid_for(d.n)), dim3(TPB), d.n, (const int32_t*)d.perm,
                         (const double*)h->M, f_dev, h->b));
  int rc = krylov(h, info);
  launch(h, -1, k_out_dd, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         (const double*)h->x, (const double*)h->xl, u_dev);
  HIPCHK(hipStreamSynchronize(h->stream));
  return rc;
}

int cdgmg_solve_rhs(cdgmg_handle* h, const double* b_dev, double* x_dev, cdgmg_solve_info* info) {
  RETURN_IF(check_handle(h));
  set_error("");
  RETURN_IF(ensure_direction(h, false));
  reset_profile(h);
  const int np = h->np;
  DLevel& d = h->lv[0];
  launch(h, -1, k_permute<double>, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         b_dev, h->b, 0);
  int rc = krylov(h, info);
  launch(h, -1, k_out_dd, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         (const double*)h->x, (const double*)h->xl, x_dev);
  HIPCHK(hipStreamSynchronize(h->stream));
  return rc;
}

int cdgmg_solve_transpose(cdgmg_handle* h, const double* g_dev, double* lam_dev, cdgmg_solve_info* info) {
  RETURN_IF(check_handle(h));
  if (h->P.beta == 0.0) return cdgmg_solve_rhs(h, g_dev, lam_dev, info);  // A = A^T
  set_error("");
  // A^T lambda = g with the transposed hierarchy; the V-cycle on A_l^T with the
  // pre- and post-sweep counts exchanged is the transpose of the forward one
  RETURN_IF(ensure_direction(h, true));
  reset_profile(h);
  const int np = h->np;
  DLevel& d = h->lv[0];
  launch(h, -1, k_permute<double>, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         g_dev, h->b, 0);
  std::swap(h->o.nu1, h->o.nu2);
  int rc = krylov(h, info);
  std::swap(h->o.nu1, h->o.nu2);
  launch(h, -1, k_out_dd, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         (const double*)h->x, (const double*)h->xl, lam_dev);
  HIPCHK(hipStreamSynchronize(h->stream));
  return rc;
}

int cdgmg_grad_kappa(cdgmg_handle* h, const double* u_dev, const double* lam_dev, double* gk_dev) {
  RETURN_IF(check_handle(h));
  set_error("");
  const int np = h->np;
  DLevel& d = h->lv[0];
  launch(h, -1, k_permute<double>, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         u_dev, h->t1, 0);
  launch(h, -1, k_permute<double>, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         lam_dev, h->t2, 0);
  NP_DISPATCH(np, launch(h, -1, k_grad_kappa<NP>, dim3(grid_for(d.n)), dim3(TPB), d.n, h->W0,
                         (const int32_t*)d.perm, (const int32_t*)d.cols, (const int64_t*)d.sblk,
                         (const double*)h->UA, (const double*)h->UH, (const int8_t*)h->hostflag,
                         (const double*)h->t1, (const double*)h->t2, gk_dev));
  HIPCHK(hipGetLastError());
  return CDGMG_OK;
}

int cdgmg_apply_mass(cdgmg_handle* h, const double* x_dev, double* y_dev) {
  RETURN_IF(check_handle(h));
  DLevel& d = h->lv[0];
  NP_DISPATCH(h->np, launch(h, -1, k_mass_apply<NP>, dim3(grid_for(d.n)), dim3(TPB), d.n, (const int32_t*)d.perm,
                            (const double*)h->M, x_dev, y_dev));
  HIPCHK(hipGetLastError());
  return CDGMG_OK;
}

int cdgmg_apply_A(cdgmg_handle* h, int level, int precision, const void* x_dev, void* y_dev) {
  RETURN_IF(check_handle(h));
  if (h->inner && level >= 1) return cdgmg_apply_A(h->inner, level - 1, precision, x_dev, y_dev);
  if (level < 0 || level > h->L || (precision != 0 && precision != 1) ||
      (precision == 1 && h->o.mg_precision != CDGMG_MG_FP32)) {
    set_error("apply_A: invalid level or precision");
    return CDGMG_ERR_ARG;
  }
  RETURN_IF(ensure_direction(h, false));
  DLevel& d = h->lv[level];
  const int np = h->np;
  if (precision == 0) {
    double *xi = h->t1, *yi = h->t2;
    launch(h, -1, k_permute<double>, dim3(grid_for(d.n * np)), dim3(TPB), d.n, np, (const int32_t*)d.perm,
           (const double*)x_dev, xi, 0);
    NP_DISPATCH(np, launch(h, -1, k_spmv<double, double, NP>, dim3(grid_for(d.n)), dim3(TPB), d.n,
                           (const int32_t*)d.cols, (const int64_t*)d.sblk, (const double*)d.A64, (const double*)xi,
                           yi));
    launch(h, -1, k_permute<double>, dim3(grid_for(d.n * np)), dim3(TPB), d.n, np, (const int32_t*)d.perm,
           (const double*)yi, (double*)y_dev, 1);
  } else {
    float *xi = (float*)h->t1, *yi = (float*)h->t2;
    launch(h, -1, k_permute<float>, dim3(grid_for(d.n * np)), dim3(TPB), d.n, np, (const int32_t*)d.perm,
           (const float*)x_dev, xi, 0);
    NP_DISPATCH(np, launch(h, -1, k_spmv<double, float, NP>, dim3(grid_for(d.n)), dim3(TPB), d.n,
                           (const int32_t*)d.cols, (const int64_t*)d.sblk, (const double*)d.A64, (const float*)xi,
                           yi));
    launch(h, -1, k_permute<float>, dim3(grid_for(d.n * np)), dim3(TPB), d.n, np, (const int32_t*)d.perm,
           (const float*)yi, (float*)y_dev, 1);
  }
  HIPCHK(hipGetLastError());
  return CDGMG_OK;
}

int cdgmg_vcycle(cdgmg_handle* h, const double* r_dev, double* z_dev) {
  RETURN_IF(check_handle(h));
  RETURN_IF(ensure_direction(h, false));
  DLevel& d = h->lv[0];
  const int np = h->np;
  launch(h, -1, k_permute<double>, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         r_dev, h->t1, 0);
  vcycle64(h, h->t1, h->t2);
  launch(h, -1, k_permute<double>, dim3(grid_for(h->N0 * np)), dim3(TPB), h->N0, np, (const int32_t*)d.perm,
         (const double*)h->t2, z_dev, 1);
  HIPCHK(hipGetLastError());
  return CDGMG_OK;
}

int cdgmg_level_info(cdgmg_handle* h, int* n_levels, int64_t* n_elem, int64_t* nnzb) {
  RETURN_IF(check_handle(h));
  if (h->inner) {  // level 0 at degree p, then the lower-degree levels
    int ni = 0;
    RETURN_IF(cdgmg_level_info(h->inner, &ni, n_elem ? n_elem + 1 : nullptr, nnzb ? nnzb + 1 : nullptr));
    if (n_levels) *n_levels = ni + 1;
    if (n_elem) n_elem[0] = h->lv[0].n;
    if (nnzb) nnzb[0] = h->lv[0].nnzb;
    return CDGMG_OK;
  }
  if (n_levels) *n_levels = h->L + 1;
  for (int l = 0; l <= h->L; ++l) {
    if (n_elem) n_elem[l] = h->lv[l].n;
    if (nnzb) nnzb[l] = h->lv[l].nnzb;
  }
  return CDGMG_OK;
}

int cdgmg_launch_info(cdgmg_handle* h, int* n_levels, int32_t* lanes_sweep, int32_t* lanes_restrict,
                      int32_t* row_threads, int* wavefronts) {
  RETURN_IF(check_handle(h));
  if (wavefronts) *wavefronts = h->H0;
  if (h->inner) {  // level 0 at degree p (level-0 kernels only), then the lower-degree levels
    int ni = 0;
    RETURN_IF(cdgmg_launch_info(h->inner, &ni, lanes_sweep ? lanes_sweep + 1 : nullptr,
                                lanes_restrict ? lanes_restrict + 1 : nullptr, row_threads ? row_threads + 1 : nullptr,
                                nullptr));
    if (n_levels) *n_levels = ni + 1;
    if (lanes_sweep) lanes_sweep[0] = 0;
    if (lanes_restrict) lanes_restrict[0] = 0;
    if (row_threads) row_threads[0] = TPB;  // k_prolong_rect
    return CDGMG_OK;
  }
  if (n_levels) *n_levels = h->L + 1;
  for (int l = 0; l <= h->L; ++l) {
    const bool grp = l >= 1 && l < h->L;
    if (lanes_sweep) lanes_sweep[l] = grp ? h->lv[l].grp_s : 0;
    if (lanes_restrict) lanes_restrict[l] = grp ? h->lv[l].grp_r : 0;
    if (row_threads) row_threads[l] = l < h->L ? row_tpb(h, l) : WAVE;
  }
  return CDGMG_OK;
}

int cdgmg_export_operator(cdgmg_handle* h, int level, int64_t* nnzb, int64_t* row_ptr, int32_t* cols,
                          double* blocks) {
  RETURN_IF(check_handle(h));
  if (h->inner && level >= 1) return cdgmg_export_operator(h->inner, level - 1, nnzb, row_ptr, cols, blocks);
  if (level < 0 || level > h->L || !nnzb) {
    set_error("export_operator: invalid argument");
    return CDGMG_ERR_ARG;
  }
  RETURN_IF(ensure_direction(h, false));
  const Level& H = h->P.lv[level];
  const DLevel& D = h->lv[level];
  const int np = h->np, np2 = np * np, nf = h->P.nf;
  // valid slots per internal row
  auto valid = [&](int64_t r, int w) {
    if (level == 0) return w == 0 || h->P.topo.nbr[(int64_t)H.perm[r] * nf + w - 1] >= 0;
    return w < H.row_len[r];
  };
  *nnzb = H.nnzb;
  if (!row_ptr || !cols || !blocks) return CDGMG_OK;
  std::vector<double> A((size_t)D.slots * np2);
  HIPCHK(hipMemcpyAsync(A.data(), D.A64, A.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  std::vector<int64_t> cnt(H.n + 1, 0);
  for (int64_t r = 0; r < H.n; ++r) {
    int c = 0;
    for (int w = 0; w < H.row_len[r]; ++w) c += valid(r, w);
    cnt[H.perm[r] + 1] = c;
  }
  for (int64_t i = 0; i < H.n; ++i) cnt[i + 1] += cnt[i];
  for (int64_t i = 0; i <= H.n; ++i) row_ptr[i] = cnt[i];
  for (int64_t r = 0; r < H.n; ++r) {
    const int64_t s = r / SLICE, lane = r % SLICE, B = H.slice_blk[s];
    std::vector<std::pair<int32_t, int>> ent;
    for (int w = 0; w < H.row_len[r]; ++w)
      if (valid(r, w)) ent.push_back({H.perm[H.cols[B + SLICE * w + lane]], w});
    std::sort(ent.begin(), ent.end());
    int64_t k = row_ptr[H.perm[r]];
    for (auto& e : ent) {
      cols[k] = e.first;
      for (int ij = 0; ij < np2; ++ij)
        blocks[k * np2 + ij] = A[(size_t)(B + SLICE * e.second) * np2 + (size_t)ij * SLICE + lane];
      ++k;
    }
  }
  return CDGMG_OK;
}

int cdgmg_node_coords(cdgmg_handle* h, double* xyz) {
  RETURN_IF(check_handle(h));
  std::copy(h->P.nodes.begin(), h->P.nodes.end(), xyz);
  return CDGMG_OK;
}

int cdgmg_set_profile(cdgmg_handle* h, int on) {
  RETURN_IF(check_handle(h));
  h->o.profile = on ? 1 : 0;
  if (h->inner) return cdgmg_set_profile(h->inner, on);
  return CDGMG_OK;
}

int cdgmg_device_bytes(cdgmg_handle* h, size_t* bytes) {
  RETURN_IF(check_handle(h));
  *bytes = h->ws->used;
  return CDGMG_OK;
}

int cdgmg_destroy(cdgmg_handle* h) {
  if (!h) return CDGMG_OK;
  if (h->inner) cdgmg_destroy(h->inner);
  // the device work of this handle ends before the caller may reuse the workspace
  if (h->ws->base) (void)hipStreamSynchronize(h->stream);
  if (h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  for (auto e : h->pool) (void)hipEventDestroy(e);
  if (h->ev_rr) (void)hipEventDestroy(h->ev_rr);
  host_free(h, h->hgmH);
  host_free(h, h->hgmY);
  host_free(h, h->hscal);
  host_free(h, h->herr);
  if (h->static_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_static_mu);
    g_static_busy[h->static_dev] = false;
  }
  delete h;
  return CDGMG_OK;
}

}  // extern "C"
