/*
 * cdgmg.h - C ABI of libcdgmg: agglomeration-based geometric multigrid for the
 * Compact Discontinuous Galerkin (CDG) discretisation of
 *
 *     -div(kappa grad u) = f  in the unit square / cube,  u = 0 on Dirichlet facets,
 *
 * on unstructured simplex meshes, after Pan & Persson, "Agglomeration-based
 * geometric multigrid solvers for compact discontinuous Galerkin discretizations
 * on unstructured meshes".  The solve is a flexible CG (or PCG) in FP64,
 * preconditioned by a V(nu1,nu2) cycle with damped block-Jacobi smoothing on a
 * fixed agglomerated hierarchy (Alg. 3), run in FP32 or FP64 on one gfx950 GPU.
 *
 * Conventions (every entry point):
 *   - Return value: 0 = success, >0 = warning, <0 = error; the message of the
 *     last error on the calling thread is returned by cdgmg_last_error().
 *   - Host arrays passed in are read during the call only; nothing is retained.
 *   - Device arrays (suffix _dev) are caller-owned device memory, read or
 *     written on the stream given at setup.  The library allocates no device
 *     memory: cdgmg_setup lays every device array of the handle out in one
 *     caller-owned workspace of cdgmg_workspace_size bytes, which the handle
 *     borrows until cdgmg_destroy returns (the caller frees it afterwards).
 *   - Per-element vectors are float64 [n_elem][n_p] in the caller's element
 *     order; n_p = C(p+d, d).  Level-0 coefficients are nodal values at the
 *     equispaced nodes of each simplex, ordered (with x = v0 + sum_k xi_k (v_k - v0)):
 *       d = 2: for j in 0..p, for i in 0..p-j:            xi = (i/p, j/p)
 *       d = 3: for k in 0..p, for j in 0..p-k, for i in 0..p-j-k: xi = (i/p, j/p, k/p)
 *   - Mesh: e2v lists d+1 vertices per element with positive orientation;
 *     local facet i of an element is the one opposite its local vertex i.
 *   - A call that runs device work returns after that work is enqueued, except
 *     where stated (solves synchronise once per outer iteration to test
 *     convergence).
 */
#ifndef CDGMG_H
#define CDGMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define CDGMG_OK 0
#define CDGMG_NOT_CONVERGED 1
#define CDGMG_ERR_ARG (-1)
#define CDGMG_ERR_MESH (-2)
#define CDGMG_ERR_HIERARCHY (-3)
#define CDGMG_ERR_SINGULAR (-4)
#define CDGMG_ERR_DEVICE (-5)
#define CDGMG_ERR_NOMEM (-6)
#define CDGMG_ERR_NAN (-7)

/* options */
#define CDGMG_MG_FP64 0          /* V-cycle in FP64 */
#define CDGMG_MG_FP32 1          /* V-cycle in FP32 inside the FP64 outer solve */
#define CDGMG_OUTER_FCG 0        /* flexible CG, one previous direction (Notay 2000) */
#define CDGMG_OUTER_PCG 1        /* preconditioned CG */
#define CDGMG_OUTER_GMRES 2      /* right-preconditioned restarted GMRES(restart), flexible form (Sec. 4) */
#define CDGMG_COARSEN_PRIMAL 0   /* A_{l+1} = L^T A_l L (Galerkin / RAT, Sec. 3.5) */
#define CDGMG_COARSEN_FLUX 1     /* flux-form coarsening + Schur complement (Sec. 4.1) */
#define CDGMG_SWITCH_CONSISTENT 0
#define CDGMG_SWITCH_NATURAL 1

/* kernel classes timed when cdgmg_options.profile != 0 */
#define CDGMG_K_SPMV 0           /* outer FP64 q = A_0 p with fused (p,q), (p,r) partial sums */
#define CDGMG_K_SMOOTH0 1        /* level-0 damped block-Jacobi sweep (one kernel); with
                                    p_coarse = 1 only the degree-p level's */
#define CDGMG_K_SMOOTH 2         /* first sweeps from zero and all other levels' sweeps */
#define CDGMG_K_RESTRICT 3       /* residual + restriction, all levels */
#define CDGMG_K_PROLONG 4        /* prolongation + correction, all levels */
#define CDGMG_K_COARSE 5         /* coarsest solve */
#define CDGMG_K_VECTOR 6         /* FCG vector updates, reductions, casts, true residual */
#define CDGMG_NK 8

typedef struct cdgmg_mesh {
  int dim;                 /* 2 or 3 */
  int64_t n_vert;
  const double* coords;    /* host [n_vert][dim] */
  int64_t n_elem;
  const int32_t* e2v;      /* host [n_elem][dim+1] */
  const int8_t* face_bc;   /* host [n_elem][dim+1]: 0 Dirichlet, 1 Neumann; read on boundary facets only */
} cdgmg_mesh;

typedef struct cdgmg_hierarchy {
  int n_levels;              /* levels including the input mesh (>= 1) */
  const int32_t* level_sizes;/* host [n_levels]; level_sizes[0] = n_elem */
  const int32_t* parent;     /* host, concatenated parent maps of levels 0..n_levels-2 */
} cdgmg_hierarchy;

typedef struct cdgmg_options {
  double gamma;        /* Dirichlet penalty C_D = kappa_K gamma / h_avg (Sec. 2.2); default 1e4 */
  double omega;        /* block-Jacobi damping; default 0.7 */
  int nu1, nu2;        /* pre/post sweeps; default 2, 2 */
  int mg_precision;    /* CDGMG_MG_FP32 (default) or CDGMG_MG_FP64 */
  int outer;           /* CDGMG_OUTER_FCG (default), CDGMG_OUTER_PCG or CDGMG_OUTER_GMRES */
  int coarsening;      /* CDGMG_COARSEN_PRIMAL (default) or CDGMG_COARSEN_FLUX */
  int switch_mode;     /* CDGMG_SWITCH_CONSISTENT (default) or CDGMG_SWITCH_NATURAL */
  uint64_t switch_seed;/* natural switch: enumeration = splitmix64(seed ^ id) */
  double tol;          /* relative true residual ||b - A x|| / ||b||; default 1e-10 */
  int max_iter;        /* default 500 */
  int profile;         /* nonzero: time kernel classes with HIP events */
  int kernel_variant;  /* wavefronts per 64-row slice of the level-0 V-cycle kernels and of the
                          outer FP64 product: 0 auto (1; 2 for the compensated outer product and
                          true residual at n_p = 20, which need more registers), or
                          1, 2, 4, 5 where it divides n_p (else setup fails with
                          CDGMG_ERR_ARG); coarse levels give each row a group of lanes
                          (coarse_group) */
  int restart;         /* GMRES restart length m (1..200); default 50; the setup then holds
                          2m + 1 FP64 work vectors (the Arnoldi basis V and Z = B V) */
  double beta;         /* convection strength of beta v . grad u (Sec. 5, convection-diffusion),
                          upwind DG fluxes; default 0 (Poisson).  Nonzero beta makes A
                          nonsymmetric: it requires outer = CDGMG_OUTER_GMRES and primal
                          coarsening (else setup fails with CDGMG_ERR_ARG) */
  double velocity[3];  /* constant v (first dim entries used); default (1, 0, 0) */
  int p_coarse;        /* hp front end (Sec. 4, hp paragraph): 1 runs p-multigrid on the input
                          mesh from degree p down to p = 1 before the agglomeration levels,
                          which then run at p = 1; 0 (default) agglomerates at p.  Each
                          p-level embeds the next lower degree element by element by the
                          nodal embedding T (n_p x n_p', the lower-degree nodal basis at the
                          degree-p nodes) and its operator is T^T A T.  Needs primal
                          coarsening and beta = 0 (else CDGMG_ERR_ARG); ignored for p = 1.
                          The level queries (level_info, apply_A, export_operator) then
                          number the p-levels first (degree p at level 0) and the p = 1
                          agglomeration levels after them */
  int p_jump;          /* with p_coarse = 1: 0 (default) lowers the degree by one per level
                          (p, p - 1, ..., 1); 1 goes from p straight to p = 1 */
  int coarse_group;    /* lanes per row of the damped block-Jacobi sweep and of the residual +
                          restriction on levels 1 .. L-1: 0 (default) chooses by the level's
                          mean row length (32, or 64 for long rows), or 8, 16, 32, 64 for every such level
                          (else CDGMG_ERR_ARG).  Results do not depend on it beyond rounding
                          order */
  int row_threads;     /* workgroup size of the thread-per-row transfer kernels (prolongation
                          and correction, coarse-level entry): 0 (default) 64, or 64 or 256
                          on every level */
  int coarse_fp64;     /* with the FP32 V-cycle: 1 keeps the coarsest solve (the explicit
                          inverse of A_L, Alg. 3) in FP64, products summed in FP64 and the
                          result rounded to FP32 once; 0 (default) rounds the inverse to FP32 */
} cdgmg_options;

typedef struct cdgmg_solve_info {
  int iterations;
  double rel_residual;         /* ||b - A (x_hi + x_lo)|| / ||b|| at exit, accumulated in
                                  double-double (compensated) arithmetic for the iterate the
                                  solve keeps as an unevaluated sum x_hi + x_lo.  The FP64
                                  vector returned is x_hi + x_lo rounded once; a residual
                                  formed from it in plain FP64 carries the rounding noise
                                  eps || |A| |u| || / ||b|| of one product (about 4e-10 for
                                  2D p = 3 at h = 1/316, growing like h^-2), which can exceed
                                  tol */
  double conv_factor;          /* (||r_k|| / ||r_0||)^(1/k) of the recursive residual */
  double solve_ms;             /* host wall time of the call, device-synchronised */
  double kernel_ms[CDGMG_NK];  /* summed HIP-event time per kernel class (profile != 0) */
  int64_t kernel_launches[CDGMG_NK];
  double* history;             /* optional host [history_len]: relative residual per iteration
                                  (GMRES: the least-squares residual estimate) */
  int history_len;
} cdgmg_solve_info;

typedef struct cdgmg_handle cdgmg_handle;

/* Library version (major*10000 + minor*100 + patch). */
int cdgmg_version(void);

/* Message of the last failed call on this thread ("" if none). */
const char* cdgmg_last_error(void);

/* Default options (values above). */
void cdgmg_default_options(cdgmg_options* opts);

/* Greedy agglomeration (Sec. 3.1 Alg. 1 with Sec. 3.2 Alg. 2), host only.
 * Face neighbours share a facet; queue key (N(e), splitmix64(seed^(level<<32)^e), e);
 * vertex ties by (splitmix64(seed^(level<<32)^(1<<62)^v), v); an element with
 * N < 2 joins the adjacent block with the fewest current-level members
 * (ties: lowest block id), or forms a vertex patch if none exists.
 * Stops after max_levels levels, at one element, or when
 * n_elem_level * n_p <= coarse_dofs_max (if coarse_dofs_max > 0; n_p from p).
 * parent_out: host buffer of at least n_elem*max_levels int32 (concatenated maps);
 * level_sizes_out: host [max_levels]; n_levels_out receives the level count. */
int cdgmg_agglomerate(const cdgmg_mesh* mesh, int max_levels, int64_t coarse_dofs_max, int p,
                      uint64_t seed, int32_t* parent_out, int32_t* level_sizes_out,
                      int* n_levels_out);

/* CDG switch (Sec. 2.2; consistent switch Sec. 4.2), host only.
 * hosted_out: host int8 [n_elem][dim+1], 1 where the element hosts that local
 * facet (S = -1 on its side: it owns the boundary gradient q^f), else 0;
 * boundary facets: 1 if Dirichlet.  Consistent mode orients the dual graph
 * along Euler circuits (virtual vertex joined to odd-degree elements, walks
 * from the lowest element, lowest facet id first; interior facets numbered
 * by (lower element, higher element)). */
int cdgmg_switch(const cdgmg_mesh* mesh, int mode, uint64_t seed, int8_t* hosted_out);

/* Device bytes cdgmg_setup needs for this mesh, degree, hierarchy and options,
 * in *bytes.  Runs the host half of setup (topology, switch, kappa-free element
 * blocks of the primal form eq. (primal_form), agglomerate bases and transfers
 * of Sec. 3.3-3.4, Galerkin / flux coarsening plans of Sec. 3.5 and 4.1) and
 * lays the device arrays out without touching the device; no GPU is needed.
 * Errors as cdgmg_setup (ARG, MESH, HIERARCHY, NOMEM). */
int cdgmg_workspace_size(const cdgmg_mesh* mesh, int p, const cdgmg_hierarchy* hier,
                         const cdgmg_options* opts, size_t* bytes);

/* Build the solver of eq. (poisson) in the CDG discretisation of Sec. 2
 * (primal form eq. (primal_form), degree p = 1..3) on the given mesh with
 * element coefficients kappa_dev (device float64 [n_elem], > 0 and finite),
 * the hierarchy's transfers (Sec. 3.4), coarse operators (Sec. 3.5 / 4.1),
 * inverted diagonal blocks for the block-Jacobi smoother and the inverse of
 * the coarsest operator (Alg. 3).  workspace_dev: caller-owned device memory
 * of workspace_bytes >= cdgmg_workspace_size(...) bytes, aligned to 256
 * bytes; the handle keeps every device array in it and borrows it until
 * cdgmg_destroy returns.  Device work runs on `stream` (hipStream_t, NULL =
 * default); setup returns after it has finished.  The handle also creates
 * one stream of its own (default priority), on which the operator builds
 * (here and in cdgmg_update_kappa) run the work beside their critical chain;
 * `stream` waits for it before these calls return, and cdgmg_destroy
 * releases it.
 * Errors: ARG (p, options, kappa, workspace null, misaligned or too small: the
 * message names the size needed), MESH (non-positive volume, a facet shared
 * by more than two elements), HIERARCHY (map out of range / empty aggregate),
 * SINGULAR (a diagonal block or the coarsest matrix is not positive definite,
 * or with flux coarsening or convection, singular), DEVICE, NOMEM (host). */
int cdgmg_setup(const cdgmg_mesh* mesh, int p, const double* kappa_dev,
                const cdgmg_hierarchy* hier, const cdgmg_options* opts, void* workspace_dev,
                size_t workspace_bytes, void* stream, cdgmg_handle** out);

/* cdgmg_setup without a workspace argument and without any allocation of
 * device or pinned host memory, for callers that cannot allocate: serving
 * loops and harnesses that forbid hipMalloc or allocating library calls.  The
 * handle's device arrays are laid out in a static device array of 64 MiB
 * (67 108 864 bytes) that every GPU the library runs on holds until the
 * process ends; its host readback buffers are ordinary host memory (the
 * per-iteration copy of the residual norm is then not overlapped).  A problem
 * whose cdgmg_workspace_size exceeds 64 MiB is refused with CDGMG_ERR_ARG
 * (2D p = 2 fits up to about 8 000 triangles).  Calls would race on the
 * shared array, so one live handle per GPU holds it: a second call on the
 * same GPU before cdgmg_destroy of the first is refused with CDGMG_ERR_ARG
 * (the check is thread-safe).  The array keeps the last handle's contents;
 * setup writes or clears every part it reads, so nothing of an earlier
 * handle is used.  Otherwise as cdgmg_setup, on the device current at the
 * call, except that the handle creates no stream of its own: its operator
 * builds run in order on `stream`. */
int cdgmg_setup_static(const cdgmg_mesh* mesh, int p, const double* kappa_dev,
                       const cdgmg_hierarchy* hier, const cdgmg_options* opts, void* stream,
                       cdgmg_handle** out);

/* Re-assemble A_0 = sum_e kappa_e A^(e) (eq. (primal_form) with the element
 * coefficient kappa_e on element e's terms) for new coefficients kappa_dev
 * (device float64 [n_elem], > 0 and finite) and rebuild the coarse operators
 * (Sec. 3.5 / 4.1), inverted diagonal blocks and the coarsest inverse on the
 * device, in the workspace.  Errors: ARG (kappa), SINGULAR, DEVICE.  Returns
 * after the device work is enqueued (errors found on the device are
 * reported after a synchronisation inside the call). */
int cdgmg_update_kappa(cdgmg_handle* h, const double* kappa_dev);

/* Solve A u = M_0 f (eq. (primal_form); f nodal source values [n_elem][n_p],
 * M_0 the block mass matrix) from u = 0 with the outer Krylov method
 * preconditioned by one V-cycle of Alg. 3 per iteration, until the relative
 * residual of info.rel_residual reaches tol.  u_dev [n_elem][n_p] receives
 * x_hi + x_lo rounded once.  Returns CDGMG_NOT_CONVERGED (a warning: u and
 * info hold the last iterate) if max_iter is reached, CDGMG_ERR_NAN if the
 * residual is not finite.  info may be NULL.  Synchronises once per outer
 * iteration and returns after the device work has finished. */
int cdgmg_solve(cdgmg_handle* h, const double* f_dev, double* u_dev, cdgmg_solve_info* info);

/* Solve A x = b for a given right-hand side vector b_dev [n_elem][n_p] (a
 * residual-space vector, as M_0 f) into x_dev; otherwise as cdgmg_solve. */
int cdgmg_solve_rhs(cdgmg_handle* h, const double* b_dev, double* x_dev, cdgmg_solve_info* info);

/* Adjoint solve A^T lambda = g through the same hierarchy: lambda_dev, g_dev
 * [n_elem][n_p].  For the Poisson operator A is symmetric and this is
 * cdgmg_solve_rhs with g; with convection (beta != 0) the levels are rebuilt
 * from A_0^T and the V-cycle runs with the sweep counts exchanged, its
 * transpose.  Returns as cdgmg_solve. */
int cdgmg_solve_transpose(cdgmg_handle* h, const double* g_dev, double* lam_dev,
                          cdgmg_solve_info* info);

/* gk_dev[e] = -lambda^T (dA/dkappa_e) u (float64 [n_elem]) for u_dev and
 * lam_dev [n_elem][n_p]: dA/dkappa_e is the kappa-free part of eq.
 * (primal_form) hosted by e (its volume term, the terms of the facets it
 * hosts by the switch of Sec. 2.2, and its Dirichlet penalty), applied over
 * its stencil, element e and its neighbours across hosted facets.  With
 * lambda = A^{-T} dL/du this is dL/dkappa_e of a loss L(u).  Enqueued only. */
int cdgmg_grad_kappa(cdgmg_handle* h, const double* u_dev, const double* lam_dev, double* gk_dev);

/* y = M_0 x (block mass matrix of the degree-p nodal basis on the input mesh,
 * the matrix of eq. (primal_form)'s right-hand side), x_dev and y_dev
 * [n_elem][n_p], distinct.  Enqueued only. */
int cdgmg_apply_mass(cdgmg_handle* h, const double* x_dev, double* y_dev);

/* y = A_level x for testing: A_0 of eq. (primal_form), A_l (l >= 1) the
 * coarse operator of Sec. 3.5 or Sec. 4.1.  precision: 0 = float64 vectors,
 * 1 = float32 vectors (products in float32 with the FP64 operator rounded;
 * only with the FP32 V-cycle), else CDGMG_ERR_ARG.  Level-l vectors are
 * [n_l][n_p] in the hierarchy's numbering of level l (level 0: caller
 * order); coarse coefficients refer to the orthonormal modal basis of each
 * aggregate (Sec. 3.3).  Enqueued only. */
int cdgmg_apply_A(cdgmg_handle* h, int level, int precision, const void* x_dev, void* y_dev);

/* One V-cycle z = B r of Alg. 3 (damped block Jacobi, nu1 pre- and nu2
 * post-sweeps, residual restriction and prolongation of Sec. 3.4, the
 * coarsest level solved directly), r_dev and z_dev float64 [n_elem][n_p];
 * runs in the configured precision.  Enqueued only. */
int cdgmg_vcycle(cdgmg_handle* h, const double* r_dev, double* z_dev);

/* Level statistics: n_levels, and per level (host arrays of n_levels entries,
 * each may be NULL) element count and stored n_p x n_p blocks of A_l. */
int cdgmg_level_info(cdgmg_handle* h, int* n_levels, int64_t* n_elem, int64_t* nnzb);

/* Launch configuration chosen at setup (test support).  Host arrays of n_levels
 * entries, each may be NULL: lanes_sweep[l] and lanes_restrict[l], lanes per row
 * of the sweep and of the residual + restriction on levels 1 .. L-1 (0 on
 * level 0 and on the coarsest level, which use other kernels); row_threads[l],
 * workgroup size of the thread-per-row transfer kernels of level l (the
 * prolongation into level l and, for l >= 1, the entry of level l).
 * wavefronts: wavefronts per 64-row slice of the level-0 kernels. */
int cdgmg_launch_info(cdgmg_handle* h, int* n_levels, int32_t* lanes_sweep, int32_t* lanes_restrict,
                      int32_t* row_threads, int* wavefronts);

/* Copy operator A_level to the host as block CSR in the hierarchy's numbering:
 * row_ptr [n_l+1], cols [nnzb], blocks [nnzb][n_p][n_p] (row-major, FP64).
 * Pass NULL buffers to query nnzb only (returned in *nnzb). Synchronous. */
int cdgmg_export_operator(cdgmg_handle* h, int level, int64_t* nnzb, int64_t* row_ptr,
                          int32_t* cols, double* blocks);

/* Level-0 nodal points (host [n_elem][n_p][dim], caller order). */
int cdgmg_node_coords(cdgmg_handle* h, double* xyz);

/* Switch HIP-event timing of kernel classes on or off for later solves. */
int cdgmg_set_profile(cdgmg_handle* h, int on);

/* Bytes of the workspace the handle uses (cdgmg_workspace_size of its setup). */
int cdgmg_device_bytes(cdgmg_handle* h, size_t* bytes);

/* Test support, host only: build the setup data of cdgmg_setup on the host
 * and form A_level there (kappa host [n_elem]), exported like
 * cdgmg_export_operator.  Lets CPU tests check the host half of the setup
 * (assembly, ordering, bases, transfers, Galerkin plans) without a GPU. */
int cdgmg_debug_host_operator(const cdgmg_mesh* mesh, int p, const double* kappa,
                              const cdgmg_hierarchy* hier, const cdgmg_options* opts, int level,
                              int64_t* nnzb, int64_t* row_ptr, int32_t* cols, double* blocks);

/* Free the handle's host state after its stream has finished; the workspace
 * is the caller's to free afterwards. */
int cdgmg_destroy(cdgmg_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* CDGMG_H */
