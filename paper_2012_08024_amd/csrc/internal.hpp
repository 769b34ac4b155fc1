// Host-side data structures of libcdgmg (no device code here).
#pragma once

#include <array>
#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "../../include/cdgmg.h"

namespace cdg {

constexpr int SLICE = 64;  // rows per slice of the sliced-ELL layouts (one wavefront)

struct Error {
  int code;
  std::string msg;
};

void set_error(const std::string& msg);
uint64_t splitmix64(uint64_t x);
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)>& body);

// ---------------------------------------------------------------- topology
struct Topology {
  int d = 0, nf = 0;     // nf = d + 1 facets per simplex
  int64_t N = 0;
  std::vector<int32_t> nbr;        // [N][nf], -1 on the boundary
  std::vector<int32_t> fid;        // [N][nf], interior facet id or -1
  std::vector<int32_t> face_a, face_ia, face_b, face_ib;  // interior facets, (lower, higher) element
  std::vector<int8_t> hosted;      // [N][nf]: element hosts this facet (interior host or Dirichlet)
};

int build_topology(const cdgmg_mesh& m, Topology& t);          // CDGMG_ERR_MESH on failure
void consistent_switch(Topology& t, const int8_t* face_bc);
void natural_switch(Topology& t, const int8_t* face_bc, uint64_t seed);

// Greedy agglomeration; returns level count, fills concatenated parents.
int agglomerate(const cdgmg_mesh& m, const Topology& t, int max_levels, int64_t coarse_dofs,
                int np, uint64_t seed, std::vector<int32_t>& parents,
                std::vector<int32_t>& sizes);

// --------------------------------------------------------- reference element
struct RefElem {
  int d = 0, p = 0, np = 0;
  std::vector<std::array<int, 3>> exps;  // graded monomial exponents
  std::vector<double> nodes;             // [np][d]
  std::vector<std::array<int, 4>> bary;  // [np]: integer barycentric coordinates p * lambda_f of each node
  // node n lies on local facet f (opposite vertex f) iff bary[n][f] == 0; the
  // trace of its basis function on every other facet is identically zero
  bool on_facet(int n, int f) const { return bary[n][f] == 0; }
  std::vector<double> coef;              // [nmono][np]: phi_n = sum_m coef[m][n] xi^m
  std::vector<double> qx, qw;            // volume rule on the reference simplex
  std::vector<double> fx, fw;            // facet rule on the reference (d-1)-simplex
  int nq = 0, nfq = 0;
  void init(int d, int p);
  void eval(const double* xi, double* phi) const;          // phi[np]
  void eval_grad(const double* xi, double* g) const;       // g[np][d]
};
void eval_monomials(int d, const std::vector<std::array<int, 3>>& exps, const double* x, double* m);
void gauss_jacobi01(int n, int alpha, std::vector<double>& x, std::vector<double>& w);
void simplex_rule(int d, int n, std::vector<double>& x, std::vector<double>& w);

// ------------------------------------------------------------- the problem
// Everything below is in *internal* order: level-l elements are renumbered so
// that the children of every level-(l+1) aggregate are contiguous.
struct Level {
  int64_t n = 0;                      // elements
  std::vector<int32_t> perm;          // internal -> hierarchy id
  std::vector<int32_t> iperm;         // hierarchy id -> internal
  // sliced-ELL pattern of A_l: rows grouped by SLICE, per-slice width
  std::vector<int32_t> row_len;       // [n]
  std::vector<int32_t> slice_w;       // [nslices]
  std::vector<int64_t> slice_blk;     // [nslices+1] block offset (in blocks of np*np, x SLICE lanes)
  std::vector<int32_t> cols;          // [sum_s slice_w*SLICE], internal column (pad = row)
  int64_t nnzb = 0;                   // stored (non-padding) blocks
  // children ranges in level l-1 (internal), for l >= 1
  std::vector<int32_t> child_start;   // [n+1]
  // parent (internal index at level l+1) of each element, for l < L
  std::vector<int32_t> parent;        // [n]
  // transfer blocks L_e (np x np, row = child basis, col = parent basis), l < L
  std::vector<double> Lblk;           // [n][np][np] row-major
  // aggregate basis (l >= 1)
  std::vector<double> center, scale, bcoef;  // [n][d], [n], [n][nmono][np]
  // Galerkin plan building A_l from A_{l-1} (l >= 1): coarse block k = row_blk[I] + t
  // accumulates L_e^T A_{l-1}(e, w) L_{col(e,w)} over plan entries
  std::vector<int64_t> row_blk;       // [n+1]
  std::vector<int64_t> plan_ptr;      // [nnzb+1]
  std::vector<int32_t> plan_e, plan_w;
  std::vector<int64_t> fine_begin;    // [n+1] range of input-mesh elements (internal order)
  int64_t slices() const { return (n + SLICE - 1) / SLICE; }
};

// Flux-form coarsening plans (Sec. 4.1) for level l -> l+1, in block indices.
// Operand references: kind + index; blocks of G_l, X and Y are stored
// component-major (component c at offset c * count).
enum OpKind : int8_t { OP_NONE = 0, OP_L = 1, OP_A = 2, OP_G = 3, OP_X = 4, OP_Y = 5, OP_MINV = 6, OP_MINVC = 7,
                       OP_M = 8 };
struct OpRef {
  int8_t kind;
  int8_t comp;   // component for G/X/Y, else 0
  int64_t idx;   // L: level-l row; A: (row, slot) packed as row * 64 + slot; G/X/Y: block; MINV: level-l row;
                 // MINVC: level-(l+1) row; M: level-l row
};
struct TPTerm {
  OpRef P, Q, R;  // contributes sign * P^T Q R (P or R may be OP_NONE = identity)
  double sign;
};
struct FluxPlan {
  // G_l pattern (level-l rows), X = G_l L pattern (level-l rows, level-(l+1) cols), Y = L^T X (= G_{l+1})
  std::vector<int64_t> g_ptr, x_ptr, y_ptr;        // row pointers
  std::vector<int32_t> g_col, x_col, y_col;        // columns
  std::vector<int64_t> xp_ptr, yp_ptr, mp_ptr;     // per-output term ranges
  std::vector<TPTerm> xp, yp, mp;                  // X blocks, Y blocks, M_{l+1} rows
  std::vector<int64_t> sp_ptr;                     // per A_{l+1} block (row_blk numbering)
  std::vector<TPTerm> sp;                          // Schur terms -X^T M_l^-1 X + Y^T M_{l+1}^-1 Y
};

struct Problem {
  int d = 0, p = 0, np = 0, nf = 0;
  int64_t N0 = 0;
  int L = 0;                          // coarsest level index
  double CD = 0.0, h_avg = 0.0, gamma = 0.0;
  Topology topo;
  RefElem ref;
  std::vector<Level> lv;
  // level-0 kappa-free data, row-major blocks indexed [row][slot] (internal order)
  std::vector<double> UA;             // [N0][nf+1][np][np]: slot 0 own block, slot s: A(r, col) / kappa_host
  std::vector<double> UH;             // [N0][nf+1][np][np]: hosted facet s-1: contribution to the neighbour's diagonal
  std::vector<int8_t> hostflag;       // [N0][nf+1]: 1 row hosts, 0 neighbour hosts, -1 none
  std::vector<int8_t> revslot;        // [N0][nf+1]: slot of this row in the neighbour's row
  std::vector<double> Mblk;           // [N0][np][np] element mass matrices
  std::vector<double> Gblk;           // [d][N0][nf+1][np][np] flux-form gradient (kappa-free)
  std::vector<double> nodes;          // [N0 caller order][np][d]
  // level 0 -> 1 transfers without stored blocks: for element r (internal
  // order) the affine map xi -> (x(xi) - c_I) / h_I into the parent's scaled
  // coordinates, u0[d] then Js[d][d] (row-major), so that
  // L_e(i, j) = sum_k mono_k(u0 + Js xi_i) bcoef_I(k, j)
  std::vector<double> aff0;           // [N0][d + d d]
  double beta = 0.0;                  // convection strength (0: none)
  std::vector<double> UC;             // [N0][nf+1][np][np] upwind convection blocks (beta != 0)
  bool flux = false;
  std::vector<FluxPlan> fp;           // [L]: plan building level l+1 from level l
  std::vector<double> G0;             // [d][nG0][np][np] block-major G_0 in the FluxPlan[0] pattern
};

int check_options(const cdgmg_options& o);
int build_problem(const cdgmg_mesh& m, int p, const cdgmg_hierarchy& h, const cdgmg_options& o,
                  Problem& P);
void flux_g0(Problem& P);
void flux_level_symbolic(Problem& P, int l, std::vector<std::vector<int32_t>>& rows,
                         std::vector<std::pair<std::pair<int32_t, int32_t>, TPTerm>>& sterms);
void flux_level_schur(Problem& P, int l, const std::vector<std::vector<int32_t>>& rows,
                      std::vector<std::pair<std::pair<int32_t, int32_t>, TPTerm>>& sterms);

}  // namespace cdg
