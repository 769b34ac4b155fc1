// HIP kernels of libcdgmg for gfx950 (see kernels.hpp for the block layouts).
// Included by solver.hip, the single device translation unit.
#include "kernels.hpp"

namespace cdg {

// =============================================================== setup kernels
// K9: A_0 = sum_e kappa_e A^(e) from the kappa-free hosted blocks, plus the
// kappa-free upwind convection blocks UC when present (UC may be null).
//   A(r, 0)  = kappa_r UA(r, 0) + sum_{w: neighbour c_w hosts} kappa_c UH(c, revslot) + UC(r, 0)
//   A(r, w)  = kappa_host UA(r, w) + UC(r, w)
template <int NP>
__global__ void k_assemble_A0(int64_t n, int W, const int32_t* __restrict__ cols, const int64_t* __restrict__ sblk,
                              const double* __restrict__ UA, const double* __restrict__ UH,
                              const int8_t* __restrict__ hostflag, const int8_t* __restrict__ revslot,
                              const double* __restrict__ kappa, const double* __restrict__ UC,
                              double* __restrict__ A) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  const double kr = kappa[r];
  for (int w = 1; w < W; ++w) {
    const int hf = hostflag[r * W + w];
    const int32_t c = cols[B + (int64_t)WAVE * w + lane];
    const double s = hf == 1 ? kr : (hf == 0 ? kappa[c] : 0.0);
#pragma unroll 10
    for (int ij = 0; ij < NP2; ++ij) {
      const int64_t o = blk_off(B, w, NP2, ij, lane);
      A[o] = s * UA[o] + (UC ? UC[o] : 0.0);
    }
  }
  // the neighbours that host a shared facet add kappa_c UH(c, revslot) to the
  // diagonal block: their block offsets and kappa first, then the entries
  constexpr int WM = 5;  // at most n_f + 1 = 5 slots (tetrahedra)
  int64_t ho[WM - 1];
  double hk[WM - 1];
  int nh = 0;
  for (int w = 1; w < W; ++w) {
    if (hostflag[r * W + w] != 0) continue;
    const int32_t c = cols[B + (int64_t)WAVE * w + lane];
    ho[nh] = blk_off(sblk[c / WAVE], revslot[r * W + w], NP2, 0, c % WAVE);
    hk[nh] = kappa[c];
    ++nh;
  }
#pragma unroll 10
  for (int ij = 0; ij < NP2; ++ij) {
    double acc = kr * UA[blk_off(B, 0, NP2, ij, lane)];
    for (int t = 0; t < nh; ++t) acc += hk[t] * UH[ho[t] + (int64_t)ij * WAVE];
    if (UC) acc += UC[blk_off(B, 0, NP2, ij, lane)];
    A[blk_off(B, 0, NP2, ij, lane)] = acc;
  }
}

// A_0^T in the same layout: out(r, 0) = A(r, 0)^T, out(r, w) = A(c, rs)^T for
// the neighbour c = cols(r, w) whose slot rs = revslot(r, w) holds A(c, r);
// slots without a neighbour (rs = 0) stay zero
template <int NP>
__global__ void k_transpose_A0(int64_t n, int W, const int64_t* __restrict__ sblk, const int32_t* __restrict__ cols,
                               const int8_t* __restrict__ revslot, const double* __restrict__ A,
                               double* __restrict__ out) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  for (int w = 0; w < W; ++w) {
    const int rs = w == 0 ? 0 : revslot[r * W + w];
    const int32_t c = w == 0 ? (int32_t)r : cols[B + (int64_t)WAVE * w + lane];
    const bool has = w == 0 || rs > 0;
    const int64_t Bc = sblk[c / WAVE];
    for (int i = 0; i < NP; ++i)
      for (int j = 0; j < NP; ++j)
        out[blk_off(B, w, NP2, i * NP + j, lane)] =
            has ? A[blk_off(Bc, rs, NP2, j * NP + i, (int)(c % WAVE))] : 0.0;
  }
}

// kappa in internal order; flags non-positive or non-finite values
__global__ void k_kappa_perm(int64_t n, const int32_t* __restrict__ perm, const double* __restrict__ kin,
                             double* __restrict__ kout, int* __restrict__ err) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double k = kin[perm[r]];
  if (!(k > 0.0) || !(k < 1e300)) *err = 1;
  kout[r] = k;
}

// K8: D^{-1} of the diagonal block (slot 0), Gauss-Jordan in place without
// pivoting (the block is symmetric positive definite: every pivot is a
// positive Schur-complement diagonal).  err is set on a non-positive pivot.
template <int NP>
__global__ __launch_bounds__(TPB) void k_diag_inverse(int64_t n, const int64_t* __restrict__ sblk,
                                                      const double* __restrict__ A, double* __restrict__ Dinv,
                                                      int* __restrict__ err, int definite) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  double* D = Dinv + (r / WAVE) * WAVE * NP2 + lane;
  if constexpr (NP <= 10) {
    // the block in registers (static indices after unrolling)
    double a[NP2];
#pragma unroll
    for (int ij = 0; ij < NP2; ++ij) a[ij] = A[blk_off(B, 0, NP2, ij, lane)];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      const double p = a[k * NP + k];
      if (definite ? !(p > 0.0) : !(p != 0.0)) {
        *err = 1;
        return;
      }
      const double ip = 1.0 / p;
      a[k * NP + k] = 1.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) a[k * NP + j] *= ip;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        if (i == k) continue;
        const double f = a[i * NP + k];
        a[i * NP + k] = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) a[i * NP + j] -= f * a[k * NP + j];
      }
    }
#pragma unroll
    for (int ij = 0; ij < NP2; ++ij) D[ij * WAVE] = a[ij];
    return;
  }
  for (int ij = 0; ij < NP2; ++ij) D[ij * WAVE] = A[blk_off(B, 0, NP2, ij, lane)];
  for (int k = 0; k < NP; ++k) {
    const double p = D[(k * NP + k) * WAVE];
    if (definite ? !(p > 0.0) : !(p != 0.0)) {
      *err = 1;
      return;
    }
    const double ip = 1.0 / p;
    D[(k * NP + k) * WAVE] = 1.0;
    for (int j = 0; j < NP; ++j) D[(k * NP + j) * WAVE] *= ip;
    for (int i = 0; i < NP; ++i) {
      if (i == k) continue;
      const double f = D[(i * NP + k) * WAVE];
      D[(i * NP + k) * WAVE] = 0.0;
      for (int j = 0; j < NP; ++j) D[(i * NP + j) * WAVE] -= f * D[(k * NP + j) * WAVE];
    }
  }
}

// K8 for the larger blocks (n_p > 10, too many for one thread's registers):
// a group of DIG = 32 lanes per row, lane j < n_p holding column j of the
// block; step k broadcasts the pivot column from lane k by shuffles.  Same
// arithmetic, in the same order, as the one-thread form above.
constexpr int DIG = 32;
template <int NP>
__global__ __launch_bounds__(TPB) void k_diag_inverse_cols(int64_t n, const int64_t* __restrict__ sblk,
                                                           const double* __restrict__ A, double* __restrict__ Dinv,
                                                           int* __restrict__ err, int definite) {
  static_assert(NP <= DIG, "one lane per column");
  constexpr int NP2 = NP * NP;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = gid / DIG;
  const int j = (int)(gid % DIG);
  if (r >= n) return;  // the whole group: r is uniform across it
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  const int jj = j < NP ? j : 0;  // lanes past n_p carry a copy of column 0, unused
  double a[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) a[i] = A[blk_off(B, 0, NP2, i * NP + jj, lane)];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    double c[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) c[i] = __shfl(a[i], k, DIG);
    const double p = c[k];
    if (definite ? !(p > 0.0) : !(p != 0.0)) bad = true;
    const double ip = 1.0 / p;
    if (jj == k) {
#pragma unroll
      for (int i = 0; i < NP; ++i) a[i] = (i == k) ? ip : 0.0 - c[i] * ip;
    } else {
      const double rk = a[k] * ip;
#pragma unroll
      for (int i = 0; i < NP; ++i)
        if (i != k) a[i] -= c[i] * rk;
      a[k] = rk;
    }
  }
  if (bad) {
    if (j == 0) *err = 1;
    return;
  }
  if (j < NP) {
    double* D = Dinv + (r / WAVE) * WAVE * NP2 + lane;
#pragma unroll
    for (int i = 0; i < NP; ++i) D[(i * NP + j) * WAVE] = a[i];
  }
}

// K7 (Galerkin): coarse block k = (I, t) accumulates L_e^T A_f(e, w) L_c over its
// plan entries (fixed order -> deterministic).  One workgroup per coarse block,
// one thread per entry (i, j); the operands of up to GCH plan entries are
// staged in LDS at once so their loads overlap.  The fine blocks of one
// sliced 64-row tile share cache lines, and the children of consecutive
// coarse rows are consecutive fine rows: consecutive coarse blocks therefore
// go to one XCD (xcd_slice), so that those lines are fetched into one L2
// instead of into all eight.
template <int NP>
__global__ void k_galerkin(int64_t nblk, const int32_t* __restrict__ blk_row, const int64_t* __restrict__ row_blk,
                           const int64_t* __restrict__ plan_ptr, const int32_t* __restrict__ plan_e,
                           const int32_t* __restrict__ plan_c, const int64_t* __restrict__ plan_a,
                           const double* __restrict__ Af, const double* __restrict__ Lf,
                           const int64_t* __restrict__ csblk, double* __restrict__ Ac) {
  constexpr int NP2 = NP * NP;
  constexpr int GCH = NP2 <= 100 ? 8 : 2;
  constexpr int NT = (NP2 + WAVE - 1) / WAVE * WAVE;  // threads per workgroup
  constexpr int NX = (GCH * NP2 + NT - 1) / NT;       // staged values per thread and operand
  __shared__ double sA[GCH][NP2], sLe[GCH][NP2], sLc[GCH][NP2], sT[GCH][NP2];
  __shared__ int64_t sa[GCH];
  __shared__ int32_t se[GCH], sc[GCH];
  const int64_t k = xcd_slice();
  if (k >= nblk) return;
  const int tid = threadIdx.x;
  const int i = tid / NP, j = tid % NP;
  double acc = 0.0;
  const int64_t q0 = plan_ptr[k], q1 = plan_ptr[k + 1];
  for (int64_t qc = q0; qc < q1; qc += GCH) {
    const int nc = (int)(q1 - qc < GCH ? q1 - qc : GCH);
    if (tid < nc) {
      sa[tid] = plan_a[qc + tid];
      se[tid] = plan_e[qc + tid];
      sc[tid] = plan_c[qc + tid];
    }
    __syncthreads();
    // all of a thread's operand loads are issued before the first LDS store
    double va[NX], ve[NX], vc[NX];
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int x = tid + u * NT;
      if (x < nc * NP2) {
        const int t = x / NP2, ij = x % NP2;
        va[u] = Af[sa[t] + (int64_t)ij * WAVE];
        ve[u] = Lf[row_off(se[t], NP2, ij)];
        vc[u] = Lf[row_off(sc[t], NP2, ij)];
      }
    }
#pragma unroll
    for (int u = 0; u < NX; ++u) {
      const int x = tid + u * NT;
      if (x < nc * NP2) {
        const int t = x / NP2, ij = x % NP2;
        sA[t][ij] = va[u];
        sLe[t][ij] = ve[u];
        sLc[t][ij] = vc[u];
      }
    }
    __syncthreads();
    for (int x = tid; x < nc * NP2; x += NT) {
      const int t = x / NP2, ij = x % NP2, ii = ij / NP, jj = ij % NP;
      double s = 0.0;
      for (int m = 0; m < NP; ++m) s += sA[t][ii * NP + m] * sLc[t][m * NP + jj];
      sT[t][ij] = s;
    }
    __syncthreads();
    if (tid < NP2)
      for (int t = 0; t < nc; ++t) {
        double s = 0.0;
        for (int m = 0; m < NP; ++m) s += sLe[t][m * NP + i] * sT[t][m * NP + j];
        acc += s;
      }
    __syncthreads();
  }
  if (tid < NP2) {
    const int32_t I = blk_row[k];
    const int t = (int)(k - row_blk[I]);
    Ac[blk_off(csblk[I / WAVE], t, NP2, tid, I % WAVE)] = acc;
  }
}

// K7 (flux form): out_o (+)= sum over its plan terms of sign * P^T Q R, in
// fixed order.  One workgroup per output block, one thread per entry.
template <int NP>
__global__ void k_triple(int64_t nout, const TPOut* __restrict__ outs, const int64_t* __restrict__ ptr,
                         const TPDev* __restrict__ ent, int accumulate) {
  constexpr int NP2 = NP * NP;
  __shared__ double sP[NP2], sQ[NP2], sR[NP2], sT[NP2];
  const int64_t o = blockIdx.x;
  if (o >= nout) return;
  const int tid = threadIdx.x;
  const int i = tid / NP, j = tid % NP;
  const TPOut out = outs[o];
  double acc = 0.0;
  if (accumulate && tid < NP2) acc = out.O[(int64_t)tid * out.so];
  for (int64_t q = ptr[o]; q < ptr[o + 1]; ++q) {
    const TPDev e = ent[q];
    if (tid < NP2) {
      sQ[tid] = e.Q[(int64_t)tid * e.sq];
      if (e.P) sP[tid] = e.P[(int64_t)tid * e.sp];
      if (e.R) sR[tid] = e.R[(int64_t)tid * e.sr];
    }
    __syncthreads();
    if (tid < NP2) {
      double s = 0.0;
      if (e.R) {
        for (int m = 0; m < NP; ++m) s += sQ[i * NP + m] * sR[m * NP + j];
      } else {
        s = sQ[tid];
      }
      sT[tid] = s;
    }
    __syncthreads();
    if (tid < NP2) {
      double s = 0.0;
      if (e.P) {
        for (int m = 0; m < NP; ++m) s += sP[m * NP + i] * sT[m * NP + j];
      } else {
        s = sT[tid];
      }
      acc += e.sign * s;
    }
    __syncthreads();
  }
  if (tid < NP2) out.O[(int64_t)tid * out.so] = acc;
}

// flux-form mass of level 0: M(e) = kappa_e^{-1} M_e (block-major output)
template <int NP>
__global__ void k_mass_kappa(int64_t n, const double* __restrict__ Mrow, const double* __restrict__ kappa,
                             double* __restrict__ Mbm) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double ik = 1.0 / kappa[r];
  for (int ij = 0; ij < NP2; ++ij) Mbm[r * NP2 + ij] = Mrow[row_off(r, NP2, ij)] * ik;
}

// inverse of block-major n_p x n_p blocks (Gauss-Jordan, no pivoting; blocks are SPD)
template <int NP>
__global__ void k_block_inverse_bm(int64_t n, const double* __restrict__ src, double* __restrict__ dst,
                                   int* __restrict__ err) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double* D = dst + r * NP2;
  for (int ij = 0; ij < NP2; ++ij) D[ij] = src[r * NP2 + ij];
  for (int k = 0; k < NP; ++k) {
    const double p = D[k * NP + k];
    if (!(p > 0.0)) {
      *err = 1;
      return;
    }
    const double ip = 1.0 / p;
    D[k * NP + k] = 1.0;
    for (int j = 0; j < NP; ++j) D[k * NP + j] *= ip;
    for (int i = 0; i < NP; ++i) {
      if (i == k) continue;
      const double f = D[i * NP + k];
      D[i * NP + k] = 0.0;
      for (int j = 0; j < NP; ++j) D[i * NP + j] -= f * D[k * NP + j];
    }
  }
}

// coarsest level: scatter the sliced blocks into a dense row-major matrix
// dense[(r n_p + i) ld + c n_p + j] += A(r, c)_{ij} over the stored blocks;
// one thread per (row, entry (i, j)) walks the row's slots in order (padding
// slots repeat the diagonal column with zero blocks, so one thread must own
// each destination)
template <int NP>
__global__ void k_dense_scatter(int64_t n, int64_t ld, const int32_t* __restrict__ cols,
                                const int64_t* __restrict__ sblk, const double* __restrict__ A,
                                double* __restrict__ dense) {
  constexpr int NP2 = NP * NP;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * NP2) return;
  const int64_t r = t / NP2;
  const int ij = (int)(t % NP2), i = ij / NP, j = ij % NP;
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  const int W = (int)((sblk[r / WAVE + 1] - B) / WAVE);
  for (int w = 0; w < W; ++w) {
    const int32_t c = cols[B + (int64_t)WAVE * w + lane];
    dense[(r * NP + i) * ld + (int64_t)c * NP + j] += A[blk_off(B, w, NP2, ij, lane)];
  }
}

// ------------------------------------------------- coarsest inverse (setup)
// Blocked Gauss-Jordan inversion in place, without pivoting (the coarsest
// Galerkin operator is SPD; a flux-coarsened one is only checked for nonzero
// pivots), on an ld x ld matrix, ld a multiple of GJB, whose padding is the
// identity.  For each diagonal block K, with P = A_KK^{-1} and all right-hand
// sides taken before the step:
//   A_KJ <- P A_KJ (J != K);  A_IJ <- A_IJ - A_IK P A_KJ (I, J != K);
//   A_IK <- -A_IK P (I != K);  A_KK <- P.
// Three launches per step: the pivot block, both panels into buffers, then
// the trailing update and the panel copies from those buffers.
constexpr int GJB = 64;

// dense <- 0 with ones on the padding diagonal (i = j >= nd)
__global__ void k_dense_init(int64_t nd, int64_t ld, double* __restrict__ dense) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ld * ld) return;
  const int64_t i = idx / ld, j = idx % ld;
  dense[idx] = (i == j && i >= nd) ? 1.0 : 0.0;
}

// diag0 <- the diagonal of the matrix before elimination
__global__ void k_dense_diag(int64_t ld, const double* __restrict__ dense, double* __restrict__ diag0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ld) diag0[i] = dense[i * ld + i];
}

// Definite mode: a pivot is the diagonal entry of a Schur complement of an
// SPD matrix, at least lambda_min; one at or below GJ_SING times the original
// diagonal entry marks a matrix that is singular in FP64 (condition above
// about 1e11), such as the operator with only Neumann boundaries, whose kernel
// holds the constants.
constexpr double GJ_SING = 1e-11;

// P = A_KK^{-1} by unblocked Gauss-Jordan (one workgroup of GJT threads, the
// block in registers);
// writes P into A_KK and into Pout; err = 1 on a pivot at or below
// GJ_SING diag0 (definite) or a zero pivot
constexpr int GJT = 1024;
__global__ __launch_bounds__(GJT) void k_gj_pivot(int64_t ld, int K, double* __restrict__ dense,
                                                  double* __restrict__ Pout, const double* __restrict__ diag0,
                                                  int* __restrict__ err, int definite) {
  // thread (i0, j), i0 < NW = GJT / GJB, keeps rows i0 + NW m, m < RM, of
  // column j in registers; per step only the pivot row and column go through
  // LDS, double-buffered by the step's parity so that one barrier per step
  // suffices.  The 64 steps are a serial chain: spreading the block over 16
  // wavefronts keeps each step's work per wavefront (RM products) short.  The
  // pivot is tested by the thread that holds it, against the original
  // diagonal entry loaded up front.
  constexpr int NW = GJT / GJB, RM = GJB / NW;
  __shared__ double rowk[2][GJB], colk[2][GJB];
  const int tid = threadIdx.x, j = tid % GJB, i0 = tid / GJB;
  double* Akk = dense + (int64_t)K * GJB * ld + (int64_t)K * GJB;
  double v[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = Akk[(int64_t)(i0 + NW * m) * ld + j];
  const double dj = diag0[(int64_t)K * GJB + j];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < GJB; ++k) {
    const int b = k & 1;
    if (i0 == k % NW) {
      const double pk = v[k / NW];
      rowk[b][j] = pk;
      if (j == k) bad = bad || (definite ? !(pk > GJ_SING * dj) : !(pk != 0.0 && pk == pk));
    }
    if (j == k)
#pragma unroll
      for (int m = 0; m < RM; ++m) colk[b][i0 + NW * m] = v[m];
    __syncthreads();
    const double p = rowk[b][k];
    const double ip = 1.0 / p;
    const double rj = rowk[b][j];
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int i = i0 + NW * m;
      const double ci = colk[b][i];
      const double gen = v[m] - ci * rj * ip;
      v[m] = (i == k) ? ((j == k) ? ip : rj * ip) : ((j == k) ? -ci * ip : gen);
    }
  }
  if (bad) *err = 1;
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int i = i0 + NW * m;
    Akk[(int64_t)i * ld + j] = v[m];
    Pout[i * GJB + j] = v[m];
  }
}

// The panel and trailing products below share one tile product: C = X Y for
// GJB x GJB tiles, X staged transposed (Xt[k][i] = X(i, k)) and Y as is, both
// in LDS; 256 threads, each with a 4 x 4 block of C in registers, summing over
// k in ascending order.  The staging issues all of a thread's global loads
// before its first LDS store, so a workgroup waits for one memory latency,
// not sixteen.  Xt's rows are padded by two entries: its transposed stores
// then spread over the banks while its rows stay 16-byte aligned.
constexpr int GJP = GJB + 2;

__device__ __forceinline__ void gj_stage(double (*Xt)[GJP], double (*Ys)[GJB], const double* X, int64_t ldx,
                                         const double* Y, int64_t ldy) {
  constexpr int NE = GJB * GJB / 256;
  double xv[NE], yv[NE];
#pragma unroll
  for (int m = 0; m < NE; ++m) {
    const int e = threadIdx.x + 256 * m, r = e / GJB, c = e % GJB;
    xv[m] = X[(int64_t)r * ldx + c];
    yv[m] = Y[(int64_t)r * ldy + c];
  }
#pragma unroll
  for (int m = 0; m < NE; ++m) {
    const int e = threadIdx.x + 256 * m, r = e / GJB, c = e % GJB;
    Xt[c][r] = xv[m];
    Ys[r][c] = yv[m];
  }
  __syncthreads();
}

__device__ __forceinline__ void gj_tile(const double (*Xt)[GJP], const double (*Ys)[GJB], double acc[4][4]) {
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  for (int k = 0; k < GJB; ++k) {
    double av[4], bv[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) av[a] = Xt[k][ti * 4 + a];
#pragma unroll
    for (int b = 0; b < 4; ++b) bv[b] = Ys[k][tj * 4 + b];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
  }
}

// C (ldc) = s * acc, the thread's 4 x 4 block
__device__ __forceinline__ void gj_store(double* C, int64_t ldc, const double acc[4][4], double s) {
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) C[(int64_t)(ti * 4 + a) * ldc + tj * 4 + b] = s * acc[a][b];
}

// Both panels of step K, from the matrix before the step, into buffers beside
// it (one launch; workgroup b < nbk takes row block J = b, the others column
// block I = b - nbk):
//   R_J = P A_KJ and Ko_J = A_KJ (row panel, [GJB][ld]);  C_I = -A_IK P ([ld][GJB]).
__global__ __launch_bounds__(256) void k_gj_panels(int64_t ld, int K, int nbk, const double* __restrict__ dense,
                                                   const double* __restrict__ P, double* __restrict__ R,
                                                   double* __restrict__ Ko, double* __restrict__ C) {
  const int b = blockIdx.x;
  const bool row = b < nbk;
  const int J = row ? b : b - nbk;
  if (J == K) return;
  __shared__ double Xt[GJB][GJP], Ys[GJB][GJB];
  double acc[4][4];
  if (row) {
    const double* Akj = dense + (int64_t)K * GJB * ld + (int64_t)J * GJB;
    gj_stage(Xt, Ys, P, GJB, Akj, ld);
    gj_tile(Xt, Ys, acc);
    gj_store(R + (int64_t)J * GJB, ld, acc, 1.0);
    for (int e = threadIdx.x; e < GJB * GJB; e += 256)
      Ko[(int64_t)(e / GJB) * ld + (int64_t)J * GJB + e % GJB] = Ys[e / GJB][e % GJB];
  } else {
    const double* Aik = dense + (int64_t)J * GJB * ld + (int64_t)K * GJB;
    gj_stage(Xt, Ys, Aik, ld, P, GJB);
    gj_tile(Xt, Ys, acc);
    gj_store(C + (int64_t)J * GJB * GJB, GJB, acc, -1.0);
  }
}

// the rest of step K (workgroup (J, I)), reading only the panel buffers:
//   A_IJ <- A_IJ - A_IK P A_KJ = A_IJ + C_I Ko_J   (I, J != K)
//   A_KJ <- R_J (J != K);  A_IK <- C_I (I != K)
__global__ __launch_bounds__(256) void k_gj_update(int64_t ld, int K, double* __restrict__ dense,
                                                   const double* __restrict__ R, const double* __restrict__ Ko,
                                                   const double* __restrict__ C) {
  const int J = blockIdx.x, I = blockIdx.y;
  if (I == K && J == K) return;
  double* Aij = dense + (int64_t)I * GJB * ld + (int64_t)J * GJB;
  if (I == K || J == K) {
    const double* src = I == K ? R + (int64_t)J * GJB : C + (int64_t)I * GJB * GJB;
    const int64_t lds = I == K ? ld : GJB;
    for (int e = threadIdx.x; e < GJB * GJB; e += 256)
      Aij[(int64_t)(e / GJB) * ld + e % GJB] = src[(int64_t)(e / GJB) * lds + e % GJB];
    return;
  }
  __shared__ double Xt[GJB][GJP], Ys[GJB][GJB];
  gj_stage(Xt, Ys, C + (int64_t)I * GJB * GJB, GJB, Ko + (int64_t)J * GJB, ld);
  double acc[4][4];
  gj_tile(Xt, Ys, acc);
  const int ti = threadIdx.x / 16, tj = threadIdx.x % 16;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) Aij[(int64_t)(ti * 4 + a) * ld + tj * 4 + b] += acc[a][b];
}

template <typename S, typename D>
__global__ void k_cast(int64_t n, const S* __restrict__ src, D* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (D)src[i];
}

// ============================================================ solve kernels
// y = A x, products in T with the stored operator (TA) rounded to T
template <typename TA, typename T, int NP>
__global__ __launch_bounds__(TPB) void k_spmv(int64_t n, const int32_t* __restrict__ cols,
                                              const int64_t* __restrict__ sblk, const TA* __restrict__ A,
                                              const T* __restrict__ x, T* __restrict__ y) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  const int W = (int)((sblk[r / WAVE + 1] - B) / WAVE);
  T acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = 0;
  for (int w = 0; w < W; ++w) {
    const int32_t c = cols[B + (int64_t)WAVE * w + lane];
    T xv[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) xv[j] = x[(int64_t)c * NP + j];
    const TA* Ab = A + (B + (int64_t)WAVE * w) * NP2 + lane;
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
      for (int j = 0; j < NP; ++j) acc[i] += (T)Ab[(i * NP + j) * WAVE] * xv[j];
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) y[r * NP + i] = acc[i];
}

template <typename T, bool NT>
__device__ __forceinline__ T ld(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

// A row of N contiguous values (a row of a row-major [rows][N] vector) in the
// widest loads or stores its alignment allows: N sizeof(T) bytes from a
// 16-byte aligned base, so every row starts on a multiple of the largest power
// of two (up to 16) dividing N sizeof(T).  A gathered neighbour row then costs
// N sizeof(T) / A memory instructions instead of N.
template <int A>
struct alignas(A) RowChunk {
  uint32_t w[A / 4];
};
template <typename T, int N>
constexpr int row_align() {
  return (N * (int)sizeof(T)) % 16 == 0 ? 16 : (N * (int)sizeof(T)) % 8 == 0 ? 8 : 4;
}
template <typename T, int N>
__device__ __forceinline__ void load_row(const T* p, T* v) {
  constexpr int A = row_align<T, N>(), C = N * (int)sizeof(T) / A;
  const RowChunk<A>* q = reinterpret_cast<const RowChunk<A>*>(p);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const RowChunk<A> t = q[c];
    __builtin_memcpy(reinterpret_cast<char*>(v) + c * A, &t, A);
  }
}
template <typename T, int N>
__device__ __forceinline__ void store_row(T* p, const T* v) {
  constexpr int A = row_align<T, N>(), C = N * (int)sizeof(T) / A;
  RowChunk<A>* q = reinterpret_cast<RowChunk<A>*>(p);
#pragma unroll
  for (int c = 0; c < C; ++c) {
    RowChunk<A> t;
    __builtin_memcpy(&t, reinterpret_cast<const char*>(v) + c * A, A);
    q[c] = t;
  }
}

// prolongation and correction: x_e += L_e x_c[parent(e)]
// Level 0 <-> 1 transfers without stored blocks (Sec. 3.4): the child's
// nodal coefficients of the parent's basis function j are its values at the
// child's nodes, L_e(i, j) = sum_k mono_k(z_i) C_I(k, j), with z_i the node i
// in the parent's scaled coordinates, z_i = u0 + Js xi_i (the element's affine
// map composed with the parent's scaling, d + d^2 values per element) and
// C_I the parent's monomial coefficients (n_p^2 values per aggregate, read
// by all of its children).  The reference nodes and the graded monomial
// exponents are compile-time tables in the order of the host's reference
// element.
template <int NP, int D>
struct ElemTab {
  static constexpr int P = D == 2 ? (NP == 3 ? 1 : NP == 6 ? 2 : 3) : (NP == 4 ? 1 : NP == 10 ? 2 : 3);
  static constexpr int NA = D + D * D;  // affine map values per element
  int ex[NP][3];                         // graded monomial exponents
  int nd[NP][3];                         // reference node i in multiples of 1/P
  constexpr ElemTab() : ex{}, nd{} {
    int k = 0;
    for (int deg = 0; deg <= P; ++deg) {
      if (D == 2) {
        for (int b = 0; b <= deg; ++b) {
          ex[k][0] = deg - b;
          ex[k][1] = b;
          ++k;
        }
      } else {
        for (int c = 0; c <= deg; ++c)
          for (int b = 0; b <= deg - c; ++b) {
            ex[k][0] = deg - b - c;
            ex[k][1] = b;
            ex[k][2] = c;
            ++k;
          }
      }
    }
    int n = 0;
    if (D == 2) {
      for (int j = 0; j <= P; ++j)
        for (int i = 0; i <= P - j; ++i) {
          nd[n][0] = i;
          nd[n][1] = j;
          ++n;
        }
    } else {
      for (int kk = 0; kk <= P; ++kk)
        for (int j = 0; j <= P - kk; ++j)
          for (int i = 0; i <= P - j - kk; ++i) {
            nd[n][0] = i;
            nd[n][1] = j;
            nd[n][2] = kk;
            ++n;
          }
    }
  }
};

// the monomials of the parent's basis at node i of this row's element; u holds
// the element's affine map (u0, then Js row by row)
template <typename T, int NP, int D>
__device__ __forceinline__ void node_monomials(const T* u, int i, T* mono) {
  constexpr ElemTab<NP, D> E{};
  T z[D];
#pragma unroll
  for (int c = 0; c < D; ++c) {
    T v = u[c];
#pragma unroll
    for (int a = 0; a < D; ++a) v += u[D + c * D + a] * (T(E.nd[i][a]) / T(E.P));
    z[c] = v;
  }
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    T v = T(1);
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
      for (int q = 0; q < 3; ++q)
        if (q < E.ex[k][c]) v *= z[c];
    mono[k] = v;
  }
}

// this lane's element map, per-row layout (NA values per row)
template <typename T, int NP, int D>
__device__ __forceinline__ void load_affine(const T* __restrict__ aff, int64_t r, T* u) {
  constexpr int NA = ElemTab<NP, D>::NA;
#pragma unroll
  for (int c = 0; c < NA; ++c) u[c] = __builtin_nontemporal_load(aff + ((r / WAVE) * NA + c) * WAVE + (r % WAVE));
}

// prolongation into level 0 with the transfer formed on the fly (Sec. 3.4):
// x_e += L_e x_I = M_e (C_I x_I), M_e(i, k) = mono_k(z_i)
template <typename T, int NP, int NF>
__global__ __launch_bounds__(TPB) void k_prolong0(int64_t n, const int32_t* __restrict__ parent,
                                                  const T* __restrict__ aff, const T* __restrict__ Cp,
                                                  const T* __restrict__ xc, T* __restrict__ x) {
  constexpr int NP2 = NP * NP, D = NF - 1;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t I = parent[r];
  T cv[NP], y[NP], xv[NP], u[ElemTab<NP, D>::NA];
  load_row<T, NP>(xc + I * NP, cv);
  const T* C = Cp + I * NP2;
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    T crow[NP];
    load_row<T, NP>(C + k * NP, crow);
    T s = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += crow[j] * cv[j];
    y[k] = s;
  }
  load_affine<T, NP, D>(aff, r, u);
  load_row<T, NP>(x + r * NP, xv);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    T mono[NP];
    node_monomials<T, NP, D>(u, i, mono);
    T s = 0;
#pragma unroll
    for (int k = 0; k < NP; ++k) s += mono[k] * y[k];
    xv[i] += s;
  }
  store_row<T, NP>(x + r * NP, xv);
}

template <typename T, int NP>
__global__ __launch_bounds__(TPB) void k_prolong(int64_t n, const int32_t* __restrict__ parent,
                                                 const T* __restrict__ Lb, const T* __restrict__ xc,
                                                 T* __restrict__ x) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t I = parent[r];
  // the parent's and this row's x with wide loads, the new row with wide stores
  T cv[NP], xv[NP];
  load_row<T, NP>(xc + I * NP, cv);
  load_row<T, NP>(x + r * NP, xv);
  const T* Lr = Lb + (r / WAVE) * WAVE * NP2 + (r % WAVE);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += __builtin_nontemporal_load(Lr + (i * NP + j) * WAVE) * cv[j];
    xv[i] += s;
  }
  store_row<T, NP>(x + r * NP, xv);
}

// coarsest: x = A_L^{-1} b, one wavefront per row; the inverse is stored with
// a leading dimension ld (a multiple of 64) and zero padding columns, b with
// zero padding up to ld, so every lane reads whole 16-byte vectors
template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int k = 4;
  __device__ static float dot(const float4& a, const float4& b) {
    return a.x * b.x + a.y * b.y + a.z * b.z + a.w * b.w;
  }
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int k = 2;
  __device__ static double dot(const double2& a, const double2& b) { return a.x * b.x + a.y * b.y; }
};

// FP64 inverse with FP32 vectors (the FP32 V-cycle with its coarsest solve in
// FP64): products and sum in FP64, x rounded once
__global__ __launch_bounds__(TPB) void k_dense_gemv_mixed(int64_t n, int64_t ld, const double* __restrict__ Ainv,
                                                          const float* __restrict__ b, float* __restrict__ x) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  const int lane = threadIdx.x % WAVE;
  if (row >= n) return;
  const double2* Ar = reinterpret_cast<const double2*>(Ainv + row * ld);
  const float2* bv = reinterpret_cast<const float2*>(b);
  const int64_t nv = ld / 2;
  double s = 0;
#pragma unroll 4
  for (int64_t c = lane; c < nv; c += WAVE) {
    const double2 a = Ar[c];
    const float2 v = bv[c];
    s += a.x * (double)v.x + a.y * (double)v.y;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) x[row] = (float)s;
}

template <typename T>
__global__ __launch_bounds__(TPB) void k_dense_gemv(int64_t n, int64_t ld, const T* __restrict__ Ainv,
                                                    const T* __restrict__ b, T* __restrict__ x) {
  using V = typename Vec16<T>::type;
  constexpr int KV = Vec16<T>::k;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x / WAVE);
  const int lane = threadIdx.x % WAVE;
  if (row >= n) return;
  const V* Ar = reinterpret_cast<const V*>(Ainv + row * ld);
  const V* bv = reinterpret_cast<const V*>(b);
  const int64_t nv = ld / KV;
  T s = 0;
#pragma unroll 4
  for (int64_t c = lane; c < nv; c += WAVE) s += Vec16<T>::dot(Ar[c], bv[c]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) x[row] = s;
}

// The coarsest level in one launch (hierarchies of three or more levels):
// every workgroup first forms the whole coarsest right-hand side in LDS,
// b_I = sum of the children's restricted residuals t_e (in the order of the
// coarse entry), then x_I = (A_L^{-1} b)_I for its own aggregate I, one
// wavefront per row as in the dense product above, and finally prolongs x_I
// into I's children on the level above, x_f[e] += L_e x_I (Sec. 3.4).  It
// replaces three launches whose work is a few microseconds each.  TA is the
// inverse's storage type (double with FP32 vectors: summed in FP64).  LDS:
// ld + NP values of T (dynamic).
template <typename T, typename TA, int NP>
__global__ __launch_bounds__(1024) void k_coarsest(int64_t n, int64_t ld, const TA* __restrict__ Ainv,
                                                   const int32_t* __restrict__ cs, const T* __restrict__ t,
                                                   const T* __restrict__ Lf, T* __restrict__ xc,
                                                   T* __restrict__ xf) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* sb = reinterpret_cast<T*>(smem);
  T* sx = sb + ld;
  using V = typename Vec16<TA>::type;
  constexpr int KV = Vec16<TA>::k;
  const int64_t I = blockIdx.x, nd = n * NP;
  const int tid = threadIdx.x, nt = blockDim.x;
  // the prolongation's operands do not depend on x_I: thread k = tid takes
  // component a of child e and loads its row of L_e and x_f first
  const int32_t e0 = cs[I];
  const int ne = cs[I + 1] - e0;
  T lv[NP], xv = 0;
  const bool own = tid < ne * NP;
  if (own) {
    const int64_t e = e0 + tid / NP;
    const int a = tid % NP;
    const T* Lr = Lf + (e / WAVE) * WAVE * NP * NP + (e % WAVE);
#pragma unroll
    for (int j = 0; j < NP; ++j) lv[j] = __builtin_nontemporal_load(Lr + (a * NP + j) * WAVE);
    xv = xf[e * NP + a];
  }
  // b in LDS: each entry's children loaded together, then summed in order
  for (int64_t k = tid; k < ld; k += nt) {
    T s = 0;
    if (k < nd) {
      const int64_t a = k / NP;
      const int j = (int)(k - a * NP);
      const int32_t c1 = cs[a + 1];
      for (int32_t e = cs[a]; e < c1; e += 4) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = e + u < c1 ? t[(int64_t)(e + u) * NP + j] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (e + u < c1) s += v[u];
      }
    }
    sb[k] = s;
  }
  __syncthreads();
  const int w = tid / WAVE, lane = tid % WAVE, nw = nt / WAVE;
  for (int i = w; i < NP; i += nw) {
    const int64_t row = I * NP + i;
    const V* Ar = reinterpret_cast<const V*>(Ainv + row * ld);
    TA s = 0;
#pragma unroll 8
    for (int64_t c = lane; c < ld / KV; c += WAVE) {
      V bv;
      if constexpr (sizeof(TA) == sizeof(T)) {
        bv = reinterpret_cast<const V*>(sb)[c];
      } else {
        bv.x = (TA)sb[2 * c];
        bv.y = (TA)sb[2 * c + 1];
      }
      s += Vec16<TA>::dot(Ar[c], bv);
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) {
      sx[i] = (T)s;
      xc[row] = (T)s;
    }
  }
  __syncthreads();
  if (own) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += lv[j] * sx[j];
    xf[(e0 + tid / NP) * (int64_t)NP + tid % NP] = xv + s;
  }
  // an aggregate of more than blockDim / n_p children: the rest in further passes
  for (int k = tid + nt; k < ne * NP; k += nt) {
    const int64_t e = e0 + k / NP;
    const int a = k % NP;
    const T* Lr = Lf + (e / WAVE) * WAVE * NP * NP + (e % WAVE);
    T s = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += __builtin_nontemporal_load(Lr + (a * NP + j) * WAVE) * sx[j];
    xf[e * NP + a] += s;
  }
}

// ------------------------------------------------------------------
// Error-free transformations (Knuth TwoSum; FMA TwoProduct) for the outer
// loop.  The relative rounding noise of a plain FP64 product A x is about
// eps * || |A| |x| || / || A x ||, which grows like h^{-2} for this operator
// (about 4e-10 on a 2D p=3 mesh with h = 1/316): above a 1e-10 target.  The
// outer q = A p and the true residual are therefore accumulated as
// double-double sums (Ogita, Rump & Oishi, "Accurate sum and dot product",
// 2005, algorithm Dot2) and the iterate is kept as x_hi + x_lo.  These
// kernels are bound by HBM bytes, so the extra FP64 operations are free.
// FMA contraction must stay off in these routines: fusing the rounded product
// p = a x into the following sum would make the error terms double-count.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = (a + b);
  const double bb = (s - a);
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void dot2_acc(double a, double x, double& s, double& c) {
#pragma clang fp contract(off)
  const double p = (a * x);
  const double ep = __builtin_fma(a, x, -p);
  double t;
  two_sum(s, p, s, t);
  c = (c + (t + ep));
}



// ------------------------------------------------------------------
// Per-row n_p x n_p blocks of level 0 (D^{-1}, the diagonal blocks A_rr) are
// stored whole or, where the operator is symmetric (no convection), as their
// upper triangle row by row, n_p (n_p + 1) / 2 values: entry (i, j) at the
// packed index of (min(i, j), max(i, j)).  Same lane-interleaved per-slice
// layout, N values per row.
template <int NP, bool SYM>
struct RowBlk {
  static constexpr int N = SYM ? NP * (NP + 1) / 2 : NP * NP;
  static constexpr __device__ int idx(int i, int j) {
    if constexpr (!SYM) {
      return i * NP + j;
    } else {
      const int a = i < j ? i : j, c = i < j ? j : i;
      return a * NP - a * (a - 1) / 2 + (c - a);
    }
  }
};

// packed upper triangle of per-row blocks: dst(s, e, lane) = (src(i, j) +
// src(j, i)) / 2 for packed index e of (i, j), i <= j; src holds whole
// blocks, sstride values per lane and slice (n_p^2 for the per-row layout,
// (n_f + 1) n_p^2 for slot 0 of the sliced level-0 operator)
template <typename T, int NP>
__global__ void k_pack_sym(int64_t ns, int64_t sstride, const double* __restrict__ src, T* __restrict__ dst) {
  constexpr int N = RowBlk<NP, true>::N;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(idx % WAVE);
  const int64_t rest = idx / WAVE;
  const int e = (int)(rest % N);
  const int64_t s = rest / N;
  if (s >= ns) return;
  int a = 0, rem = e;
  while (rem >= NP - a) {
    rem -= NP - a;
    ++a;
  }
  const int c = a + rem;
  const double* S = src + s * sstride * WAVE + lane;
  dst[(s * N + e) * WAVE + lane] = (T)(0.5 * (S[(a * NP + c) * WAVE] + S[(c * NP + a) * WAVE]));
}

// Level 0 in facet-trace form.  In the primal form (eq. (primal_form)) the
// element K couples to its neighbour K' across the facet f only through the
// terms that f's host contributes: jumps of traces on f, lifted traces, and
// the host's normal derivatives paired with the other side's trace.  The
// neighbour's basis therefore enters A(K, K') only through its trace on f, and
// with the nodal basis the trace of a function whose node is off f vanishes
// identically.  So an off-diagonal block of A_0 has nonzero entries only
//   - in the columns of the neighbour's facet nodes, when K hosts f
//     ("column" kind: A(K, K') = V P_f'^T, V n_p x n_fn), or
//   - in the rows of K's facet nodes, when K' hosts f ("row" kind:
//     A(K, K') = P_f V^T),
// n_fn = p + 1 (2D) or (p + 1)(p + 2) / 2 (3D) facet nodes of n_p.  The host
// assembly sets the vanishing traces to exact zeros, and setup checks that
// every dropped entry is zero.  Both kinds store V, n_p x n_fn values: in
// canonical order v[i][k] (i < n_p, k < n_fn) at
//     ((s n_f + w) n_p n_fn + i n_fn + k) 64 + lane      (slice s, facet slot w),
// column kind: v[i][k] = A(r, c)[i][fn(c's facet, k)]; row kind:
// v[j][k] = A(r, c)[fn(r's facet w, k)][j].  meta[(s n_f + w) 64 + lane] is the
// neighbour's local facet (column kind) or n_f (row kind); boundary slots are
// zero column-kind blocks with the row itself as column.
//
// The level-0 V-cycle runs on this form without prescaling: a damped
// block-Jacobi sweep is x <- (1 - omega) x + omega D^{-1} (b - A_off x)
// (D^{-1} A_rr = I), the restricted residual L_e^T (b - A_rr x - A_off x).
// Per element this reads n_f n_p n_fn off-diagonal values and D^{-1} (n_p^2)
// instead of the n_f n_p^2 of a prescaled D^{-1} A_off.
//
// H wavefronts share a 64-row slice (H divides n_p): wavefront h owns output
// rows i in [h NI, (h + 1) NI), NI = n_p / H, of the column-kind products and
// the input components j in the same range of the row-kind ones; the row-kind
// partial sums (all n_p rows) are added across wavefronts through LDS.

constexpr int deg_of(int np, int d) {
  return d == 2 ? (np == 3 ? 1 : np == 6 ? 2 : 3) : (np == 4 ? 1 : np == 10 ? 2 : 3);
}
constexpr int facet_nodes(int np, int nf) {
  return nf == 3 ? deg_of(np, 2) + 1 : (deg_of(np, 3) + 1) * (deg_of(np, 3) + 2) / 2;
}
// the k-th node (in the nodal order of the element) on local facet f, the facet
// opposite vertex f: the nodes whose f-th integer barycentric coordinate is 0
constexpr int facet_node(int np, int nf, int f, int k) {
  const int d = nf - 1, p = deg_of(np, d);
  int n = 0, cnt = 0;
  for (int c = 0; c <= (d == 3 ? p : 0); ++c)
    for (int j = 0; j <= p - c; ++j)
      for (int i = 0; i <= p - j - c; ++i) {
        const int lam[4] = {p - i - j - c, i, j, c};
        if (lam[f] == 0) {
          if (cnt == k) return n;
          ++cnt;
        }
        ++n;
      }
  return 0;
}
template <int NP, int NF>
struct FacetTab {
  static constexpr int NFN = facet_nodes(NP, NF);
  int v[NF][NFN];
  constexpr FacetTab() : v() {
    for (int f = 0; f < NF; ++f)
      for (int k = 0; k < NFN; ++k) v[f][k] = facet_node(NP, NF, f, k);
  }
};
// node of the k-th facet node on a facet chosen at run time (k fixed)
template <int NP, int NF>
__device__ __forceinline__ int facet_node_at(int f, int k) {
  constexpr FacetTab<NP, NF> FT{};
  int v = FT.v[0][k];
#pragma unroll
  for (int g = 1; g < NF; ++g) v = f == g ? FT.v[g][k] : v;
  return v;
}

// sums of products: plain (rounded each step, contracted to FMA) or Dot2
// (Ogita-Rump-Oishi, value s + c); addlo adds a product of a low-order part
template <typename T, bool COMP>
struct Acc {
  T s = T(0);
  __device__ __forceinline__ void add(T a, T x) { s += a * x; }
  __device__ __forceinline__ void addlo(T a, T x) { s += a * x; }
  __device__ __forceinline__ void merge(const Acc& o) { s += o.s; }
  __device__ __forceinline__ T value() const { return s; }
  __device__ __forceinline__ T lo() const { return T(0); }
  __device__ __forceinline__ void set_lo(T) {}
};
template <>
struct Acc<double, true> {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ double lo() const { return c; }
  __device__ __forceinline__ void set_lo(double v) { c = v; }
  __device__ __forceinline__ void add(double a, double x) { dot2_acc(a, x, s, c); }
  __device__ __forceinline__ void addlo(double a, double x) { c = __builtin_fma(a, x, c); }
  __device__ __forceinline__ void merge(const Acc& o) {
#pragma clang fp contract(off)
    double e;
    two_sum(s, o.s, s, e);
    c = (c + (o.c + e));
  }
  __device__ __forceinline__ double value() const {
#pragma clang fp contract(off)
    return s + c;
  }
};

// This wavefront's share of sign * A_off x at row r = 64 s + lane: column-kind
// blocks into acc[t] (row h NI + t), row-kind blocks into sc[i] (all rows,
// partial over this wavefront's input components).  With LO the vector is
// x + xl (xl the low-order part, accumulated without compensation).  The slot
// loop is not unrolled, so that one slot's values are in registers at a time;
// the row-kind sums go to r's facet-w nodes through a branch on the
// (wavefront-uniform) slot.
template <typename T, int NP, int H, int NF, bool COMP, bool LO, bool NT>
__device__ __forceinline__ void off0(int64_t s, int lane, int h, const int32_t* __restrict__ cols,
                                     const int8_t* __restrict__ meta, const T* __restrict__ Ac,
                                     const T* __restrict__ x, const T* __restrict__ xl, T sign,
                                     Acc<T, COMP>* acc, Acc<T, COMP>* sc) {
  constexpr FacetTab<NP, NF> FT{};
  constexpr int NFN = FacetTab<NP, NF>::NFN, NPF = NP * NFN, NI = NP / H;
  // columns and kinds of all slots first: each slot's gathers then wait for
  // one memory latency only
  int32_t cw[NF];
  int kw[NF];
#pragma unroll
  for (int w = 0; w < NF; ++w) {
    cw[w] = cols[(s * (NF + 1) + w + 1) * WAVE + lane];
    kw[w] = meta[(s * NF + w) * WAVE + lane];
  }
#pragma unroll 1
  for (int w = 0; w < NF; ++w) {
    int32_t cv = cw[0];
    int kd = kw[0];
#pragma unroll
    for (int g = 1; g < NF; ++g) {
      cv = w == g ? cw[g] : cv;
      kd = w == g ? kw[g] : kd;
    }
    const int64_t cb = (int64_t)cv * NP;
    const bool row = kd == NF;
    T xo[NI], xs[NFN], xol[LO ? NI : 1], xsl[LO ? NFN : 1];
    if constexpr (H == 1) {
      // the whole neighbour row in a few wide loads; its facet values by selection
      load_row<T, NP>(x + cb, xo);
      if constexpr (LO) load_row<T, NP>(xl + cb, xol);
#pragma unroll
      for (int k = 0; k < NFN; ++k) {
        T v = xo[FT.v[0][k]], vl = LO ? xol[LO ? FT.v[0][k] : 0] : T(0);
#pragma unroll
        for (int g = 1; g < NF; ++g) {
          v = kd == g ? xo[FT.v[g][k]] : v;
          if constexpr (LO) vl = kd == g ? xol[FT.v[g][k]] : vl;
        }
        xs[k] = row ? T(0) : v;
        if constexpr (LO) xsl[k] = row ? T(0) : vl;
      }
    } else {
#pragma unroll
      for (int t = 0; t < NI; ++t) {
        xo[t] = x[cb + h * NI + t];
        if constexpr (LO) xol[t] = xl[cb + h * NI + t];
      }
#pragma unroll
      for (int k = 0; k < NFN; ++k) {
        const int64_t a = cb + facet_node_at<NP, NF>(kd, k);
        xs[k] = row ? T(0) : x[a];
        if constexpr (LO) xsl[k] = row ? T(0) : xl[a];
      }
    }
    Acc<T, COMP> sw[NFN];
    const T* V = Ac + ((s * NF + w) * NPF + (int64_t)h * NI * NFN) * WAVE + lane;
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const T xr = row ? xo[t] : T(0);
      const T xrl = LO && row ? xol[LO ? t : 0] : T(0);
#pragma unroll
      for (int k = 0; k < NFN; ++k) {
        const T v = sign * ld<T, NT>(V + (t * NFN + k) * WAVE);
        acc[t].add(v, xs[k]);
        sw[k].add(v, xr);
        if constexpr (LO) {
          acc[t].addlo(v, xsl[k]);
          sw[k].addlo(v, xrl);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < NF; ++g)
      if (w == g)
#pragma unroll
        for (int k = 0; k < NFN; ++k) sc[FT.v[g][k]].merge(sw[k]);
  }
}

// Adds the row-kind partial sums of all wavefronts of the slice to acc (this
// wavefront's rows), summed in wavefront order through one n_p x 64 LDS buffer
// (shc: the low-order parts, COMP).  Every thread of the workgroup calls it.
template <typename T, int NP, int H, bool COMP>
__device__ __forceinline__ void gather_rows(int lane, int h, bool valid, Acc<T, COMP>* acc, Acc<T, COMP>* sc,
                                            T* shs, T* shc) {
  constexpr int NI = NP / H;
  if constexpr (H == 1) {
#pragma unroll
    for (int t = 0; t < NI; ++t) acc[t].merge(sc[t]);
  } else {
    for (int g = 0; g < H; ++g) {
      if (h == g && valid) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          Acc<T, COMP> o = sc[i];
          if (g > 0) {
            Acc<T, COMP> prev;
            prev.s = shs[i * WAVE + lane];
            if constexpr (COMP) prev.set_lo(shc[i * WAVE + lane]);
            prev.merge(sc[i]);
            o = prev;
          }
          shs[i * WAVE + lane] = o.s;
          if constexpr (COMP) shc[i * WAVE + lane] = o.lo();
        }
      }
      __syncthreads();
    }
    if (valid) {
#pragma unroll
      for (int t = 0; t < NI; ++t) {
        Acc<T, COMP> o;
        o.s = shs[(h * NI + t) * WAVE + lane];
        if constexpr (COMP) o.set_lo(shc[(h * NI + t) * WAVE + lane]);
        acc[t].merge(o);
      }
    }
    __syncthreads();
  }
}

// every wavefront of the slice gets the whole vector v (NP values; this
// wavefront holds rows h NI + t in own[t]) through LDS
template <typename T, int NP, int H>
__device__ __forceinline__ void share_rows(int lane, int h, bool valid, const T* own, T* all, T* sh) {
  constexpr int NI = NP / H;
  if constexpr (H == 1) {
#pragma unroll
    for (int i = 0; i < NP; ++i) all[i] = own[i];
  } else {
    if (valid)
#pragma unroll
      for (int t = 0; t < NI; ++t) sh[(h * NI + t) * WAVE + lane] = own[t];
    __syncthreads();
    if (valid)
#pragma unroll
      for (int i = 0; i < NP; ++i) all[i] = sh[i * WAVE + lane];
  }
}

// sweep on level 0: x_out = (1 - omega) x + omega D^{-1} (b - A_off x); with
// DOT also the slice's partial sum of (x_out, dv) in FP64 (part[slice])
template <typename T, int NP, int H, int NF, bool DOT, bool SYM>
__global__ __launch_bounds__(WAVE * H) void k_sweep0(int64_t n, const int32_t* __restrict__ cols,
                                                     const int8_t* __restrict__ meta, const T* __restrict__ Ac,
                                                     const T* __restrict__ Dinv, const T* __restrict__ b,
                                                     const T* __restrict__ xin, T omega, T* __restrict__ xout,
                                                     const double* __restrict__ dv, double* __restrict__ part, int rev) {
  constexpr int NP2 = NP * NP, NI = NP / H;
  __shared__ T sh[H > 1 ? NP * WAVE : 1];
  const int lane = threadIdx.x % WAVE, h = threadIdx.x / WAVE;
  const int64_t sl = slice_order(rev), r = sl * WAVE + lane;
  const bool valid = r < n;
  Acc<T, false> acc[NI], sc[NP];
  if (valid) {
    if constexpr (H == 1) {
      T bv[NP];
      load_row<T, NP>(b + r * NP, bv);
#pragma unroll
      for (int t = 0; t < NP; ++t) acc[t].s = bv[t];
    } else {
#pragma unroll
      for (int t = 0; t < NI; ++t) acc[t].s = b[r * NP + h * NI + t];
    }
    off0<T, NP, H, NF, false, false, false>(sl, lane, h, cols, meta, Ac, xin, nullptr, T(-1), acc, sc);
  }
  gather_rows<T, NP, H, false>(lane, h, valid, acc, sc, sh, nullptr);
  T own[NI], sv[NP];
#pragma unroll
  for (int t = 0; t < NI; ++t) own[t] = acc[t].value();
  share_rows<T, NP, H>(lane, h, valid, own, sv, sh);
  double d = 0.0;
  if constexpr (H == 1 && sizeof(T) == 4) {
    // whole rows in and out with wide accesses
    if (valid) {
      const T* D = Dinv + sl * WAVE * RowBlk<NP, SYM>::N + lane;
      T xv[NP], xn[NP];
      load_row<T, NP>(xin + r * NP, xv);
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        T y = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) y += D[RowBlk<NP, SYM>::idx(i, j) * WAVE] * sv[j];
        xn[i] = xv[i] + omega * (y - xv[i]);
      }
      store_row<T, NP>(xout + r * NP, xn);
      if constexpr (DOT) {
        double dq[NP];
        load_row<double, NP>(dv + r * NP, dq);
#pragma unroll
        for (int i = 0; i < NP; ++i) d += (double)xn[i] * dq[i];
      }
    }
  } else if (valid) {
    const T* D = Dinv + sl * WAVE * RowBlk<NP, SYM>::N + lane;
    // FP32 blocks: all of D^{-1}'s loads in flight at once; FP64: two rows
    constexpr int UF = sizeof(T) == 4 ? NI : 2;
#pragma unroll UF
    for (int t = 0; t < NI; ++t) {
      const int i = h * NI + t;
      T y = 0;
#pragma unroll
      for (int j = 0; j < NP; ++j) y += D[RowBlk<NP, SYM>::idx(i, j) * WAVE] * sv[j];
      const int64_t k = r * NP + i;
      const T xi = xin[k];
      const T v = xi + omega * (y - xi);
      xout[k] = v;
      if constexpr (DOT) d += (double)v * dv[k];
    }
  }
  if constexpr (DOT) {
    __shared__ double shd[H];
    d = block_sum(d, shd);
    if (threadIdx.x == 0) part[sl] = d;
  }
}

// residual of level 0 in this wavefront's rows: b - A_rr x - A_off x, then the
// whole residual vector of the row in res[NP] (every thread calls it)
template <typename T, int NP, int H, int NF, bool SYM>
__device__ __forceinline__ void residual0(int64_t sl, int64_t r, int lane, int h, bool valid,
                                          const int32_t* __restrict__ cols, const int8_t* __restrict__ meta,
                                          const T* __restrict__ Ac, const T* __restrict__ Ad,
                                          const T* __restrict__ b, const T* __restrict__ x, T* sh, T* res) {
  constexpr int NP2 = NP * NP, NI = NP / H;
  Acc<T, false> acc[NI], sc[NP];
  if (valid) {
    const T* Dg = Ad + sl * WAVE * RowBlk<NP, SYM>::N + lane;
    if constexpr (H == 1 && sizeof(T) == 4) {
      T bv[NP], xr[NP];
      load_row<T, NP>(b + r * NP, bv);
      load_row<T, NP>(x + r * NP, xr);
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        acc[i].s = bv[i];
#pragma unroll
        for (int j = 0; j < NP; ++j) acc[i].add(-__builtin_nontemporal_load(Dg + RowBlk<NP, SYM>::idx(i, j) * WAVE), xr[j]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NI; ++t) acc[t].s = b[r * NP + h * NI + t];
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        const T xj = x[r * NP + j];
#pragma unroll
        for (int t = 0; t < NI; ++t)
          acc[t].add(-__builtin_nontemporal_load(Dg + RowBlk<NP, SYM>::idx(h * NI + t, j) * WAVE), xj);
      }
    }
    off0<T, NP, H, NF, false, false, false>(sl, lane, h, cols, meta, Ac, x, nullptr, T(-1), acc, sc);
  }
  gather_rows<T, NP, H, false>(lane, h, valid, acc, sc, sh, nullptr);
  T own[NI];
#pragma unroll
  for (int t = 0; t < NI; ++t) own[t] = acc[t].value();
  share_rows<T, NP, H>(lane, h, valid, own, res, sh);
}

// residual + restriction on level 0: t_e = L_e^T (b - A x)_e
template <typename T, int NP, int H, int NF, bool SYM>
__global__ __launch_bounds__(WAVE * H) void k_restrict0(int64_t n, const int32_t* __restrict__ cols,
                                                        const int8_t* __restrict__ meta, const T* __restrict__ Ac,
                                                        const T* __restrict__ Ad, const T* __restrict__ b,
                                                        const T* __restrict__ x, const T* __restrict__ aff,
                                                        const int32_t* __restrict__ parent,
                                                        const T* __restrict__ Cp, T* __restrict__ t_out, int rev) {
  constexpr int NP2 = NP * NP, NI = NP / H, D = NF - 1;
  __shared__ T sh[H > 1 ? NP * WAVE : 1];
  const int lane = threadIdx.x % WAVE, h = threadIdx.x / WAVE;
  const int64_t sl = slice_order(rev), r = sl * WAVE + lane;
  const bool valid = r < n;
  T res[NP];
  residual0<T, NP, H, NF, SYM>(sl, r, lane, h, valid, cols, meta, Ac, Ad, b, x, sh, res);
  if (!valid) return;
  // t = L_e^T res = C_I^T w, w_k = sum_i mono_k(z_i) res_i
  T u[ElemTab<NP, D>::NA], w[NP];
  load_affine<T, NP, D>(aff, r, u);
#pragma unroll
  for (int k = 0; k < NP; ++k) w[k] = T(0);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    T mono[NP];
    node_monomials<T, NP, D>(u, i, mono);
#pragma unroll
    for (int k = 0; k < NP; ++k) w[k] += mono[k] * res[i];
  }
  const T* C = Cp + (int64_t)parent[r] * NP2;
  if constexpr (H == 1) {
    T tv[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) tv[j] = T(0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      T crow[NP];
      load_row<T, NP>(C + k * NP, crow);
#pragma unroll
      for (int j = 0; j < NP; ++j) tv[j] += crow[j] * w[k];
    }
    store_row<T, NP>(t_out + r * NP, tv);
  } else {
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const int j = h * NI + t;
      T s = 0;
#pragma unroll
      for (int k = 0; k < NP; ++k) s += C[k * NP + j] * w[k];
      t_out[r * NP + j] = s;
    }
  }
}

// level-0 entry from the FP64 outer residual: b = (T) r, x = omega D^{-1} b
// (the first sweep from zero)
template <typename T, int NP, int H, bool SYM>
__global__ __launch_bounds__(WAVE * H) void k_entry0(int64_t n, const double* __restrict__ src,
                                                     const T* __restrict__ Dinv, T omega, T* __restrict__ b,
                                                     T* __restrict__ x) {
  constexpr int NP2 = NP * NP, NI = NP / H;
  const int lane = threadIdx.x % WAVE, h = threadIdx.x / WAVE;
  const int64_t sl = xcd_slice(), r = sl * WAVE + lane;
  if (r >= n) return;
  T v[NP];
  {
    double rv[NP];
    load_row<double, NP>(src + r * NP, rv);
#pragma unroll
    for (int j = 0; j < NP; ++j) v[j] = (T)rv[j];
  }
  const T* D = Dinv + sl * WAVE * RowBlk<NP, SYM>::N + lane;
  if constexpr (H == 1 && sizeof(T) == 4) {
    T xv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < NP; ++j) s += D[RowBlk<NP, SYM>::idx(i, j) * WAVE] * v[j];
      xv[i] = omega * s;
    }
    store_row<T, NP>(b + r * NP, v);
    store_row<T, NP>(x + r * NP, xv);
  } else {
#pragma unroll
    for (int t = 0; t < NI; ++t) b[r * NP + h * NI + t] = v[h * NI + t];
    constexpr int UF = sizeof(T) == 4 ? NI : 2;
#pragma unroll UF
    for (int t = 0; t < NI; ++t) {
      const int i = h * NI + t;
      T s = 0;
#pragma unroll
      for (int j = 0; j < NP; ++j) s += D[RowBlk<NP, SYM>::idx(i, j) * WAVE] * v[j];
      x[r * NP + i] = omega * s;
    }
  }
}

// setup: the facet-trace form of the off-diagonal level-0 blocks from the
// dense sliced A_0 (FP64) in precision T, one thread per (slice, slot, value,
// lane); err = 1 if a dropped entry of the block is not zero
template <typename T, int NP, int NF>
__global__ void k_compress0(int64_t n, int64_t ns, const double* __restrict__ A, const int8_t* __restrict__ meta,
                            T* __restrict__ Ac, int* __restrict__ err) {
  constexpr FacetTab<NP, NF> FT{};
  constexpr int NFN = FacetTab<NP, NF>::NFN, NPF = NP * NFN, NP2 = NP * NP;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(idx % WAVE);
  int64_t rest = idx / WAVE;
  const int m = (int)(rest % NPF);
  rest /= NPF;
  const int w = (int)(rest % NF);
  const int64_t s = rest / NF;
  if (s >= ns) return;
  const int i = m / NFN, k = m % NFN;
  const int kd = meta[(s * NF + w) * WAVE + lane];
  int fr = 0, fc = 0;  // r's facet-w node and c's facet node of index k
#pragma unroll
  for (int g = 0; g < NF; ++g) {
    if (g == w) fr = FT.v[g][k];
    if (g == kd) fc = FT.v[g][k];
  }
  const int a = kd == NF ? fr : i, bb = kd == NF ? i : fc;
  const double* blk = A + ((s * (NF + 1) + w + 1) * WAVE) * NP2 + lane;
  if (s * WAVE + lane >= n) {  // rows past the last element: zero blocks
    Ac[((s * NF + w) * NPF + m) * WAVE + lane] = T(0);
    return;
  }
  Ac[((s * NF + w) * NPF + m) * WAVE + lane] = (T)blk[(a * NP + bb) * WAVE];
  // check: the threads of values (i, k), k < n_fn, check row i (column kind)
  // or column i (row kind) of the block off the kept facet nodes, thread k
  // the entries q = k, k + n_fn, ...
  {
    const int f = kd == NF ? w : kd;
    bool bad = false;
#pragma unroll
    for (int q0 = 0; q0 < NP; q0 += NFN) {
      const int q = q0 + k;
      if (q < NP) {
        bool on = false;
#pragma unroll
        for (int kk = 0; kk < NFN; ++kk) on = on || q == facet_node_at<NP, NF>(f, kk);
        const double v = kd == NF ? blk[(q * NP + i) * WAVE] : blk[(i * NP + q) * WAVE];
        if (!on && v != 0.0) bad = true;
      }
    }
    if (bad) *err = 1;
  }
}

// setup: the diagonal blocks of the dense sliced A_0 in the per-row layout, in T
template <typename T, int NP, int NF>
__global__ void k_diag0(int64_t ns, const double* __restrict__ A, T* __restrict__ Ad) {
  constexpr int NP2 = NP * NP;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(idx % WAVE);
  const int64_t rest = idx / WAVE;
  const int ij = (int)(rest % NP2);
  const int64_t s = rest / NP2;
  if (s >= ns) return;
  Ad[(s * NP2 + ij) * WAVE + lane] = (T)A[(s * (NF + 1) * NP2 + ij) * WAVE + lane];
}

// ------------------------------------------------------------------
// Coarse-level V-cycle kernels on D^{-1}-prescaled operators.  The damped
// block-Jacobi sweep x <- x + omega D^{-1} (b - A x) is evaluated as
//     x <- (1 - omega) x + omega (bt - At_off x),   bt = D^{-1} b,  At = D^{-1} A,
// where the diagonal block of At is the identity and is not stored, and the
// restricted residual L_e^T (b - A x)_e as Lt_e^T (bt - At x)_e with
// Lt_e = D_e^T L_e.  These sweeps read neither D^{-1} nor the diagonal block.

// coarse-level entry: b_I = sum over children of t_e; bt = D^{-1} b, x = omega bt
// (no D^{-1}: the coarsest level, bt receives b itself)
template <typename T, int NP>
__global__ __launch_bounds__(TPB) void k_entry_c(int64_t n, const int32_t* __restrict__ child_start,
                                                 const T* __restrict__ t, const T* __restrict__ Dinv, T omega,
                                                 T* __restrict__ bt, T* __restrict__ x) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  T bv[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) bv[j] = 0;
  // children two at a time with wide loads, summed in order
  const int32_t c1 = child_start[r + 1];
  for (int32_t e = child_start[r]; e < c1; e += 2) {
    T v0[NP], v1[NP];
    load_row<T, NP>(t + (int64_t)e * NP, v0);
    const bool two = e + 1 < c1;
    if (two) load_row<T, NP>(t + (int64_t)(e + 1) * NP, v1);
#pragma unroll
    for (int j = 0; j < NP; ++j) bv[j] += v0[j];
    if (two) {
#pragma unroll
      for (int j = 0; j < NP; ++j) bv[j] += v1[j];
    }
  }
  if (Dinv == nullptr) {
#pragma unroll
    for (int j = 0; j < NP; ++j) bt[r * NP + j] = bv[j];
    return;
  }
  const T* D = Dinv + (r / WAVE) * WAVE * NP2 + (r % WAVE);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    T s = 0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += D[(i * NP + j) * WAVE] * bv[j];
    bt[r * NP + i] = s;
    x[r * NP + i] = omega * s;
  }
}

// Coarse levels (G lanes per row): row r's off-diagonal blocks are a dense
// n_p x (len_r - 1) n_p strip, component-major, unpadded, at (woff[r] - r) n_p^2;
// the G lanes of row r take strip columns k = g, g + G, ... for every
// component, and the n_p partial sums are reduced with xor-shuffles inside the
// aligned G-lane group.  64 / G rows share a wavefront, so short rows still
// keep many independent loads in flight.  Columns: wcols[woff[r] + 1 + w].
template <int G, typename T>
__device__ __forceinline__ T group_allsum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T, int NP, int G>
__device__ __forceinline__ void grp_scaled_residual(int64_t r, int g, const int32_t* __restrict__ wcols,
                                                    const int64_t* __restrict__ woff, const T* __restrict__ R,
                                                    const T* __restrict__ x, T* res) {
  // U strip columns per lane per chunk: all their loads are issued before the
  // first product, so a chunk costs one memory latency
  constexpr int U = G >= 32 ? 2 : 64 / G;
  const int64_t o = woff[r];
  const int K = (int)(woff[r + 1] - o - 1) * NP;
  const T* Rr = R + (o - r) * NP * NP;
  T acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = 0;
  for (int k0 = g; k0 < K; k0 += U * G) {
    // column indices and strip values first (independent), then the x gather;
    // past the strip end a lane re-reads its first column (in bounds, weight 0)
    int c[U], j[U];
    T xv[U], rv[U][NP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * G;
      const int kk = k < K ? k : g;
      const int w = kk / NP;
      j[u] = kk - w * NP;
      c[u] = wcols[o + 1 + w];
#pragma unroll
      for (int i = 0; i < NP; ++i) rv[u][i] = Rr[(int64_t)i * K + kk];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T v = x[(int64_t)c[u] * NP + j[u]];
      xv[u] = k0 + u * G < K ? v : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < NP; ++i) acc[i] += rv[u][i] * xv[u];
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) res[i] = group_allsum<G>(acc[i]);
}

// lane g of a group writes components g, g + G, ...  With PROL (the last
// post-sweep of a level) the group then also prolongs its new x_r into the
// children e of r on the finer level, x_f[e] += L_e x_r (Sec. 3.4): that
// correction needs only this row's final value, so it saves the separate
// prolongation launch.  cs: the level's child ranges; Lf: the finer level's
// L_e blocks (per-row layout).
template <typename T, int NP, int G, bool PROL = false>
__global__ __launch_bounds__(TPB) void k_sweep_grp(int64_t n, const int32_t* __restrict__ wcols,
                                                   const int64_t* __restrict__ woff, const T* __restrict__ R,
                                                   const T* __restrict__ bt, const T* __restrict__ xin, T omega,
                                                   T* __restrict__ xout, const int32_t* __restrict__ cs = nullptr,
                                                   const T* __restrict__ Lf = nullptr, T* __restrict__ xf = nullptr) {
  constexpr int NP2 = NP * NP;
  const int64_t gid = (int64_t)blockIdx.x * TPB + threadIdx.x;
  const int64_t r = gid / G;
  const int g = (int)(gid % G);
  if (r >= n) return;
  T sum[NP];
  grp_scaled_residual<T, NP, G>(r, g, wcols, woff, R, xin, sum);
  if constexpr (!PROL) {
#pragma unroll
    for (int m = 0; m < (NP + G - 1) / G; ++m) {
      const int i = g + m * G;
      if (i < NP) {
        T si = sum[0];
#pragma unroll
        for (int q = 1; q < NP; ++q)
          if (q == i) si = sum[q];
        const T xi = xin[r * NP + i];
        xout[r * NP + i] = xi + omega * (bt[r * NP + i] - xi - si);
      }
    }
  } else {
    // every lane forms the whole new x_r (the same values in every lane)
    T xn[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const T xi = xin[r * NP + i];
      xn[i] = xi + omega * (bt[r * NP + i] - xi - sum[i]);
    }
#pragma unroll
    for (int m = 0; m < (NP + G - 1) / G; ++m) {
      const int i = g + m * G;
      if (i < NP) {
        T v = xn[0];
#pragma unroll
        for (int q = 1; q < NP; ++q)
          if (q == i) v = xn[q];
        xout[r * NP + i] = v;
      }
    }
    // consecutive lanes take consecutive children (consecutive rows of the
    // finer level) for one component, so the L_e loads of a group coalesce
    const int32_t e0 = cs[r], ne = cs[r + 1] - e0;
    for (int q = g; q < ne * NP; q += G) {
      const int64_t e = e0 + q % ne;
      const int i = q / ne;
      const T* Le = Lf + (e / WAVE) * WAVE * NP2 + (int64_t)i * NP * WAVE + (e % WAVE);
      T s = 0;
#pragma unroll
      for (int j = 0; j < NP; ++j) s += __builtin_nontemporal_load(Le + j * WAVE) * xn[j];
      xf[e * NP + i] += s;
    }
  }
}

// every lane forms the whole scaled residual of its row (n_p values), then
// lane g writes t_j = sum_i Lt(i, j) res_i for j = g, g + G, ... (column j
// of the row's Lt contiguous)
template <typename T, int NP, int G>
__global__ __launch_bounds__(TPB) void k_restrict_grp(int64_t n, const int32_t* __restrict__ wcols,
                                                      const int64_t* __restrict__ woff, const T* __restrict__ R,
                                                      const T* __restrict__ bt, const T* __restrict__ x,
                                                      const T* __restrict__ Lt, T* __restrict__ t) {
  constexpr int NP2 = NP * NP;
  const int64_t gid = (int64_t)blockIdx.x * TPB + threadIdx.x;
  const int64_t r = gid / G;
  const int g = (int)(gid % G);
  if (r >= n) return;
  T res[NP];
  grp_scaled_residual<T, NP, G>(r, g, wcols, woff, R, x, res);
#pragma unroll
  for (int i = 0; i < NP; ++i) res[i] = bt[r * NP + i] - x[r * NP + i] - res[i];
#pragma unroll
  for (int m = 0; m < (NP + G - 1) / G; ++m) {
    const int j = g + m * G;
    if (j < NP) {
      T col[NP];
      load_row<T, NP>(Lt + r * NP2 + j * NP, col);
      T s = 0;
#pragma unroll
      for (int i = 0; i < NP; ++i) s += col[i] * res[i];
      t[r * NP + j] = s;
    }
  }
}

// ------------------------------------------------------------------
// hp front end: the lower-degree space embedded element by element by the
// constant nodal embedding T (n_p0 x n_p1, row-major).  Level-0 blocks of the
// lower-degree operator are T^T A_0(r, w) T in the same sliced pattern (both
// patterns hold W = n_f + 1 slots per slice), one thread per (slice, slot, k,
// l, lane).
template <int NP0, int NP1>
__global__ void k_galerkin_p(int64_t ns, int W, const double* __restrict__ A0, const double* __restrict__ Tm,
                             double* __restrict__ A1) {
  constexpr int N0 = NP0 * NP0, N1 = NP1 * NP1;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(idx % WAVE);
  int64_t rest = idx / WAVE;
  const int kl = (int)(rest % N1);
  rest /= N1;
  const int w = (int)(rest % W);
  const int64_t s = rest / W;
  if (s >= ns) return;
  const int k = kl / NP1, l = kl % NP1;
  const int64_t slot = s * W + w;  // the slot's block index in both layouts
  const double* a = A0 + slot * WAVE * N0 + lane;
  double acc = 0.0;
  for (int i = 0; i < NP0; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < NP0; ++j) t += a[(i * NP0 + j) * WAVE] * Tm[j * NP1 + l];
    acc += Tm[i * NP1 + k] * t;
  }
  A1[slot * WAVE * N1 + (int64_t)kl * WAVE + lane] = acc;
}

// level-0 residual + restriction to the lower-degree space, FP64 output for
// the lower hierarchy: t_r = T^T (b - A x)_r with the constant embedding T
// (n_p0 x n_p1, row-major)
template <typename T, int NP0, int NP1, int H, int NF, bool SYM>
__global__ __launch_bounds__(WAVE * H) void k_restrict0_rect(int64_t n, const int32_t* __restrict__ cols,
                                                             const int8_t* __restrict__ meta, const T* __restrict__ Ac,
                                                             const T* __restrict__ Ad, const T* __restrict__ b,
                                                             const T* __restrict__ x, const T* __restrict__ Tm,
                                                             double* __restrict__ t_out, int rev) {
  __shared__ T sh[H > 1 ? NP0 * WAVE : 1];
  const int lane = threadIdx.x % WAVE, h = threadIdx.x / WAVE;
  const int64_t sl = slice_order(rev), r = sl * WAVE + lane;
  const bool valid = r < n;
  T res[NP0];
  residual0<T, NP0, H, NF, SYM>(sl, r, lane, h, valid, cols, meta, Ac, Ad, b, x, sh, res);
  if (!valid) return;
  for (int j = h; j < NP1; j += H) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < NP0; ++i) s += Tm[i * NP1 + j] * res[i];
    t_out[r * NP1 + j] = (double)s;
  }
}

// prolongation from the lower-degree space: x_r += T z_r
template <typename T, int NP0, int NP1>
__global__ __launch_bounds__(TPB) void k_prolong_rect(int64_t n, const T* __restrict__ Tm, const T* __restrict__ z,
                                                      T* __restrict__ x) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  T zv[NP1];
#pragma unroll
  for (int k = 0; k < NP1; ++k) zv[k] = z[r * NP1 + k];
#pragma unroll
  for (int i = 0; i < NP0; ++i) {
    T s = 0;
#pragma unroll
    for (int k = 0; k < NP1; ++k) s += Tm[i * NP1 + k] * zv[k];
    x[r * NP0 + i] += s;
  }
}

// ----------------------------------------------------------- prescaling (setup)
// coarse strips: off-diagonal blocks of D^{-1} A, component-major, unpadded;
// one thread per (stored block b, i, j), b over the level's row-major blocks
template <typename T, int NP>
__global__ void k_scale_wpr(int64_t nnzb, const int32_t* __restrict__ blk_row, const int64_t* __restrict__ sblk,
                            const int64_t* __restrict__ woff, const double* __restrict__ A,
                            const double* __restrict__ Dinv, T* __restrict__ R) {
  constexpr int NP2 = NP * NP;
  // consecutive blocks (consecutive rows, sharing the lines of their
  // lane-interleaved D^{-1} and A entries) on one XCD
  const int64_t idx = xcd_slice() * blockDim.x + threadIdx.x;
  if (idx >= nnzb * NP2) return;
  const int64_t b = idx / NP2;
  const int ij = (int)(idx % NP2), i = ij / NP, j = ij % NP;
  const int64_t r = blk_row[b];
  const int64_t o = woff[r];
  const int w = (int)(b - o);
  if (w == 0) return;  // diagonal block
  const int K = (int)(woff[r + 1] - o - 1) * NP;
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  const double* D = Dinv + (r / WAVE) * WAVE * NP2 + lane;
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < NP; ++m) acc += D[(i * NP + m) * WAVE] * A[blk_off(B, w, NP2, m * NP + j, lane)];
  R[(o - r) * NP2 + (int64_t)i * K + (w - 1) * NP + j] = (T)acc;
}

// Lt_e = D_e^T L_e (D_e the diagonal block of A), so that
// Lt^T (D^{-1} r) = L^T r also for a nonsymmetric D; stored column by column
// per row, Lt_e(i, j) at e n_p^2 + j n_p + i, so that the restriction's lane
// for output j reads its column with wide loads; one thread per (row, i, j),
// rows fastest
template <typename T, int NP>
__global__ void k_scale_L(int64_t n, const int64_t* __restrict__ sblk, const double* __restrict__ A,
                          const double* __restrict__ L, T* __restrict__ Lt) {
  constexpr int NP2 = NP * NP;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(idx % WAVE);
  const int64_t rest = idx / WAVE;
  const int ij = (int)(rest % NP2);
  const int64_t s = rest / NP2;
  const int64_t r = s * WAVE + lane;
  if (r >= n) return;
  const int i = ij / NP, j = ij % NP;
  const int64_t B = sblk[s];
  double acc = 0.0;
#pragma unroll
  for (int m = 0; m < NP; ++m) acc += A[blk_off(B, 0, NP2, m * NP + i, lane)] * L[row_off(r, NP2, m * NP + j)];
  Lt[r * NP2 + j * NP + i] = (T)acc;
}

// ---------------------------------------------------------- outer (FP64) kernels
// b = M_0 f (caller order -> internal order)
template <int NP>
__global__ __launch_bounds__(TPB) void k_mass_in(int64_t n, const int32_t* __restrict__ perm,
                                                 const double* __restrict__ M, const double* __restrict__ f,
                                                 double* __restrict__ b) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t e = perm[r];
  double fv[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) fv[j] = f[e * NP + j];
  const double* Mr = M + (r / WAVE) * WAVE * NP2 + (r % WAVE);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += Mr[(i * NP + j) * WAVE] * fv[j];
    b[r * NP + i] = s;
  }
}

// y[perm[r]] = M_0 x[perm[r]] in caller order
template <int NP>
__global__ __launch_bounds__(TPB) void k_mass_apply(int64_t n, const int32_t* __restrict__ perm,
                                                    const double* __restrict__ M, const double* __restrict__ x,
                                                    double* __restrict__ y) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int64_t e = perm[r];
  double xv[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) xv[j] = x[e * NP + j];
  const double* Mr = M + (r / WAVE) * WAVE * NP2 + (r % WAVE);
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) s += Mr[(i * NP + j) * WAVE] * xv[j];
    y[e * NP + i] = s;
  }
}

// permutation of per-row vectors: dir 0: out[r] = in[perm[r]] (into internal), 1: out[perm[r]] = in[r]
template <typename T>
__global__ void k_permute(int64_t n, int np, const int32_t* __restrict__ perm, const T* __restrict__ in,
                          T* __restrict__ out, int dir) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * np) return;
  const int64_t r = idx / np, j = idx % np;
  if (dir == 0)
    out[idx] = in[(int64_t)perm[r] * np + j];
  else
    out[(int64_t)perm[r] * np + j] = in[idx];
}

// partial dot products: part[d * gridDim.x + block] for d < nd
__global__ __launch_bounds__(TPB) void k_dots(int64_t m, int nd, const double* __restrict__ a0,
                                              const double* __restrict__ b0, const double* __restrict__ a1,
                                              const double* __restrict__ b1, double* __restrict__ part) {
  __shared__ double sh[TPB / WAVE];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    s0 += a0[i] * b0[i];
    if (nd > 1) s1 += a1[i] * b1[i];
  }
  s0 = block_sum(s0, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s0;
  if (nd > 1) {
    s1 = block_sum(s1, sh);
    if (threadIdx.x == 0) part[gridDim.x + blockIdx.x] = s1;
  }
}

// Krylov scalars from the reduced dots: 0 FCG beta, 1 PCG beta, 2 FCG alpha,
// 3 PCG alpha (each also keeps the denominator for the next iteration)
__device__ __forceinline__ void krylov_scalars(double* s, int mode) {
  if (mode == 0) s[SC_BETA] = s[SC_ZQ] / s[SC_PQOLD];
  if (mode == 1) s[SC_BETA] = s[SC_ZR] / s[SC_ZROLD];
  if (mode == 2) {
    s[SC_ALPHA] = s[SC_PR] / s[SC_PQ];
    s[SC_PQOLD] = s[SC_PQ];
  }
  if (mode == 3) {
    s[SC_ALPHA] = s[SC_ZR] / s[SC_PQ];
    s[SC_ZROLD] = s[SC_ZR];
  }
}

// fixed-order reduction of nd partial arrays (nb entries each) into
// scal[off + d]; then, for mode >= 0, the Krylov scalars of that mode
// (one workgroup of RED_T threads; each thread's loads are issued together)
constexpr int RED_T = 1024;
__global__ __launch_bounds__(RED_T) void k_reduce(const double* __restrict__ part, int nb, int nd,
                                                  double* __restrict__ scal, int off, int mode) {
  __shared__ double sh[RED_T / WAVE];
  for (int d = 0; d < nd; ++d) {
    double s = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * RED_T < nb; i += 4 * RED_T) {
      const double a0 = part[d * nb + i], a1 = part[d * nb + i + RED_T], a2 = part[d * nb + i + 2 * RED_T],
                   a3 = part[d * nb + i + 3 * RED_T];
      s += (a0 + a1) + (a2 + a3);
    }
    for (; i < nb; i += RED_T) s += part[d * nb + i];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) scal[off + d] = s;
  }
  if (threadIdx.x == 0 && mode >= 0) krylov_scalars(scal, mode);
}


// x_hi + x_lo += alpha p (double-double); r -= alpha q; partial ||r||^2
__global__ __launch_bounds__(TPB) void k_update_xr2(int64_t m, const double* __restrict__ p,
                                                    const double* __restrict__ q, double* __restrict__ xh,
                                                    double* __restrict__ xl, double* __restrict__ r,
                                                    const double* __restrict__ s, double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double sh[TPB / WAVE];
  const double a = s[SC_ALPHA];
  double rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    const double y = (a * p[i]);
    const double ey = __builtin_fma(a, p[i], -y);
    double hi, e;
    two_sum(__builtin_nontemporal_load(xh + i), y, hi, e);
    const double lo = (__builtin_nontemporal_load(xl + i) + (e + ey));
    const double nh = (hi + lo);
    __builtin_nontemporal_store(nh, xh + i);
    __builtin_nontemporal_store((lo - (nh - hi)), xl + i);
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    rr += ri * ri;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = rr;
}

// ------------------------------------------------------------ GMRES (Sec. 4)
// Arnoldi basis V and preconditioned basis Z are row-major [vector][ld].
// k_multi_dot: partial sums of (V_i, w), i < nv, GMV vectors per pass over
// w; part[i gridDim.x + block].
constexpr int GMV = 8;
__global__ __launch_bounds__(TPB) void k_multi_dot(int64_t m, int nv, const double* __restrict__ V, int64_t ldv,
                                                   const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sh[TPB / WAVE];
  for (int g0 = 0; g0 < nv; g0 += GMV) {
    double acc[GMV];
#pragma unroll
    for (int t = 0; t < GMV; ++t) acc[t] = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
      const double wk = w[k];
#pragma unroll
      for (int t = 0; t < GMV; ++t)
        if (g0 + t < nv) acc[t] += V[(int64_t)(g0 + t) * ldv + k] * wk;
    }
#pragma unroll
    for (int t = 0; t < GMV; ++t) {
      const double s = block_sum(acc[t], sh);
      if (threadIdx.x == 0 && g0 + t < nv) part[(int64_t)(g0 + t) * gridDim.x + blockIdx.x] = s;
    }
  }
}

// w -= sum_{i < nv} h_i V_i
__global__ void k_multi_axpy(int64_t m, int nv, const double* __restrict__ V, int64_t ldv,
                             const double* __restrict__ hc, double* __restrict__ w) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  double s = 0.0;
  for (int i = 0; i < nv; ++i) s += hc[i] * V[(int64_t)i * ldv + k];
  w[k] -= s;
}

// dst = src / sqrt(*nrm2) (in place allowed)
__global__ void k_scale_vec(int64_t m, const double* src, const double* __restrict__ nrm2, double* dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  dst[k] = src[k] / sqrt(*nrm2);
}

// x_hi + x_lo += sum_{j < nk} y_j Z_j: the correction in FP64, added to the
// double-double iterate without rounding
__global__ void k_update_x_multi(int64_t m, int nk, const double* __restrict__ Z, int64_t ldz,
                                 const double* __restrict__ y, double* __restrict__ xh, double* __restrict__ xl) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double c = 0.0;
  for (int j = 0; j < nk; ++j) c = __builtin_fma(y[j], Z[(int64_t)j * ldz + i], c);
  double hi, e;
  two_sum(xh[i], c, hi, e);
  const double lo = (xl[i] + e);
  const double nh = (hi + lo);
  xh[i] = nh;
  xl[i] = (lo - (nh - hi));
}

// Outer FP64 product q = A_0 p on the facet-trace form (diagonal blocks dense,
// read from the sliced A_0 at slot 0) with the partial sums of (p, q) and
// (p, r) per slice (DOTS); COMP accumulates in Dot2.  All operator loads are
// non-temporal (read once per outer iteration).
template <int NP, int H, int NF, bool SYM, bool COMP, bool DOTS = true>
__global__ __launch_bounds__(WAVE * H) void k_spmv0(int64_t n, const int32_t* __restrict__ cols,
                                                    const int8_t* __restrict__ meta, const double* __restrict__ A,
                                                    const double* __restrict__ Ac, const double* __restrict__ p,
                                                    const double* __restrict__ rr, double* __restrict__ q,
                                                    double* __restrict__ part) {
#pragma clang fp contract(off)
  constexpr int NP2 = NP * NP, NI = NP / H;
  __shared__ double shs[H > 1 ? NP * WAVE : 1], shc[H > 1 && COMP ? NP * WAVE : 1];
  __shared__ double sh[H];
  const int lane = threadIdx.x % WAVE, h = threadIdx.x / WAVE;
  const int64_t sl = xcd_slice(), r = sl * WAVE + lane;
  const bool valid = r < n;
  Acc<double, COMP> acc[NI], sc[NP];
  if (valid) {
    // the diagonal blocks: slot 0 of the sliced A_0, or packed (SYM)
    const double* Dg = A + (SYM ? sl * RowBlk<NP, true>::N : sl * (NF + 1) * NP2) * WAVE + lane;
    if constexpr (SYM && H == 1) {
      // each stored entry loaded once and applied to both of its positions;
      // every row still receives its terms in ascending column order
      double pv[NP];
      load_row<double, NP>(p + r * NP, pv);
#pragma unroll
      for (int a = 0; a < NP; ++a)
#pragma unroll
        for (int c = a; c < NP; ++c) {
          const double v = __builtin_nontemporal_load(Dg + RowBlk<NP, true>::idx(a, c) * WAVE);
          acc[a].add(v, pv[c]);
          if (c != a) acc[c].add(v, pv[a]);
        }
    } else {
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        const double xj = p[r * NP + j];
#pragma unroll
        for (int t = 0; t < NI; ++t)
          acc[t].add(__builtin_nontemporal_load(Dg + RowBlk<NP, SYM>::idx(h * NI + t, j) * WAVE), xj);
      }
    }
    off0<double, NP, H, NF, COMP, false, true>(sl, lane, h, cols, meta, Ac, p, nullptr, 1.0, acc, sc);
  }
  gather_rows<double, NP, H, COMP>(lane, h, valid, acc, sc, shs, shc);
  double pq = 0.0, pr = 0.0;
  if (valid) {
    if constexpr (H == 1) {
      double qv[NP], pv[NP], rv[NP];
#pragma unroll
      for (int i = 0; i < NP; ++i) qv[i] = acc[i].value();
      store_row<double, NP>(q + r * NP, qv);
      if constexpr (DOTS) {
        load_row<double, NP>(p + r * NP, pv);
        load_row<double, NP>(rr + r * NP, rv);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          pq = __builtin_fma(pv[i], qv[i], pq);
          pr = __builtin_fma(pv[i], rv[i], pr);
        }
      }
    } else {
#pragma unroll
      for (int t = 0; t < NI; ++t) {
        const int i = h * NI + t;
        const double qi = acc[t].value();
        q[r * NP + i] = qi;
        if constexpr (DOTS) {
          const double pi = p[r * NP + i];
          pq = __builtin_fma(pi, qi, pq);
          pr = __builtin_fma(pi, rr[r * NP + i], pr);
        }
      }
    }
  }
  if constexpr (DOTS) {
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) part[sl] = pq;
    pr = block_sum(pr, sh);
    if (threadIdx.x == 0) part[gridDim.x + sl] = pr;
  }
}

// true residual rt = b - A (xh + xl) on the facet-trace form, compensated;
// partial ||rt||^2 per slice
template <int NP, int H, int NF, bool SYM>
__global__ __launch_bounds__(WAVE * H) void k_residual0(int64_t n, const int32_t* __restrict__ cols,
                                                        const int8_t* __restrict__ meta, const double* __restrict__ A,
                                                        const double* __restrict__ Ac, const double* __restrict__ b,
                                                        const double* __restrict__ xh, const double* __restrict__ xl,
                                                        double* __restrict__ rt, double* __restrict__ part) {
#pragma clang fp contract(off)
  constexpr int NP2 = NP * NP, NI = NP / H;
  __shared__ double shs[H > 1 ? NP * WAVE : 1], shc[H > 1 ? NP * WAVE : 1];
  __shared__ double sh[H];
  const int lane = threadIdx.x % WAVE, h = threadIdx.x / WAVE;
  const int64_t sl = xcd_slice(), r = sl * WAVE + lane;
  const bool valid = r < n;
  Acc<double, true> acc[NI], sc[NP];
  if (valid) {
    const double* Dg = A + (SYM ? sl * RowBlk<NP, true>::N : sl * (NF + 1) * NP2) * WAVE + lane;
#pragma unroll
    for (int t = 0; t < NI; ++t) acc[t].s = b[r * NP + h * NI + t];
    if constexpr (SYM && H == 1) {
      double hv[NP], lv[NP];
      load_row<double, NP>(xh + r * NP, hv);
      load_row<double, NP>(xl + r * NP, lv);
#pragma unroll
      for (int a = 0; a < NP; ++a)
#pragma unroll
        for (int c = a; c < NP; ++c) {
          const double v = -__builtin_nontemporal_load(Dg + RowBlk<NP, true>::idx(a, c) * WAVE);
          acc[a].add(v, hv[c]);
          acc[a].addlo(v, lv[c]);
          if (c != a) {
            acc[c].add(v, hv[a]);
            acc[c].addlo(v, lv[a]);
          }
        }
    } else {
#pragma unroll 2
      for (int j = 0; j < NP; ++j) {
        const double hj = xh[r * NP + j], lj = xl[r * NP + j];
#pragma unroll
        for (int t = 0; t < NI; ++t) {
          const double a = -__builtin_nontemporal_load(Dg + RowBlk<NP, SYM>::idx(h * NI + t, j) * WAVE);
          acc[t].add(a, hj);
          acc[t].addlo(a, lj);
        }
      }
    }
    off0<double, NP, H, NF, true, true, true>(sl, lane, h, cols, meta, Ac, xh, xl, -1.0, acc, sc);
  }
  gather_rows<double, NP, H, true>(lane, h, valid, acc, sc, shs, shc);
  double rr = 0.0;
  if (valid) {
#pragma unroll
    for (int t = 0; t < NI; ++t) {
      const double v = acc[t].value();
      rt[r * NP + h * NI + t] = v;
      rr = __builtin_fma(v, v, rr);
    }
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part[sl] = rr;
}

// out[perm[r]] = xh[r] + xl[r]
__global__ void k_out_dd(int64_t n, int np, const int32_t* __restrict__ perm, const double* __restrict__ xh,
                         const double* __restrict__ xl, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * np) return;
  const int64_t r = idx / np, j = idx % np;
  out[(int64_t)perm[r] * np + j] = xh[idx] + xl[idx];
}

// scalar bookkeeping (single thread)
// mode 0: FCG beta = s[ZQ] / s[PQOLD]; mode 1: PCG beta = s[ZR] / s[ZROLD]
// mode 2: FCG alpha = s[PR] / s[PQ], PQOLD = PQ; mode 3: PCG alpha = s[ZR] / s[PQ], ZROLD = ZR

// p = z + sign * beta * p  (first iteration: p = z); z in the multigrid
// precision; four entries per thread with wide loads and stores
constexpr int UP_K = 4;
template <typename T>
__global__ __launch_bounds__(TPB) void k_update_p(int64_t m, const T* __restrict__ z, double* __restrict__ p,
                                                  const double* __restrict__ s, double sign, int first) {
  const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * UP_K;
  if (i0 >= m) return;
  const double c = first ? 0.0 : sign * s[SC_BETA];
  if (i0 + UP_K <= m) {
    T zv[UP_K];
    double pv[UP_K];
    load_row<T, UP_K>(z + i0, zv);
    if (!first) load_row<double, UP_K>(p + i0, pv);
#pragma unroll
    for (int k = 0; k < UP_K; ++k) pv[k] = first ? (double)zv[k] : (double)zv[k] + c * pv[k];
    store_row<double, UP_K>(p + i0, pv);
  } else {
    for (int64_t i = i0; i < m; ++i) {
      const double zi = (double)z[i];
      p[i] = first ? zi : zi + c * p[i];
    }
  }
}

// partial sums of (z, v), z in the multigrid precision, grid-stride
template <typename T>
__global__ __launch_bounds__(TPB) void k_dot_t(int64_t m, const T* __restrict__ z, const double* __restrict__ v,
                                               double* __restrict__ part) {
  __shared__ double sh[TPB / WAVE];
  double s0 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
    s0 += (double)z[i] * v[i];
  s0 = block_sum(s0, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s0;
}

// x += alpha p; r -= alpha q; partial ||r||^2
__global__ __launch_bounds__(TPB) void k_update_xr(int64_t m, const double* __restrict__ p,
                                                   const double* __restrict__ q, double* __restrict__ x,
                                                   double* __restrict__ r, const double* __restrict__ s,
                                                   double* __restrict__ part) {
  __shared__ double sh[TPB / WAVE];
  const double a = s[SC_ALPHA];
  double rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
    __builtin_nontemporal_store(__builtin_nontemporal_load(x + i) + a * p[i], x + i);
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    rr += ri * ri;
  }
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = rr;
}


// g_e = -[ lam_e^T UA(e,0) u_e + sum_{hosted w} ( lam_e^T UA(e,w) u_c + u_e^T UA(e,w) lam_c
//          + lam_c^T UH(e,w) u_c ) ]   (caller-order output)
template <int NP>
__global__ __launch_bounds__(TPB) void k_grad_kappa(int64_t n, int W, const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ cols,
                                                    const int64_t* __restrict__ sblk,
                                                    const double* __restrict__ UA, const double* __restrict__ UH,
                                                    const int8_t* __restrict__ hostflag,
                                                    const double* __restrict__ u, const double* __restrict__ lam,
                                                    double* __restrict__ g) {
  constexpr int NP2 = NP * NP;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int lane = (int)(r % WAVE);
  const int64_t B = sblk[r / WAVE];
  double ue[NP], le[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    ue[j] = u[r * NP + j];
    le[j] = lam[r * NP + j];
  }
  double acc = 0.0;
  for (int i = 0; i < NP; ++i) {
    double s = 0.0;
    for (int j = 0; j < NP; ++j) s += UA[blk_off(B, 0, NP2, i * NP + j, lane)] * ue[j];
    acc += le[i] * s;
  }
  for (int w = 1; w < W; ++w) {
    if (hostflag[r * W + w] != 1) continue;
    const int32_t c = cols[B + (int64_t)WAVE * w + lane];
    double uc[NP], lc[NP];
    for (int j = 0; j < NP; ++j) {
      uc[j] = u[(int64_t)c * NP + j];
      lc[j] = lam[(int64_t)c * NP + j];
    }
    for (int i = 0; i < NP; ++i) {
      double s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int j = 0; j < NP; ++j) {
        const double a = UA[blk_off(B, w, NP2, i * NP + j, lane)];
        const double hh = UH[blk_off(B, w, NP2, i * NP + j, lane)];
        s1 += a * uc[j];
        s2 += a * lc[j];
        s3 += hh * uc[j];
      }
      acc += le[i] * s1 + ue[i] * s2 + lc[i] * s3;
    }
  }
  g[perm[r]] = -acc;
}

}  // namespace cdg
