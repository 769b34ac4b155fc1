// Device kernels of libcdgmg (gfx950, wave64).
//
// Block layouts (all levels): rows are grouped in slices of 64 (one wavefront).
// Operator blocks use a sliced-ELL layout: slice s owns W_s slots; the n_p x n_p
// block of (row r = 64 s + lane, slot w) is stored at
//     ((B_s + 64 w) * n_p^2) + (i n_p + j) * 64 + lane ,   B_s = slice_blk[s],
// so for fixed (w, i, j) the 64 rows of a slice are contiguous (coalesced).
// Per-row blocks (D^{-1}, coarse-level transfer blocks L_e, mass blocks) use
// the same layout with W = 1: (64 s) n_p^2 + (i n_p + j) 64 + lane; level 0 of a symmetric
// operator keeps D^{-1} and its diagonal blocks as upper triangles
// (n_p (n_p + 1) / 2 values per row, RowBlk in kernels.inl).  Vectors are
// row-major [row][n_p].  Slot 0 of every row is its diagonal block.  Level 0
// of the solve keeps its off-diagonal blocks in facet-trace form (their
// facet-node rows or columns only; kernels.inl) and forms its transfers L_e
// from each element's affine map and its parent's monomial coefficients.
//
// Cache use: the FP32 level-0 V-cycle data (the facet-trace values and D^{-1},
// 140 MB at 2D p = 3, 2e5 elements) is read four times per cycle and fits
// the 256 MB last-level cache in part.  The streams read once per cycle or
// per outer iteration (the FP64 outer operator, transfer data) use
// non-temporal loads so that they do not push it out.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cdg {

constexpr int WAVE = 64;
constexpr int TPB = 256;  // threads per block for row kernels (4 slices)

// device scalar slots of the outer Krylov loop
enum {
  SC_ZQ = 0, SC_PQOLD, SC_PQ, SC_PR, SC_RR, SC_BETA, SC_ALPHA, SC_ZR, SC_ZROLD, SC_BB, SC_TMP, SC_N = 16
};

// one term sign * P^T Q R of a plan-driven block product; element (i, j) of an
// operand X with stride s is X[(i n_p + j) s]; P or R null means identity
struct TPDev {
  const double* P;
  const double* Q;
  const double* R;
  int32_t sp, sq, sr, pad;
  double sign;
};
struct TPOut {
  double* O;
  int64_t so;
};

struct DevEll {
  int64_t n;              // rows
  const int32_t* cols;    // [sum W_s * 64]
  const int64_t* sblk;    // [nslices + 1]
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2:
// block b runs on XCD b % 8.  Rows follow the mesh order (neighbours mostly
// lie in nearby slices), so a kernel with one block per slice gives XCD k the
// k-th contiguous run of slices, and the neighbour gathers of its rows hit its
// own L2.  A bijection of [0, gridDim.x).
constexpr int NXCD = 8;
__device__ __forceinline__ int64_t xcd_slice() {
  const int64_t nb = gridDim.x, b = blockIdx.x;
  const int64_t q = nb / NXCD, rem = nb % NXCD, k = b % NXCD;
  return k * q + (k < rem ? k : rem) + b / NXCD;
}

// Passes over the level-0 V-cycle operator alternate their direction (rev):
// the operator is slightly larger than what the last-level cache keeps of it,
// and a pass that starts where the previous one ended finds that end still
// cached, where a pass in the same direction would find its start evicted.
// The order of rows does not change a Jacobi sweep's result.
__device__ __forceinline__ int64_t slice_order(int rev) {
  const int64_t s = xcd_slice();
  return rev ? (int64_t)gridDim.x - 1 - s : s;
}

__device__ __forceinline__ int64_t blk_off(int64_t B, int w, int np2, int ij, int lane) {
  return (B + (int64_t)WAVE * w) * np2 + (int64_t)ij * WAVE + lane;
}
__device__ __forceinline__ int64_t row_off(int64_t r, int np2, int ij) {
  return (r / WAVE) * WAVE * np2 + (int64_t)ij * WAVE + (r % WAVE);
}

// wave64 + block reduction of a double; result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int k = 0; k < nw; ++k) s += sh[k];
  }
  __syncthreads();
  return s;
}

}  // namespace cdg
