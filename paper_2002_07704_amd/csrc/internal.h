// Internal helpers shared by the HIP translation units of liblnv.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lnv.h"

namespace lnv {

// ---------------------------------------------------------------- errors
void set_hip_error(hipError_t e);

#define LNV_HIP(call)                          \
  do {                                         \
    hipError_t e_ = (call);                    \
    if (e_ != hipSuccess) {                    \
      ::lnv::set_hip_error(e_);                \
      return LNV_EHIP;                         \
    }                                          \
  } while (0)

#define LNV_LAUNCH_CHECK() LNV_HIP(hipGetLastError())

#define LNV_TRY(expr)            \
  do {                           \
    int st_ = (expr);            \
    if (st_ != LNV_OK) return st_; \
  } while (0)

// ---------------------------------------------------------------- launch shape
constexpr int kWave = 64;
constexpr int kNumXcd = 8;           // MI355X: 8 accelerator complex dies
constexpr int kVecGrid = 1024;       // fixed grid of the pattern-vector kernels

// Workgroups are dispatched round-robin over the XCDs (workgroup b runs on
// XCD b % 8).  Remapping gives XCD x the contiguous logical range
// [x*per, (x+1)*per), so neighbouring work items (spatially close atoms)
// share one XCD's L2.  The grid must be a multiple of 8.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int per = nblocks / kNumXcd;
  return (bid % kNumXcd) * per + bid / kNumXcd;
}

inline int round_up(int a, int b) { return (a + b - 1) / b * b; }

// Fixed-order wavefront sum (butterfly): identical association every run.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Block sum of one value per thread (blockDim.x a multiple of 64, <= 1024).
// Result valid in thread 0.  Fixed order.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int q = 0; q < nw; ++q) t += sh[q];
  return t;
}

// ---------------------------------------------------------------- symmetric halves
// Half of a symmetric pattern holding each pair {r, c} of different row groups
// once, balanced over the rows.  Rows are grouped in fours (singly when n is
// not a multiple of 4); inside one group every block is kept (both (r, c) and
// (c, r), which the mirror averages); for groups A != B (m groups) when the
// cyclic group offset D = (B - A) mod m has 2D < m, ties 2D = m by A < B.
// Every row keeps about half of its columns (the plain upper triangle c >= r
// keeps nearly all of an early row's columns and few of a late row's), and an
// atom stored as 4 rows keeps or drops a whole 4x4-blocked tile with another
// atom, so the half of a tile4 pattern is tile4.
__host__ __device__ inline bool in_half(int n, int r, int c) {
  const int g = (n & 3) == 0 ? 2 : 0;
  const int A = r >> g, B = c >> g, m = n >> g;
  if (A == B) return true;
  int D = B - A;
  if (D < 0) D += m;
  return 2 * D < m || (2 * D == m && A < B);
}

// Whether rows r and c fall in one group of the half's row grouping (then
// both (r, c) and (c, r) are in the half).
__host__ __device__ inline bool same_group(int n, int r, int c) {
  const int g = (n & 3) == 0 ? 2 : 0;
  return (r >> g) == (c >> g);
}

// ---------------------------------------------------------------- spatial index
// Kernel-side view of a pattern's lnv_index (passed by value).
struct Ix {
  const int* tab;
  const int* cell;
  const int* slot;
  const int* rp;      // the pattern's row_ptr (sub-row offsets of atom units)
  int g0, g1, g2, r0, r1, r2, w0, w1, w2, occ, qs;
  long long stride;
  long long sent;     // index of the table's trailing -1 entry (n_units * stride)
  int full;           // every axis's window is the whole axis
};

inline Ix make_ix(const lnv_pattern* p) {
  const lnv_index& x = p->ix;
  Ix v;
  v.tab = x.tab;
  v.cell = x.cell;
  v.slot = x.slot;
  v.rp = p->row_ptr;
  v.g0 = x.g[0]; v.g1 = x.g[1]; v.g2 = x.g[2];
  v.r0 = x.r[0]; v.r1 = x.r[1]; v.r2 = x.r[2];
  v.w0 = x.w[0]; v.w1 = x.w[1]; v.w2 = x.w[2];
  v.occ = x.occ;
  v.qs = x.qs;
  v.stride = x.stride;
  v.sent = (long long)(p->n >> x.qs) * x.stride;
  v.full = x.w[0] == x.g[0] && x.w[1] == x.g[1] && x.w[2] == x.g[2];
  return v;
}

inline bool has_ix(const lnv_pattern* p) { return p && p->ix.tab != nullptr; }

// Window coordinate of cell coordinate cb seen from ca (both in [0, g)),
// r <= g - 1: the wrapped offset (cb - ca + r) mod g, valid when below the
// window width w; when the window spans the whole axis (w == g) the absolute
// coordinate cb itself (every cell is in the window, and the coordinate of
// a column no longer depends on the row).
__device__ __forceinline__ int ix_axis(int cb, int ca, int r, int g, int w) {
  if (w == g) return cb;
  int d = cb - ca + r;
  d += d < 0 ? g : 0;
  d -= d >= g ? g : 0;
  return d;
}

// Offset in a row unit's table of the unit with packed cell cb and slot sb,
// seen from a row unit in packed cell ca; -1 outside the window.
__device__ __forceinline__ int ix_off(const Ix& x, int ca, int cb, int sb) {
  const int d0 = ix_axis(cb & 1023, ca & 1023, x.r0, x.g0, x.w0);
  const int d1 = ix_axis((cb >> 10) & 1023, (ca >> 10) & 1023, x.r1, x.g1, x.w1);
  const int d2 = ix_axis(cb >> 20, ca >> 20, x.r2, x.g2, x.w2);
  if (d0 >= x.w0 || d1 >= x.w1 || d2 >= x.w2) return -1;
  return ((d0 * x.w1 + d1) * x.w2 + d2) * x.occ + sb;
}

// Position of the block of unit row a, unit column b (the block of their
// first rows), or -1.
__device__ __forceinline__ int ix_unit(const Ix& x, int a, int b) {
  // with every window spanning its axis the row's cell does not matter
  const int o = ix_off(x, x.full ? 0 : x.cell[a], x.cell[b], x.slot[b]);
  return o < 0 ? -1 : x.tab[(size_t)a * x.stride + o];
}

// Position of block (i, j), or -1.
__device__ __forceinline__ int ix_find(const Ix& x, int i, int j) {
  const int e = ix_unit(x, i >> x.qs, j >> x.qs);
  if (e < 0 || x.qs == 0) return e;
  const int m = (1 << x.qs) - 1;
  const int i0 = i & ~m;
  return e + (i & m) * (x.rp[i0 + 1] - x.rp[i0]) + (j & m);
}

// ---------------------------------------------------------------- checks
// FP64 matrix (every call but the multiply and transpose takes FP64 only).
inline bool bsm_ok(const lnv_bsm* M) {
  return M && M->pat && M->val && M->dtype == LNV_F64 && M->pat->n > 0;
}

// FP64 or FP32 matrix.
inline bool bsm_ok_any(const lnv_bsm* M) {
  return M && M->pat && M->val && (M->dtype == LNV_F64 || M->dtype == LNV_F32) &&
         M->pat->n > 0;
}

// Internal multiply used by the public wrappers and by eval / CG.
//  store: write C;  m1/m2: dot partners on C's pattern (values, may be null)
//  partials: [2*C.n_items];  skip: device flag, kernel returns when != 0.
//  A, B, C share one dtype (FP64, or FP32 with FP32 accumulation); m1, m2
//  have C's dtype; the trace partials are FP64 either way.
int multiply_launch(double alpha, const lnv_bsm* A, const lnv_bsm* B, int transB,
                    double beta, const lnv_bsm* C, int store, const void* m1,
                    const void* m2, double* partials, const double* skip,
                    hipStream_t s);

// C1 = A1.B1 and C2 = A2.B2 (alpha 1, beta 0) in one launch when A1, A2 share
// a pattern and C1, C2 share a pattern with 4-row cluster plans; otherwise
// two multiply_launch calls.  Traces as in multiply_launch, per product.
int multiply_pair_launch(const lnv_bsm* A1, const lnv_bsm* B1, const lnv_bsm* C1,
                         const lnv_bsm* A2, const lnv_bsm* B2, const lnv_bsm* C2, int store,
                         const void* m11, const void* m12, double* part1, const void* m21,
                         const void* m22, double* part2, const double* skip, hipStream_t s);

// Symmetric products: U holds the blocks of C's symmetric pattern in the half
// in_half (pattern from lnv_pattern_half, with its own lut), C's pattern has
// lut and items.  mirror_launch fills C from U (C_ij = U_ij in the half,
// U_ji^T outside it, the symmetric part of U_ii on the diagonal); skip as in
// multiply_launch.
bool sym_ready(const lnv_bsm* U, const lnv_bsm* C);
int mirror_launch(const lnv_bsm* U, const lnv_bsm* C, hipStream_t s,
                  const double* skip = nullptr);

// AT (values on the pattern of A's transpose) = A^T block by block: block p
// of A goes, transposed, to position perm[p] (lnv_pattern_transpose_map).
int transpose_values(const lnv_bsm* A, const int32_t* perm, void* AT, hipStream_t s);

// Whether multiply_launch takes transB = 2 (B symmetric, its half stored)
// for these operands with store and no traces: the atom-tile path.
bool half_b_ok(const lnv_bsm* A, const lnv_bsm* B, const lnv_bsm* C);

// Number of dot partials (work items) multiply_launch writes for C.
int multiply_nparts(const lnv_bsm* A, const lnv_bsm* B, int transB, const lnv_bsm* C);

// Extreme eigenvalues of L S (occupation numbers) from `steps` Lanczos steps
// in the S inner product: out[0] <= out[1] (device), work: device
// [lnv_lanczos_len(n)].  No allocation, no host synchronisation.
int occupation_bounds(const lnv_bsm* L, const lnv_bsm* S, int steps, double* work, double* out,
                      hipStream_t s);

// Whether the optional multiply timing (lnv_timing_enable) is on: it creates
// HIP events as launches need them.
bool timing_on();

inline int32_t partial_items(const lnv_pattern* p) {
  return p->n_items > p->n_cl_items ? p->n_items : p->n_cl_items;
}

}  // namespace lnv
