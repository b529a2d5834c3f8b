// a3: numeric block-sparse multiply, FP64, 4x4 atom blocks.
//
// C_ij = alpha * sum_k A_ik op(B)_kj + beta * C_ij for the blocks (i,j) of
// C's pattern only -- the range-truncated sparse products through which
// every LNV quantity is formed at linear cost (Sec. II.C.2).
//
// Mapping to CDNA4 (gfx950):
//  * One wavefront owns up to 64 consecutive blocks (i, j_0..j_63) of one
//    output row and keeps each lane's 4x4 accumulator in registers for the
//    whole contraction (no atomics, fixed summation order).
//  * The k loop runs over A's row i, identical for every lane, so the A block
//    is wave-uniform and lives in scalar registers (one s_load per block,
//    broadcast to all 64 lanes by the VALU's scalar operand).
//  * Each lane finds B_kj in O(1) through the spatial index of B's pattern
//    (one table entry per window cell and slot, see lnv_index; the lane's
//    column is fixed, so only the step's row k changes the entry) and
//    streams the 128-byte block as 8 dwordx4 loads; index loads run ahead of
//    the block loads.
//  * Products are 64 v_fma_f64 per (i,k,j) triple on the FP64 VALU, which on
//    MI355X has the same 78.6 TFLOP/s peak as the FP64 matrix cores; a 4x4
//    block triple is far smaller than an MFMA tile and packing several atoms
//    into a tile multiplies the flops of these range-limited patterns by ~5.
//  * Workgroups of 4 wavefronts; logical workgroup ids are remapped so each
//    XCD processes a contiguous range of rows (spatially close atoms share
//    the B blocks in that XCD's L2).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>
#include <vector>

#include "internal.h"

namespace lnv {
namespace {

// Values are stored as T; products and sums are formed in Acc: FP64 / FP64,
// or for the mixed-precision products FP32 values with FP32 multiply-add
// (Acc = float) or with FP64 multiply-add (Acc = double: the product of two
// FP32 values is exact in FP64, so only the sums round).
template <int TRANS_B, typename T, typename Acc>
__device__ __forceinline__ void block_fma(Acc (&acc)[16], const T (&a)[16], const T (&b)[16]) {
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const T bv = TRANS_B ? b[c * 4 + m] : b[m * 4 + c];
        acc[r * 4 + c] = fma((Acc)a[r * 4 + m], (Acc)bv, acc[r * 4 + c]);
      }
}

// One 4x4 block as 16-byte vector loads / stores (8 for FP64, 4 for FP32).
__device__ __forceinline__ void load_block(double (&b)[16], const double* __restrict__ p) {
  const double2* q = reinterpret_cast<const double2*>(p);
#pragma unroll
  for (int h = 0; h < 8; ++h) {
    const double2 v = q[h];
    b[2 * h] = v.x;
    b[2 * h + 1] = v.y;
  }
}

__device__ __forceinline__ void load_block(float (&b)[16], const float* __restrict__ p) {
  const float4* q = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const float4 v = q[h];
    b[4 * h] = v.x;
    b[4 * h + 1] = v.y;
    b[4 * h + 2] = v.z;
    b[4 * h + 3] = v.w;
  }
}

__device__ __forceinline__ void store_block(double* __restrict__ p, const double (&o)[16]) {
  double2* q = reinterpret_cast<double2*>(p);
#pragma unroll
  for (int h = 0; h < 8; ++h) q[h] = make_double2(o[2 * h], o[2 * h + 1]);
}

__device__ __forceinline__ void store_block(float* __restrict__ p, const float (&o)[16]) {
  float4* q = reinterpret_cast<float4*>(p);
#pragma unroll
  for (int h = 0; h < 4; ++h) q[h] = make_float4(o[4 * h], o[4 * h + 1], o[4 * h + 2], o[4 * h + 3]);
}

// Epilogue of one output block: out = alpha acc + beta C_old, optional store,
// and the FP64 trace contributions <m1, out>, <m2, out>.
template <int STORE, int NDOT, typename T, typename Acc>
__device__ __forceinline__ void finish_block(const Acc (&acc)[16], T* __restrict__ c_val,
                                             size_t cp, double alpha, double beta,
                                             const T* __restrict__ m1,
                                             const T* __restrict__ m2, double& d1, double& d2) {
  T out[16];
  const Acc al = (Acc)alpha, be = (Acc)beta;
  if (beta != 0.0) {
    T old[16];
    load_block(old, c_val + cp);
#pragma unroll
    for (int e = 0; e < 16; ++e) out[e] = (T)(al * acc[e] + be * (Acc)old[e]);
  } else {
#pragma unroll
    for (int e = 0; e < 16; ++e) out[e] = (T)(al * acc[e]);
  }
  if (STORE) store_block(c_val + cp, out);
  if (NDOT >= 1) {
    T mv[16];
    load_block(mv, m1 + cp);
#pragma unroll
    for (int e = 0; e < 16; ++e) d1 = fma((double)mv[e], (double)out[e], d1);
  }
  if (NDOT >= 2) {
    T mv[16];
    load_block(mv, m2 + cp);
#pragma unroll
    for (int e = 0; e < 16; ++e) d2 = fma((double)mv[e], (double)out[e], d2);
  }
}

// Lookups of B's blocks for a lane whose output column j is fixed for the
// whole contraction: the column's half of the window lookup (its cell, slot
// and sub-column) is taken once, the step's row k supplies the rest.
struct ColKey {
  int cb, sb, jt;
};

__device__ __forceinline__ ColKey col_key(const Ix& x, int j) {
  const int b = j >> x.qs;
  return ColKey{x.cell[b], x.slot[b], j & ((1 << x.qs) - 1)};
}

// Position of B's block (k, j), or -1.
__device__ __forceinline__ int find_kj(const Ix& x, const ColKey& c, int k) {
  const int a = k >> x.qs;
  const int o = ix_off(x, x.cell[a], c.cb, c.sb);
  if (o < 0) return -1;
  const int e = x.tab[(size_t)a * x.stride + o];
  if (e < 0 || x.qs == 0) return e;
  const int k0 = k & ~3;
  return e + (k & 3) * (x.rp[k0 + 1] - x.rp[k0]) + c.jt;
}

// The transposed read op(B) = B^T needs block (j, k): row j is the lane's.
struct RowKey {
  int ca, it, len;
  size_t base;
};

__device__ __forceinline__ RowKey row_key(const Ix& x, int j) {
  const int a = j >> x.qs;
  const int j0 = j & ~((1 << x.qs) - 1);
  return RowKey{x.cell[a], j & ((1 << x.qs) - 1), x.qs ? x.rp[j0 + 1] - x.rp[j0] : 0,
                (size_t)a * x.stride};
}

__device__ __forceinline__ int find_jk(const Ix& x, const RowKey& r, int k) {
  const int b = k >> x.qs;
  const int o = ix_off(x, r.ca, x.cell[b], x.slot[b]);
  if (o < 0) return -1;
  const int e = x.tab[r.base + o];
  if (e < 0 || x.qs == 0) return e;
  return e + r.it * r.len + (k & 3);
}

// Table entry address of block (k, j) for the index loads of the pipelined
// kernels (column j fixed per lane, row k's packed cell ck uniform per step):
// the sentinel entry (-1) when j is outside the window of k or the lane idle.
// o_full: the lane's offset when every window spans its axis (then it does
// not depend on k), -1 for an idle lane.
__device__ __forceinline__ const int* entry_kj(const Ix& x, int k, int ck, int cb, int sb,
                                               bool act, int o_full) {
  const int o = x.full ? o_full : (act ? ix_off(x, ck, cb, sb) : -1);
  return x.tab + (o < 0 ? (size_t)x.sent : (size_t)(k >> x.qs) * x.stride + o);
}

// One row piece per wave, one lane per output column (TC: C's value type,
// T: A's and B's).
template <int TRANS_B, int STORE, int NDOT, typename T, typename Acc, typename TC = T>
__global__ __launch_bounds__(256) void k_mul44(
    int n, int n_items, const int* __restrict__ items, const int* __restrict__ a_rp,
    const int* __restrict__ a_col, const T* __restrict__ a_val, Ix bx,
    const T* __restrict__ b_val, const int* __restrict__ c_rp, const int* __restrict__ c_col,
    TC* __restrict__ c_val, double alpha, double beta, const TC* __restrict__ m1,
    const TC* __restrict__ m2, double* __restrict__ partials, const double* __restrict__ skip) {
  if (skip != nullptr && *skip != 0.0) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (item >= n_items) return;
  const int lane = threadIdx.x & 63;
  const int i = items[2 * item];
  const int c0 = items[2 * item + 1];
  const int cnt = min(kWave, c_rp[i + 1] - c0);
  const bool act = lane < cnt;
  const int j = act ? c_col[c0 + lane] : 0;
  // op(B)_kj: B's block (k, j), or for the transposed read block (j, k)
  const ColKey ck = col_key(bx, j);
  const RowKey rk = row_key(bx, j);
  auto bpos = [&](int k) -> int { return TRANS_B ? find_jk(bx, rk, k) : find_kj(bx, ck, k); };
  const int t0 = a_rp[i], t1 = a_rp[i + 1];

  Acc acc[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) acc[e] = 0;

  T bA[16], bB[16], a[16];
  int pA = -1, pB = -1;
  if (act && t0 < t1) pA = bpos(a_col[t0]);
  if (act && t0 + 1 < t1) pB = bpos(a_col[t0 + 1]);
  if (pA >= 0) load_block(bA, b_val + (size_t)pA * 16);

  for (int t = t0; t < t1; t += 2) {
    // step t: consume bA, fetch bB (step t+1) and the index of step t+2
    int pA2 = -1;
    if (act && t + 2 < t1) pA2 = bpos(a_col[t + 2]);
    if (pB >= 0) load_block(bB, b_val + (size_t)pB * 16);
    {
      const T* ap = a_val + (size_t)t * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = ap[q];
      if (pA >= 0) block_fma<TRANS_B>(acc, a, bA);
    }
    if (t + 1 >= t1) break;
    // step t+1: consume bB, fetch bA (step t+2) and the index of step t+3
    int pB2 = -1;
    if (act && t + 3 < t1) pB2 = bpos(a_col[t + 3]);
    if (pA2 >= 0) load_block(bA, b_val + (size_t)pA2 * 16);
    {
      const T* ap = a_val + (size_t)(t + 1) * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) a[q] = ap[q];
      if (pB >= 0) block_fma<TRANS_B>(acc, a, bB);
    }
    pA = pA2;
    pB = pB2;
  }

  double d1 = 0.0, d2 = 0.0;
  if (act) finish_block<STORE, NDOT>(acc, c_val, (size_t)(c0 + lane) * 16, alpha, beta, m1, m2, d1, d2);
  if (NDOT >= 1) {
    d1 = wave_sum(d1);
    if (NDOT >= 2) d2 = wave_sum(d2);
    if (lane == 0) {
      partials[2 * item] = d1;
      partials[2 * item + 1] = d2;
    }
  }
}

// Clustered variant with one lane per column (G = 1), software-pipelined so
// that the only memory round trips a contraction step exposes are its A
// blocks' (scalar loads, shared by the 4 waves of a cluster).  Per step t a
// wave issues, in this order: one index load (lanes 0-3: the 4 rows' A
// positions of step t+1, lanes 4-7: those of step t+3, lanes 8-31: k of step
// t+4, lanes 32-63: the packed cell of that k), the B index (the table entry
// of B's spatial index) of step t+3, the B block of step t+2 and
// a vector load of the 4 A blocks of step t+2 (one element per lane; it only
// brings them into L2 ahead of the scalar loads, which then hit there); it
// then multiplies B(t) into the rows present.  Every vector load is issued
// unconditionally -- steps before the first or past the last read clamped
// indices, idle lanes column 0's entry, missing B blocks block 0 -- so each
// iteration issues the same loads in the same order and the waits count them
// exactly (idle lanes and columns outside the window of k read the index's
// trailing -1): step t waits for the previous step's index loads and for B(t),
// never for B(t+1), B(t+2) in flight.  The loop starts two steps early, so
// the first blocks are fetched by the loop body itself.
template <typename T, typename Acc>
__device__ __forceinline__ void rows_fma(Acc (&acc)[4][16], const T (&b)[16], const int (&pos)[4],
                                         const T* __restrict__ a_val) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int p0 = pos[2 * h], p1 = pos[2 * h + 1];
    T a0[16], a1[16];
    if (p0 >= 0) {
      const T* ap = a_val + (size_t)p0 * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) a0[q] = ap[q];
    }
    if (p1 >= 0) {
      const T* ap = a_val + (size_t)p1 * 16;
#pragma unroll
      for (int q = 0; q < 16; ++q) a1[q] = ap[q];
    }
    if (p0 >= 0) block_fma<0>(acc[2 * h], a0, b);
    if (p1 >= 0) block_fma<0>(acc[2 * h + 1], a1, b);
  }
}

// PAIR: a second product in the same launch, selected by blockIdx.y, with
// the same A and C patterns (so the same cluster plans and pieces) and its
// own values, B and traces (all from kernel arguments, so the A blocks stay
// on the scalar path).
template <int PAIR, int STORE, int NDOT, typename T, typename Acc>
__global__ __launch_bounds__(256) void k_mul44c1(
    int n, int n_items, const int* __restrict__ items, const int* __restrict__ ka_ptr,
    const int* __restrict__ ka_col, const int* __restrict__ ka_pos,
    const int* __restrict__ ka_key, const T* __restrict__ a_val1, Ix bx1,
    const T* __restrict__ b_val1, const int* __restrict__ jc_ptr,
    const int* __restrict__ jc_col, const int* __restrict__ jc_pos, T* __restrict__ c_val1,
    double alpha, double beta, const T* __restrict__ m1_1, const T* __restrict__ m2_1,
    double* __restrict__ partials1, const double* __restrict__ skip,
    const T* __restrict__ a_val2, Ix bx2,
    const T* __restrict__ b_val2, T* __restrict__ c_val2, const T* __restrict__ m1_2,
    const T* __restrict__ m2_2, double* __restrict__ partials2) {
  if (skip != nullptr && *skip != 0.0) return;
  const bool second = PAIR && blockIdx.y != 0;
  const T* __restrict__ a_val = second ? a_val2 : a_val1;
  const Ix bx = second ? bx2 : bx1;
  const T* __restrict__ b_val = second ? b_val2 : b_val1;
  T* __restrict__ c_val = second ? c_val2 : c_val1;
  const T* __restrict__ m1 = second ? m1_2 : m1_1;
  const T* __restrict__ m2 = second ? m2_2 : m2_1;
  double* __restrict__ partials = second ? partials2 : partials1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (item >= n_items) return;
  const int lane = threadIdx.x & 63;
  const int c = items[2 * item];
  const int p0 = items[2 * item + 1];
  const int cnt = min(kWave, jc_ptr[c + 1] - p0);
  const bool act = lane < cnt;
  const int j = act ? jc_col[p0 + lane] : 0;
  int opos[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) opos[r] = act ? jc_pos[(size_t)(p0 + lane) * 4 + r] : -1;
  // the column's half of B's window lookup (B's units are rows here)
  const int cb = bx.cell[j], sb = bx.slot[j];
  const int o_full = act ? ix_off(bx, 0, cb, sb) : -1;
  const int t0 = ka_ptr[c], t1 = ka_ptr[c + 1];

  Acc acc[4][16];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[r][e] = 0;

  if (t0 < t1) {
    const int tl = t1 - 1;
    // index loads of step t: A positions of steps t+1 (lanes 0-3) and t+3
    // (lanes 4-7), k of step t+4 (lanes 8-31) and its cell (lanes 32-63)
    auto idx_src = [&](int t) -> const int* {
      return lane < 4    ? ka_pos + (size_t)min(max(t + 1, t0), tl) * 4 + lane
             : lane < 8  ? ka_pos + (size_t)min(max(t + 3, t0), tl) * 4 + (lane - 4)
             : lane < 32 ? ka_col + min(t + 4, tl)
                         : ka_key + 2 * (size_t)min(t + 4, tl);
    };
    // A element of step t+2 this lane loads ahead (row lane/16, entry lane%16)
    const int ar = (lane >> 4) & 3, ae = lane & 15;
    const int ts = t0 - 2;
    // the loads of the step before the first: B index of step t0 (as L2),
    // the index vector (k of step t0+1 in lanes 8-63) and a B block into b1
    // (block 0, never used).  The block's offset is an opaque zero computed
    // from the index vector, so it is issued last, as in every loop step, and
    // the counts of loads in flight at the loop head agree on both paths.
    int l0 = -1, l1 = -1;                      // B positions (index table entries)
    int l2 = *entry_kj(bx, ka_col[t0], ka_key[2 * (size_t)t0], cb, sb, act, o_full);
    int iv = *idx_src(ts - 1);
    T b0[16], b1[16], b2[16];
    int zero = 0;
    asm volatile("" : "+v"(zero) : "v"(iv));
    load_block(b1, b_val + (size_t)zero * 16);
    T x0 = a_val[zero], x1 = x0, x2 = x0;

// step t: consume BC = B(t) (index LC), issue B(t+2) into BN from index L2,
// overwrite LC with the index of step t+3
#define LNV_C1_STEP(t, BC, BN, LC, L2, XC)                                     \
  {                                                                            \
    const int ivn = *idx_src(t);                                               \
    const int k3 = __builtin_amdgcn_readlane(iv, 8);                           \
    const int c3 = __builtin_amdgcn_readlane(iv, 32);                          \
    int pos[4], pf[4];                                                         \
    _Pragma("unroll") for (int r = 0; r < 4; ++r) {                            \
      pos[r] = __builtin_amdgcn_readlane(iv, r);                               \
      pf[r] = __builtin_amdgcn_readlane(iv, 4 + r);                            \
    }                                                                          \
    const bool use = act && (t) >= t0 && (t) < t1 && LC >= 0;                  \
    LC = *entry_kj(bx, k3, c3, cb, sb, act, o_full);                           \
    load_block(BN, b_val + (size_t)max(L2, 0) * 16);                           \
    asm volatile("" ::"v"(XC));                                                \
    {                                                                          \
      const int pa = ar == 0 ? pf[0] : ar == 1 ? pf[1] : ar == 2 ? pf[2] : pf[3]; \
      XC = a_val[(size_t)max(pa, 0) * 16 + ae];                                \
    }                                                                          \
    if ((t) >= t0 && (t) < t1 && use) rows_fma(acc, BC, pos, a_val);          \
    iv = ivn;                                                                  \
  }
    for (int t = ts; t < t1; t += 3) {
      LNV_C1_STEP(t, b0, b2, l0, l2, x0)
      LNV_C1_STEP(t + 1, b1, b0, l1, l0, x1)
      LNV_C1_STEP(t + 2, b2, b1, l2, l1, x2)
    }
    asm volatile("" ::"v"(x0), "v"(x1), "v"(x2));
#undef LNV_C1_STEP
  }

  double d1 = 0.0, d2 = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
    if (opos[r] >= 0)
      finish_block<STORE, NDOT>(acc[r], c_val, (size_t)opos[r] * 16, alpha, beta, m1, m2, d1, d2);
  if (NDOT >= 1) {
    d1 = wave_sum(d1);
    if (NDOT >= 2) d2 = wave_sum(d2);
    if (lane == 0) {
      partials[2 * item] = d1;
      partials[2 * item + 1] = d2;
    }
  }
}

// ------------------------------------------------------------------ atom tiles
// Atoms with 13 support functions (the DZP-like silicon basis) are stored as
// 4 consecutive 4x4-blocked rows each (padded to 16 functions), so the block
// of an atom pair is a dense 16x16 tile and an atom triple (i,k,j) is a dense
// 16x16x16 contraction: the shape of the matrix-core (MFMA) instructions.
// Requirements (checked on the host): A's and B's patterns are "tile4" (the 4
// rows of an atom hold the same columns, in aligned runs 4b..4b+3, so a tile's
// 16 sub-blocks sit at pos(sub-row 0) + s*len + t), A and C carry 16-row
// cluster plans (4 atoms per cluster, the union of their columns in aligned
// runs of 4), B carries its spatial index over atoms (qs = 2).
//
// A wavefront owns 4 cluster atoms x NB column atoms, i.e. 4*NB accumulator
// tiles (4 values per lane per tile), and runs the k loop over the cluster's
// union of A columns one atom (4 union entries) per step; each A tile is used
// for NB outputs, each B tile for the 4 cluster atoms.  Tiles missing from A,
// B or the output are skipped with wave-uniform branches.
//
// Operand layout (all modes): lane l = i + 16c holds row i of A's tile at
// k = 4c..4c+3 (one 4-value row of a 4x4 block: a 16-byte load in FP32) and
// column i of B's tile at k = 4c..4c+3 (four values 16 bytes apart).
// Arithmetic modes (MODE):
//  TM_F32    v_mfma_f32_16x16x4_f32, four per tile and step: instruction p
//            takes the p-th of each lane's four values, i.e. contracts
//            k = 4c + p over the lane groups c (the instruction's 16x4 by
//            4x16 operands with k permuted; the sum over p covers all 16 k).
//  TM_F64    v_mfma_f64_16x16x4_f64, the same in FP64 (FP64 storage, or FP32
//            storage widened exactly: FP64 products and sums).
//  TM_F16X3  FP16 hi/lo split on v_mfma_f32_16x16x16_f16 (whose operands are
//            exactly these four-value rows and columns): x*2^8 = hi + lo with
//            hi = fp16(x*2^8), lo = fp16(x*2^8 - hi) (22 significant bits in
//            all), and A.B formed as Ah.Bh + Ah.Bl + Al.Bh (the dropped Al.Bl
//            is ~2^-22 of a term), then scaled by 2^-16.  The 2^8 scaling
//            keeps lo out of FP16's subnormal range for |x| >= 5e-4 and
//            overflows for |x| >= 255 (far above any entry of S, H, L or
//            their products here).
// Output tile: lane l = n + 16g holds column n, rows 4g..4g+3 (FP32
// accumulators) or rows g, g+4, g+8, g+12 (FP64), as measured on gfx950.
// Steps: a ballot scan finds the steps with a pair to multiply, 64 at a time
// (one step per lane, see k_tile16); the fragments of the next kept step are
// loaded before the current step's products, all unconditionally from
// clamped positions, so the compiler's wait counts stay exact.
enum { TM_F32 = 0, TM_F64 = 1, TM_F16X3 = 2 };

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4_t __attribute__((ext_vector_type(4)));

template <int MODE>
struct TileAcc {
  using type = f32x4_t;
};
template <>
struct TileAcc<TM_F64> {
  using type = f64x4_t;
};

constexpr float kF16Scale = 256.0f;               // 2^8 per operand
constexpr double kF16Unscale = 1.0 / 65536.0;     // 2^-16 on the product

__device__ __forceinline__ void split_f16(const float (&x)[4], f16x4_t& hi, f16x4_t& lo) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const float s = x[e] * kF16Scale;
    const _Float16 h = (_Float16)s;
    hi[e] = h;
    lo[e] = (_Float16)(s - (float)h);
  }
}

// Fragments of one step: a[ar][.] for the 4 cluster atoms, b[q][.] for the NB
// column atoms (block positions pa / pb of sub-row 0, -1 when the tile is
// missing; rowA[ar] = (lane's sub-row) * A's row length of that atom).  Lane
// l = i + 16c holds a[ar][w] = A[i][4c + w] (row i of the tile: one 4-value
// row of block (i>>2, c)) and b[q][w] = B[4c + w][i] (column i of block
// (c, i>>2)), w = 0..3.  TB = 1 reads B as the transpose of the stored
// matrix B': B[4c + w][i] = B'[i][4c + w], row i of the tile (j, k) of B',
// a 4-value row of its block (i>>2, c); lenB then holds, per column atom q,
// the row length of that atom in B' (lenBq), else lenB is the step's.
// TB = 2: B is symmetric and stored as the blocks of its half (in_half):
// tile (k, j_q) is read as stored when (k, j_q) is in the half and as the
// transpose of tile (j_q, k) otherwise (bit q of tmask), each in the layout
// above.
template <typename T>
__device__ __forceinline__ void tile_load_a_row(T (&a)[4], int pa, const T* __restrict__ a_val,
                                                int rowA, int li, int lq, int amax) {
  const int blk = min(max(pa, 0) + rowA + lq, amax);
  const T* ap = a_val + (size_t)blk * 16 + (li & 3) * 4;
#pragma unroll
  for (int w = 0; w < 4; ++w) a[w] = ap[w];
}

template <typename T>
__device__ __forceinline__ void tile_load_a(T (&a)[4][4], const int (&pa)[4],
                                            const T* __restrict__ a_val, const int (&rowA)[4],
                                            int li, int lq, int amax) {
#pragma unroll
  for (int ar = 0; ar < 4; ++ar) tile_load_a_row<T>(a[ar], pa[ar], a_val, rowA[ar], li, lq, amax);
}

template <int NB, int TB, typename T>
__device__ __forceinline__ void tile_load_b(T (&b)[NB][4], const int (&pb)[NB], int lenB,
                                            const int (&lenBq)[NB], const T* __restrict__ b_val,
                                            int li, int lq, int bmax, int tmask = 0) {
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    if (TB == 1 || (TB == 2 && ((tmask >> q) & 1))) {
      const int blk = min(max(pb[q], 0) + (li >> 2) * lenBq[q] + lq, bmax);
      const T* bp = b_val + (size_t)blk * 16 + (li & 3) * 4;
#pragma unroll
      for (int w = 0; w < 4; ++w) b[q][w] = bp[w];
    } else {
      const int blk = min(max(pb[q], 0) + lq * lenB + (li >> 2), bmax);
      const T* bp = b_val + (size_t)blk * 16 + (li & 3);
#pragma unroll
      for (int w = 0; w < 4; ++w) b[q][w] = bp[w * 4];
    }
  }
}

template <int NB, int TB, typename T>
__device__ __forceinline__ void tile_load(T (&a)[4][4], T (&b)[NB][4], const int (&pa)[4],
                                          const int (&pb)[NB], int lenB, const int (&lenBq)[NB],
                                          const T* __restrict__ a_val,
                                          const T* __restrict__ b_val, const int (&rowA)[4],
                                          int li, int lq, int amax, int bmax, int tmask) {
  tile_load_a<T>(a, pa, a_val, rowA, li, lq, amax);
  tile_load_b<NB, TB, T>(b, pb, lenB, lenBq, b_val, li, lq, bmax, tmask);
}

// Products of one step on the matrix cores: act bit 4q + ar set where A's
// tile of cluster atom ar, B's tile of column atom q and the output tile all
// exist (the other pairs are not multiplied).
// done(ar) runs once the products no longer read A's fragment ar (FP64 and
// FP32: after its row of products; FP16 split: after all of them), so the
// caller can load the next step's fragment into it while the later rows
// multiply.
struct NoRowDone {
  __device__ void operator()(int) const {}
};

template <int MODE, int NB, typename T, typename AccT, typename RowDone = NoRowDone>
__device__ __forceinline__ void tile_mma(AccT (&acc)[4][NB], const T (&a)[4][4],
                                         const T (&b)[NB][4], int act,
                                         RowDone done = RowDone{}) {
  if constexpr (MODE == TM_F16X3) {
    f16x4_t ah[4], al[4], bh[NB], bl[NB];
#pragma unroll
    for (int ar = 0; ar < 4; ++ar) split_f16(a[ar], ah[ar], al[ar]);
#pragma unroll
    for (int q = 0; q < NB; ++q) split_f16(b[q], bh[q], bl[q]);
#pragma unroll
    for (int ar = 0; ar < 4; ++ar) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (!((act >> (4 * q + ar)) & 1)) continue;
        // the step's three products start from zero and join the running sum
        // through a rounded VALU add, so rounding in the matrix unit's own
        // accumulation does not build up over the contraction
        f32x4_t t = {0.f, 0.f, 0.f, 0.f};
        t = __builtin_amdgcn_mfma_f32_16x16x16f16(al[ar], bh[q], t, 0, 0, 0);
        t = __builtin_amdgcn_mfma_f32_16x16x16f16(ah[ar], bl[q], t, 0, 0, 0);
        t = __builtin_amdgcn_mfma_f32_16x16x16f16(ah[ar], bh[q], t, 0, 0, 0);
        acc[ar][q] += t;
      }
    }
    // the next step's A loads after all products (issued right after the
    // split they made the split's step 9% slower on the 32768-atom cell)
#pragma unroll
    for (int ar = 0; ar < 4; ++ar) done(ar);
  } else {
#pragma unroll
    for (int ar = 0; ar < 4; ++ar) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (!((act >> (4 * q + ar)) & 1)) continue;
        // instruction p contracts k = 4c + p over the lane groups c
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          if constexpr (MODE == TM_F64)
            acc[ar][q] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[ar][p], (double)b[q][p],
                                                             acc[ar][q], 0, 0, 0);
          else
            acc[ar][q] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[ar][p], (float)b[q][p],
                                                             acc[ar][q], 0, 0, 0);
        }
      }
      done(ar);
    }
  }
}

// One step of a piece's contraction: the cluster atoms' A tile positions,
// the column atoms' B tile positions (-1: missing), B's row length of the
// step's atom, the pairs to multiply (tile_mma).
template <int NB>
struct TileStep {
  int pa[4], pb[NB], lenB, act, tmask;
};

// Atom-tile multiply on the matrix cores.  A wave owns one piece: the 4
// atoms of a 16-row cluster c (4 rows each) times NB column atoms of the
// cluster's output list, 4 x NB output tiles of 16 x 16 held in the matrix
// accumulators; the contraction runs over the atoms k of the cluster's
// contraction list (the union of its rows' columns of A).
//
// The list is scanned 64 steps at a time, one step per lane: each lane looks
// up its step's A tiles (the cluster plan) and B tiles (B's spatial index,
// cell window of atom k against each column atom's cell), and a ballot keeps
// the steps with at least one pair to multiply -- with finite ranges most
// steps of a piece meet none of its column atoms.  The kept steps are then
// taken in order (lowest lane first), their positions read from the owning
// lane, the fragments of the next kept step loaded while the current one
// multiplies.  Lookups are independent per lane, so a chunk costs one
// round of memory latency rather than one per step; the products and their
// order are those of the full list.
template <int NB, int MODE, int TB, int STORE, int NDOT, typename T>
__global__ __launch_bounds__(256, 2) void k_tile16(
    int n, int n_items, const int* __restrict__ items, const int* __restrict__ ka_ptr,
    const int* __restrict__ ka_col, const int* __restrict__ ka_pos,
    const int* __restrict__ ka_key, const int* __restrict__ a_rp, const T* __restrict__ a_val,
    int a_nnzb, Ix bx, const T* __restrict__ b_val, int b_nnzb,
    const int* __restrict__ jc_ptr, const int* __restrict__ jc_col,
    const int* __restrict__ jc_pos, T* __restrict__ c_val, double alpha, double beta,
    const T* __restrict__ m1, const T* __restrict__ m2, double* __restrict__ partials,
    const double* __restrict__ skip) {
  using AccT = typename TileAcc<MODE>::type;
  if (skip != nullptr && *skip != 0.0) return;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int item = xcd_remap(blockIdx.x, gridDim.x) * 4 + wave;
  if (item >= n_items) return;
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lq = lane >> 4;
  const int c = items[2 * item];
  const int p0 = items[2 * item + 1];
  const int ncol = min(4 * NB, jc_ptr[c + 1] - p0);
  const int r0 = c * 16;
  // output tiles present (bit 4q + ar): sub-row 0 / sub-column 0 of the tile
  // is present whenever any of its blocks is (tile4 outputs)
  int here = 0;
  if (lane < 4 * NB) {
    const int ar = lane & 3, q = lane >> 2;
    here = 4 * q < ncol && jc_pos[(size_t)(p0 + 4 * q) * 16 + 4 * ar] >= 0;
  }
  const uint64_t cmask = __ballot(here);
  // the piece's column atoms: unit in B's index, cell (-1 past the piece's
  // end), slot; TB: row lengths in B' of those atoms
  int jb[NB], jcell[NB], jslot[NB], lenBq[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const bool ok = 4 * q < ncol;
    const int jr = jc_col[p0 + (ok ? 4 * q : 0)];
    jb[q] = jr >> 2;
    jcell[q] = ok ? bx.cell[jb[q]] : -1;
    jslot[q] = bx.slot[jb[q]];
    lenBq[q] = TB ? bx.rp[jr + 1] - bx.rp[jr] : 0;   // TB = 2: B's own rows (B = B')
  }
  int rowA[4];
#pragma unroll
  for (int ar = 0; ar < 4; ++ar) {
    const int r = r0 + 4 * ar;
    const int len = r < n ? a_rp[r + 1] - a_rp[r] : 0;
    rowA[ar] = (li >> 2) * len;  // this lane's sub-row of the tile
  }
  const int t0 = ka_ptr[c], t1 = ka_ptr[c + 1];
  const int nsteps = (t1 - t0) >> 2;  // atoms of the contraction union
  const int amax = a_nnzb - 1, bmax = b_nnzb - 1;

  AccT acc[4][NB];
#pragma unroll
  for (int ar = 0; ar < 4; ++ar)
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[ar][q][v] = 0;

  // this lane's step of the current chunk (positions as in TileStep) and the
  // chunk's kept steps not yet taken
  int cpa[4], cpb[NB], clen = 0, cact = 0, ctr = 0;
  uint64_t rem = 0;
  int base = -64;
  auto scan = [&]() {
    const int s = min(base + lane, nsteps - 1);
    const int t = t0 + 4 * s;
    const int kk = ka_col[t];  // B's row 4k of the step's atom k
    const int ck = ka_key[2 * (size_t)t], sk = ka_key[2 * (size_t)t + 1];
#pragma unroll
    for (int ar = 0; ar < 4; ++ar) cpa[ar] = ka_pos[(size_t)t * 16 + 4 * ar];
    clen = TB == 1 ? 0 : bx.rp[kk + 1] - bx.rp[kk];
    int act = 0, tr = 0;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      // tile (k, j_q) of B, TB = 1: tile (j_q, k) of B'; TB = 2: the stored
      // one of the pair (the half's); the index's trailing -1 outside the
      // window
      const bool tq = TB == 1 || (TB == 2 && !in_half(n, kk, 4 * jb[q]));
      tr |= (int)tq << q;
      const int o = jcell[q] < 0 ? -1
                    : tq         ? ix_off(bx, jcell[q], ck, sk)
                                 : ix_off(bx, ck, jcell[q], jslot[q]);
      const int* src = o < 0 ? bx.tab + bx.sent
                             : bx.tab + (size_t)(tq ? jb[q] : kk >> 2) * bx.stride + o;
      cpb[q] = *src;
#pragma unroll
      for (int ar = 0; ar < 4; ++ar)
        if (cpa[ar] >= 0 && cpb[q] >= 0 && ((cmask >> (4 * q + ar)) & 1u))
          act |= 1 << (4 * q + ar);
    }
    cact = act;
    ctr = tr;
    rem = __ballot(base + lane < nsteps && act != 0);
  };
  // the next kept step (false past the list's end: e then names no tile,
  // its loads stay in bounds and nothing is multiplied)
  auto next = [&](TileStep<NB>& e) -> bool {
    while (rem == 0) {
      base += 64;
      if (base >= nsteps) {
#pragma unroll
        for (int ar = 0; ar < 4; ++ar) e.pa[ar] = -1;
#pragma unroll
        for (int q = 0; q < NB; ++q) e.pb[q] = -1;
        e.lenB = 0;
        e.act = 0;
        e.tmask = 0;
        return false;
      }
      scan();
    }
    const int m = __builtin_ctzll(rem);
    rem &= rem - 1;
#pragma unroll
    for (int ar = 0; ar < 4; ++ar) e.pa[ar] = __builtin_amdgcn_readlane(cpa[ar], m);
#pragma unroll
    for (int q = 0; q < NB; ++q) e.pb[q] = __builtin_amdgcn_readlane(cpb[q], m);
    e.lenB = __builtin_amdgcn_readlane(clen, m);
    e.act = __builtin_amdgcn_readlane(cact, m);
    e.tmask = TB == 2 ? __builtin_amdgcn_readlane(ctr, m) : 0;
    return true;
  };

  if (nsteps > 0 && (MODE == TM_F64 || (MODE == TM_F16X3 && NB == 4))) {
    // the A fragments single-buffered (loaded after the products that read
    // them), the B fragments double-buffered: one more wave fits a SIMD --
    // FP64 4 x 2 tiles three instead of two, FP64 4 x 4 tiles (accumulators
    // in the architectural registers under the two-wave launch bound) two
    // instead of one, the FP16 split's 4 x 4 tiles three instead of two
    // (measured on the 32768-atom cell: 4%, 14% and 12% faster; where the
    // wave count does not change the exposed A loads cost 5-7%, so the
    // other shapes keep both double-buffered)
    T fa[4][4], fb0[NB][4], fb1[NB][4];
    TileStep<NB> e0, e1;
    if (next(e0)) {
      tile_load_a<T>(fa, e0.pa, a_val, rowA, li, lq, amax);
      tile_load_b<NB, TB, T>(fb0, e0.pb, e0.lenB, lenBq, b_val, li, lq, bmax, e0.tmask);
      // each A row of the next step is loaded as soon as the current step's
      // products are done with that row
      for (;;) {
        const bool h1 = next(e1);
        tile_load_b<NB, TB, T>(fb1, e1.pb, e1.lenB, lenBq, b_val, li, lq, bmax, e1.tmask);
        tile_mma<MODE, NB>(acc, fa, fb0, e0.act, [&](int ar) {
          tile_load_a_row<T>(fa[ar], e1.pa[ar], a_val, rowA[ar], li, lq, amax);
        });
        if (!h1) break;
        const bool h0 = next(e0);
        tile_load_b<NB, TB, T>(fb0, e0.pb, e0.lenB, lenBq, b_val, li, lq, bmax, e0.tmask);
        tile_mma<MODE, NB>(acc, fa, fb1, e1.act, [&](int ar) {
          tile_load_a_row<T>(fa[ar], e0.pa[ar], a_val, rowA[ar], li, lq, amax);
        });
        if (!h0) break;
      }
    }
  } else if (nsteps > 0) {
    T fa0[4][4], fb0[NB][4], fa1[4][4], fb1[NB][4];
    TileStep<NB> e0, e1;
    if (next(e0)) {
      tile_load<NB, TB, T>(fa0, fb0, e0.pa, e0.pb, e0.lenB, lenBq, a_val, b_val, rowA, li, lq,
                           amax, bmax, e0.tmask);
      // two kept steps per turn, fragments double-buffered; the loads of the
      // step after the one multiplied are issued first (unconditionally, so
      // the wait before each product covers the older loads only)
      for (;;) {
        const bool h1 = next(e1);
        tile_load<NB, TB, T>(fa1, fb1, e1.pa, e1.pb, e1.lenB, lenBq, a_val, b_val, rowA, li,
                             lq, amax, bmax, e1.tmask);
        tile_mma<MODE, NB>(acc, fa0, fb0, e0.act);
        if (!h1) break;
        const bool h0 = next(e0);
        tile_load<NB, TB, T>(fa0, fb0, e0.pa, e0.pb, e0.lenB, lenBq, a_val, b_val, rowA, li,
                             lq, amax, bmax, e0.tmask);
        tile_mma<MODE, NB>(acc, fa1, fb1, e1.act);
        if (!h0) break;
      }
    }
  }

  // epilogue: lane (n + 16g) holds column n of each tile (column n&3 of
  // block n>>2), in register v the tile row 4g + v (FP32 accumulators) or
  // 4v + g (v_mfma_f64_16x16x4_f64), i.e. sub-row (row >> 2), row (row & 3)
  // of that 4x4 block.  The output positions are loaded first, all at once
  // (unconditionally, a missing tile reading the piece's first entry), so
  // their latency is paid once per wave instead of once per element.
  const double sc = MODE == TM_F16X3 ? kF16Unscale : 1.0;
  const int g = lq, nn = li;
  // FP64: the four sub-rows v of the lane's rows (4 consecutive entries);
  // FP32 accumulators: sub-row g for every v
  int opos[4][NB][MODE == TM_F64 ? 4 : 1];
#pragma unroll
  for (int ar = 0; ar < 4; ++ar)
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = p0 + 4 * q + (nn >> 2);
      const bool ok = ((cmask >> (4 * q + ar)) & 1u) && e < p0 + ncol;
      const int* src = jc_pos + (size_t)(ok ? e : p0) * 16 + 4 * ar;
      if constexpr (MODE == TM_F64) {
        const int4 v4 = *reinterpret_cast<const int4*>(src);
        opos[ar][q][0] = ok ? v4.x : -1;
        opos[ar][q][1] = ok ? v4.y : -1;
        opos[ar][q][2] = ok ? v4.z : -1;
        opos[ar][q][3] = ok ? v4.w : -1;
      } else {
        const int pp = src[g];
        opos[ar][q][0] = ok ? pp : -1;
      }
    }
  double d1 = 0.0, d2 = 0.0;
#pragma unroll
  for (int ar = 0; ar < 4; ++ar)
#pragma unroll
    for (int q = 0; q < NB; ++q) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = MODE == TM_F64 ? 4 * v + g : 4 * g + v;
        const int pos = opos[ar][q][MODE == TM_F64 ? v : 0];
        if (pos < 0) continue;
        const size_t at = (size_t)pos * 16 + (row & 3) * 4 + (nn & 3);
        const double val = alpha * (sc * (double)acc[ar][q][v]);
        const T out = (T)(beta != 0.0 ? val + beta * (double)c_val[at] : val);
        if (STORE) c_val[at] = out;
        if (NDOT >= 1) d1 = fma((double)m1[at], (double)out, d1);
        if (NDOT >= 2) d2 = fma((double)m2[at], (double)out, d2);
      }
    }
  if (NDOT >= 1) {
    d1 = wave_sum(d1);
    if (NDOT >= 2) d2 = wave_sum(d2);
    if (lane == 0) {
      partials[2 * item] = d1;
      partials[2 * item + 1] = d2;
    }
  }
}

template <typename T>
using KernelT16Fn = void (*)(int, int, const int*, const int*, const int*, const int*,
                             const int*, const int*, const T*, int, Ix, const T*, int,
                             const int*, const int*, const int*, T*, double, double, const T*,
                             const T*, double*, const double*);

template <int NB, int MODE, int TB, typename T>
KernelT16Fn<T> pick_t16(int store, int ndot) {
  if (store) {
    if (ndot == 0) return k_tile16<NB, MODE, TB, 1, 0, T>;
    if (ndot == 1) return k_tile16<NB, MODE, TB, 1, 1, T>;
    return k_tile16<NB, MODE, TB, 1, 2, T>;
  }
  if (ndot == 1) return k_tile16<NB, MODE, TB, 0, 1, T>;
  return k_tile16<NB, MODE, TB, 0, 2, T>;
}

template <int NB, int MODE, typename T>
KernelT16Fn<T> pick_t16_tb(int transB, int store, int ndot) {
  if (transB == 2)   // B symmetric, stored as its half: stored products only
    return store && ndot == 0 ? k_tile16<NB, MODE, 2, 1, 0, T> : nullptr;
  return transB ? pick_t16<NB, MODE, 1, T>(store, ndot) : pick_t16<NB, MODE, 0, T>(store, ndot);
}

template <typename T>
using KernelC1Fn = void (*)(int, int, const int*, const int*, const int*, const int*,
                            const int*, const T*, Ix, const T*, const int*, const int*,
                            const int*, T*, double, double, const T*, const T*, double*,
                            const double*, const T*, Ix, const T*, T*, const T*, const T*,
                            double*);

template <int PAIR, typename T, typename Acc>
KernelC1Fn<T> pick_c1(int store, int ndot) {
  if (store) {
    if (ndot == 0) return k_mul44c1<PAIR, 1, 0, T, Acc>;
    if (ndot == 1) return k_mul44c1<PAIR, 1, 1, T, Acc>;
    return k_mul44c1<PAIR, 1, 2, T, Acc>;
  }
  if (ndot == 1) return k_mul44c1<PAIR, 0, 1, T, Acc>;
  return k_mul44c1<PAIR, 0, 2, T, Acc>;
}

template <typename T>
using KernelFn = void (*)(int, int, const int*, const int*, const int*, const T*, Ix, const T*,
                          const int*, const int*, T*, double, double, const T*, const T*,
                          double*, const double*);

// FP32 A and B, FP64 C: FP64 multiply-add (exact FP32 products, FP64 sums).
using KernelMixFn = void (*)(int, int, const int*, const int*, const int*, const float*, Ix,
                             const float*, const int*, const int*, double*, double, double,
                             const double*, const double*, double*, const double*);

template <int TB>
KernelMixFn pick_mix(int store, int ndot) {
  if (store) {
    if (ndot == 0) return k_mul44<TB, 1, 0, float, double, double>;
    if (ndot == 1) return k_mul44<TB, 1, 1, float, double, double>;
    return k_mul44<TB, 1, 2, float, double, double>;
  }
  if (ndot == 1) return k_mul44<TB, 0, 1, float, double, double>;
  return k_mul44<TB, 0, 2, float, double, double>;
}

template <int TB, typename T, typename Acc>
KernelFn<T> pick_store(int store, int ndot) {
  if (store) {
    if (ndot == 0) return k_mul44<TB, 1, 0, T, Acc>;
    if (ndot == 1) return k_mul44<TB, 1, 1, T, Acc>;
    return k_mul44<TB, 1, 2, T, Acc>;
  }
  if (ndot == 1) return k_mul44<TB, 0, 1, T, Acc>;
  return k_mul44<TB, 0, 2, T, Acc>;
}

// ------------------------------------------------------------------ timing
struct Timer {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  size_t used = 0;
};
Timer g_timer;

}  // namespace

bool timing_on() { return g_timer.on; }

namespace {

int timer_begin(hipStream_t s, hipEvent_t* stop) {
  if (!g_timer.on) return LNV_OK;
  if (g_timer.used == g_timer.ev.size()) {
    hipEvent_t a, b;
    LNV_HIP(hipEventCreate(&a));
    LNV_HIP(hipEventCreate(&b));
    g_timer.ev.emplace_back(a, b);
  }
  auto& pr = g_timer.ev[g_timer.used++];
  LNV_HIP(hipEventRecord(pr.first, s));
  *stop = pr.second;
  return LNV_OK;
}

int g_f32_acc = LNV_ACC_F32;  // accumulation of the FP32 products

bool plan_ok(const lnv_pattern* p) {
  return p->cl_ptr && p->cl_col && p->cl_pos && p->cl_cell;
}

}  // namespace

// The pipelined 4-row kernel: 4-row cluster plans on A and C (one lane per
// output column), B indexed by rows (4x4-blocked atoms, or rows of atoms
// split over several rows).
bool use_clustered(const lnv_bsm* A, const lnv_bsm* B, int transB, const lnv_bsm* C) {
  const lnv_pattern *pa = A->pat, *pb = B->pat, *pc = C->pat;
  return !transB && pa->cl_m == 4 && pc->cl_m == 4 && pc->cl_g == 1 && plan_ok(pa) &&
         plan_ok(pc) && pc->cl_items && has_ix(pb) && pb->ix.qs == 0 && pb->nnzb > 0;
}

// Atom-tile (MFMA) multiply: 16-row cluster plans on A and C, tile4 patterns
// on A, B and C (see k_tile16), B's index over atoms, row count a multiple
// of 4; op(B) = B^T reads B's tiles transposed.
bool use_tiles(const lnv_bsm* A, const lnv_bsm* B, int transB, const lnv_bsm* C) {
  const lnv_pattern *pa = A->pat, *pb = B->pat, *pc = C->pat;
  (void)transB;
  return pa->cl_m == 16 && pc->cl_m == 16 && (pc->cl_g == 4 || pc->cl_g == 8) &&
         pa->tile4 == 1 && pb->tile4 == 1 && pc->tile4 == 1 && has_ix(pb) && pb->ix.qs == 2 &&
         pa->n % 4 == 0 && plan_ok(pa) && plan_ok(pc) && pc->cl_items && pa->row_ptr &&
         pb->row_ptr && pa->nnzb > 0 && pb->nnzb > 0 && pa->nnzb < INT32_MAX &&
         pb->nnzb < INT32_MAX;
}

bool half_b_ok(const lnv_bsm* A, const lnv_bsm* B, const lnv_bsm* C) {
  return bsm_ok_any(A) && bsm_ok_any(B) && bsm_ok_any(C) && A->dtype == C->dtype &&
         B->dtype == C->dtype && A->blk == 4 && B->blk == 4 && C->blk == 4 &&
         A->pat->n == B->pat->n && A->pat->n == C->pat->n && use_tiles(A, B, 2, C);
}

int multiply_nparts(const lnv_bsm* A, const lnv_bsm* B, int transB, const lnv_bsm* C) {
  if (A->dtype != C->dtype) return C->pat->n_items;  // FP32 into FP64: row kernel
  return use_clustered(A, B, transB, C) || use_tiles(A, B, transB, C) ? C->pat->n_cl_items
                                                                      : C->pat->n_items;
}

namespace {

// Arithmetic of the atom-tile multiply for storage type T: FP64 storage runs
// FP64 MFMA; FP32 storage follows the process-wide accumulation mode.
template <typename T>
int tile_mode() {
  if (std::is_same<T, double>::value || g_f32_acc == LNV_ACC_F64) return TM_F64;
  return g_f32_acc == LNV_ACC_F16X3 ? TM_F16X3 : TM_F32;
}

template <typename T>
int launch_tiles(double alpha, const lnv_bsm* A, const lnv_bsm* B, int transB, double beta,
                 const lnv_bsm* C, int store, const T* m1, const T* m2, double* partials,
                 const double* skip, int ndot, hipStream_t s) {
  const lnv_pattern *pa = A->pat, *pb = B->pat, *pc = C->pat;
  if (pc->n_cl_items == 0) return LNV_OK;
  const int wgs = round_up((pc->n_cl_items + 3) / 4, kNumXcd);
  const bool nb4 = pc->cl_g == 4;  // 4 column atoms per wave (cl_g 8: 2)
  KernelT16Fn<T> fn = nullptr;
  const int mode = tile_mode<T>();
  const int tb = transB;
  if (mode == TM_F64) {
    fn = nb4 ? pick_t16_tb<4, TM_F64, T>(tb, store, ndot)
             : pick_t16_tb<2, TM_F64, T>(tb, store, ndot);
  } else {
    if constexpr (std::is_same<T, float>::value) {
      if (mode == TM_F16X3)
        fn = nb4 ? pick_t16_tb<4, TM_F16X3, T>(tb, store, ndot)
                 : pick_t16_tb<2, TM_F16X3, T>(tb, store, ndot);
      else
        fn = nb4 ? pick_t16_tb<4, TM_F32, T>(tb, store, ndot)
                 : pick_t16_tb<2, TM_F32, T>(tb, store, ndot);
    }
  }
  if (!fn) return LNV_EUNSUPPORTED;
  hipEvent_t stop = nullptr;
  LNV_TRY(timer_begin(s, &stop));
  fn<<<wgs, 256, 0, s>>>(pa->n, pc->n_cl_items, pc->cl_items, pa->cl_ptr, pa->cl_col,
                         pa->cl_pos, pa->cl_cell, pa->row_ptr, static_cast<const T*>(A->val),
                         (int)pa->nnzb, make_ix(pb), static_cast<const T*>(B->val),
                         (int)pb->nnzb, pc->cl_ptr, pc->cl_col, pc->cl_pos,
                         static_cast<T*>(C->val), alpha, beta, m1, m2, partials, skip);
  LNV_LAUNCH_CHECK();
  if (stop) LNV_HIP(hipEventRecord(stop, s));
  return LNV_OK;
}

template <typename T, typename Acc>
int launch_typed(double alpha, const lnv_bsm* A, const lnv_bsm* B, int transB, double beta,
                 const lnv_bsm* C, int store, const void* m1v, const void* m2v,
                 double* partials, const double* skip, int ndot, hipStream_t s) {
  const lnv_pattern *pa = A->pat, *pb = B->pat, *pc = C->pat;
  const T* av = static_cast<const T*>(A->val);
  const T* bv = static_cast<const T*>(B->val);
  T* cv = static_cast<T*>(C->val);
  const T* m1 = static_cast<const T*>(m1v);
  const T* m2 = static_cast<const T*>(m2v);
  if (use_tiles(A, B, transB, C))
    return launch_tiles<T>(alpha, A, B, transB, beta, C, store, m1, m2, partials, skip, ndot, s);
  if (use_clustered(A, B, transB, C)) {
    if (pc->n_cl_items == 0) return LNV_OK;
    const int wgs = round_up((pc->n_cl_items + 3) / 4, kNumXcd);
    hipEvent_t stop = nullptr;
    LNV_TRY(timer_begin(s, &stop));
    KernelC1Fn<T> fn = pick_c1<0, T, Acc>(store, ndot);
    fn<<<wgs, 256, 0, s>>>(pa->n, pc->n_cl_items, pc->cl_items, pa->cl_ptr, pa->cl_col,
                           pa->cl_pos, pa->cl_cell, av, make_ix(pb), bv, pc->cl_ptr, pc->cl_col,
                           pc->cl_pos, cv, alpha, beta, m1, m2, partials, skip, nullptr,
                           make_ix(pb), nullptr, nullptr, nullptr, nullptr, nullptr);
    LNV_LAUNCH_CHECK();
    if (stop) LNV_HIP(hipEventRecord(stop, s));
    return LNV_OK;
  }
  if (pc->n_items == 0) return LNV_OK;
  const int wgs = round_up((pc->n_items + 3) / 4, kNumXcd);
  hipEvent_t stop = nullptr;
  LNV_TRY(timer_begin(s, &stop));
  KernelFn<T> fn =
      transB ? pick_store<1, T, Acc>(store, ndot) : pick_store<0, T, Acc>(store, ndot);
  fn<<<wgs, 256, 0, s>>>(pa->n, pc->n_items, pc->items, pa->row_ptr, pa->col, av, make_ix(pb),
                         bv, pc->row_ptr, pc->col, cv, alpha, beta, m1, m2, partials, skip);
  LNV_LAUNCH_CHECK();
  if (stop) LNV_HIP(hipEventRecord(stop, s));
  return LNV_OK;
}

// Two products C1 = A1.B1, C2 = A2.B2 in one launch of the pipelined kernel
// (A1, A2 on one pattern, C1, C2 on one pattern with a 4-row cluster plan):
// the pieces of both fill the device together (grid y = product).
template <typename T, typename Acc>
int launch_pair_typed(const lnv_bsm* A1, const lnv_bsm* B1, const lnv_bsm* C1,
                      const lnv_bsm* A2, const lnv_bsm* B2, const lnv_bsm* C2, int store,
                      const void* m11, const void* m12, double* part1, const void* m21,
                      const void* m22, double* part2, const double* skip, int ndot,
                      hipStream_t s) {
  const lnv_pattern *pa = A1->pat, *pc = C1->pat;
  if (pc->n_cl_items == 0) return LNV_OK;
  const int wgs = round_up((pc->n_cl_items + 3) / 4, kNumXcd);
  hipEvent_t stop = nullptr;
  LNV_TRY(timer_begin(s, &stop));
  KernelC1Fn<T> fn = pick_c1<1, T, Acc>(store, ndot);
  fn<<<dim3(wgs, 2), 256, 0, s>>>(
      pa->n, pc->n_cl_items, pc->cl_items, pa->cl_ptr, pa->cl_col, pa->cl_pos, pa->cl_cell,
      static_cast<const T*>(A1->val), make_ix(B1->pat), static_cast<const T*>(B1->val),
      pc->cl_ptr, pc->cl_col, pc->cl_pos, static_cast<T*>(C1->val), 1.0, 0.0,
      static_cast<const T*>(m11), static_cast<const T*>(m12), part1, skip,
      static_cast<const T*>(A2->val), make_ix(B2->pat), static_cast<const T*>(B2->val),
      static_cast<T*>(C2->val), static_cast<const T*>(m21), static_cast<const T*>(m22), part2);
  LNV_LAUNCH_CHECK();
  if (stop) LNV_HIP(hipEventRecord(stop, s));
  return LNV_OK;
}

}  // namespace

int multiply_pair_launch(const lnv_bsm* A1, const lnv_bsm* B1, const lnv_bsm* C1,
                         const lnv_bsm* A2, const lnv_bsm* B2, const lnv_bsm* C2, int store,
                         const void* m11, const void* m12, double* part1, const void* m21,
                         const void* m22, double* part2, const double* skip, hipStream_t s) {
  const int ndot = m12 ? 2 : (m11 ? 1 : 0);
  const bool pairable =
      bsm_ok_any(A1) && bsm_ok_any(B1) && bsm_ok_any(C1) && bsm_ok_any(A2) && bsm_ok_any(B2) &&
      bsm_ok_any(C2) && A1->pat == A2->pat && C1->pat == C2->pat && A1->dtype == C1->dtype &&
      B1->dtype == C1->dtype && A2->dtype == C1->dtype && B2->dtype == C1->dtype &&
      C2->dtype == C1->dtype && A1->blk == 4 && B1->blk == 4 && C1->blk == 4 && B2->blk == 4 &&
      use_clustered(A1, B1, 0, C1) && use_clustered(A2, B2, 0, C2) &&
      B1->pat->n == C1->pat->n && B2->pat->n == C1->pat->n &&
      ndot == (m22 ? 2 : (m21 ? 1 : 0)) && (ndot == 0 || (part1 && part2)) && (store || ndot > 0);
  if (!pairable) {  // two launches
    LNV_TRY(multiply_launch(1.0, A1, B1, 0, 0.0, C1, store, m11, m12, part1, skip, s));
    return multiply_launch(1.0, A2, B2, 0, 0.0, C2, store, m21, m22, part2, skip, s);
  }
  if (C1->dtype == LNV_F32) {
    if (g_f32_acc == LNV_ACC_F64)
      return launch_pair_typed<float, double>(A1, B1, C1, A2, B2, C2, store, m11, m12, part1,
                                              m21, m22, part2, skip, ndot, s);
    return launch_pair_typed<float, float>(A1, B1, C1, A2, B2, C2, store, m11, m12, part1, m21,
                                           m22, part2, skip, ndot, s);
  }
  return launch_pair_typed<double, double>(A1, B1, C1, A2, B2, C2, store, m11, m12, part1, m21,
                                           m22, part2, skip, ndot, s);
}

namespace {

// FP32 A and B into an FP64 C (row kernel).
int launch_mix(double alpha, const lnv_bsm* A, const lnv_bsm* B, int transB, double beta,
               const lnv_bsm* C, int store, const void* m1, const void* m2, double* partials,
               const double* skip, int ndot, hipStream_t s) {
  const lnv_pattern *pa = A->pat, *pb = B->pat, *pc = C->pat;
  if (pc->n_items == 0) return LNV_OK;
  const int wgs = round_up((pc->n_items + 3) / 4, kNumXcd);
  hipEvent_t stop = nullptr;
  LNV_TRY(timer_begin(s, &stop));
  KernelMixFn fn = transB ? pick_mix<1>(store, ndot) : pick_mix<0>(store, ndot);
  fn<<<wgs, 256, 0, s>>>(pa->n, pc->n_items, pc->items, pa->row_ptr, pa->col,
                         static_cast<const float*>(A->val), make_ix(pb),
                         static_cast<const float*>(B->val), pc->row_ptr, pc->col,
                         static_cast<double*>(C->val), alpha, beta,
                         static_cast<const double*>(m1), static_cast<const double*>(m2),
                         partials, skip);
  LNV_LAUNCH_CHECK();
  if (stop) LNV_HIP(hipEventRecord(stop, s));
  return LNV_OK;
}

}  // namespace

int multiply_launch(double alpha, const lnv_bsm* A, const lnv_bsm* B, int transB,
                    double beta, const lnv_bsm* C, int store, const void* m1,
                    const void* m2, double* partials, const double* skip,
                    hipStream_t s) {
  if (!bsm_ok_any(A) || !bsm_ok_any(B) || !bsm_ok_any(C)) return LNV_EINVAL;
  const bool mix = A->dtype == LNV_F32 && B->dtype == LNV_F32 && C->dtype == LNV_F64;
  if (!mix && (A->dtype != C->dtype || B->dtype != C->dtype)) return LNV_EUNSUPPORTED;
  if (A->blk != 4 || B->blk != 4 || C->blk != 4) return LNV_EUNSUPPORTED;
  const lnv_pattern *pa = A->pat, *pb = B->pat, *pc = C->pat;
  if (pa->n != pb->n || pa->n != pc->n) return LNV_EPATTERN;
  if (!pa->row_ptr || !pa->col || !pc->row_ptr || !pc->col || !pc->items) return LNV_EPATTERN;
  if (!has_ix(pb)) return LNV_EPATTERN;
  const int ndot = m2 ? 2 : (m1 ? 1 : 0);
  if (m2 && !m1) return LNV_EINVAL;
  if (ndot > 0 && !partials) return LNV_EINVAL;
  if (!store && ndot == 0) return LNV_EINVAL;
  if (transB < 0 || transB > 2) return LNV_EINVAL;
  // B symmetric and stored as its half: atom tiles only (a tile4 half keeps
  // or drops whole atom tiles), stored products without dots
  if (transB == 2 && (mix || !use_tiles(A, B, transB, C) || ndot > 0)) return LNV_EUNSUPPORTED;
  if (mix) return launch_mix(alpha, A, B, transB, beta, C, store, m1, m2, partials, skip, ndot, s);
  if (C->dtype == LNV_F32) {
    if (g_f32_acc == LNV_ACC_F64)
      return launch_typed<float, double>(alpha, A, B, transB, beta, C, store, m1, m2, partials,
                                         skip, ndot, s);
    return launch_typed<float, float>(alpha, A, B, transB, beta, C, store, m1, m2, partials,
                                      skip, ndot, s);
  }
  return launch_typed<double, double>(alpha, A, B, transB, beta, C, store, m1, m2, partials,
                                      skip, ndot, s);
}

}  // namespace lnv

using namespace lnv;

extern "C" int lnv_bsm_multiply(double alpha, const lnv_bsm* A, const lnv_bsm* B,
                                int32_t transB, double beta, lnv_bsm* C, hipStream_t s) {
  return multiply_launch(alpha, A, B, transB, beta, C, 1, nullptr, nullptr, nullptr, nullptr,
                         s);
}

extern "C" int lnv_multiply_ws_bytes(const lnv_bsm* A, const lnv_bsm* B, int32_t transB,
                                     const lnv_bsm* C, int32_t with_dot, int64_t* bytes_out) {
  if (!bsm_ok_any(A) || !bsm_ok_any(B) || !bsm_ok_any(C) || !bytes_out) return LNV_EINVAL;
  *bytes_out = with_dot ? 2 * (int64_t)multiply_nparts(A, B, transB, C) * (int64_t)sizeof(double)
                        : 0;
  return LNV_OK;
}

extern "C" int lnv_set_f32_accumulation(int32_t acc) {
  if (acc != LNV_ACC_F32 && acc != LNV_ACC_F64 && acc != LNV_ACC_F16X3) return LNV_EINVAL;
  g_f32_acc = acc;
  return LNV_OK;
}

extern "C" int lnv_timing_enable(int32_t on) {
  g_timer.on = on != 0;
  return LNV_OK;
}

extern "C" int lnv_timing_reset(void) {
  g_timer.used = 0;
  return LNV_OK;
}

extern "C" int lnv_timing_read(double* ms_total, int64_t* launches) {
  if (!ms_total || !launches) return LNV_EINVAL;
  double tot = 0.0;
  for (size_t q = 0; q < g_timer.used; ++q) {
    auto& pr = g_timer.ev[q];
    LNV_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    LNV_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    tot += ms;
  }
  *ms_total = tot;
  *launches = (int64_t)g_timer.used;
  return LNV_OK;
}
