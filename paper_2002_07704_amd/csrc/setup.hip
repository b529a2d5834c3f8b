// Set-up kernels of the LNV hot path, run once per geometry:
//   a0  range patterns (neighbour lists)            Sec. II.C.2 range rule
//   a1  synthetic S and H blocks                    stand-in for Eq. (2)
//   a2  patterns of block-sparse products           Sec. II.C.2 sparse products
//   index tables and work lists of a pattern
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "internal.h"

namespace lnv {
namespace {

// ------------------------------------------------------------------ scans
// In-place exclusive scan of data[0..n) into data[0..n] (data[n] = total) by
// one workgroup of 1024 threads; each thread scans a contiguous chunk.
template <typename T>
__global__ __launch_bounds__(1024) void k_scan(T* __restrict__ data, int n) {
  __shared__ T part[1024];
  const int tid = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int b = min(n, tid * chunk), e = min(n, b + chunk);
  T s = 0;
  for (int q = b; q < e; ++q) s += data[q];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    T run = 0;
    for (int q = 0; q < 1024; ++q) {
      const T v = part[q];
      part[q] = run;
      run += v;
    }
    data[n] = run;
  }
  __syncthreads();
  T run = part[tid];
  for (int q = b; q < e; ++q) {
    const T v = data[q];
    data[q] = run;
    run += v;
  }
}

// ------------------------------------------------------------------ a0
// One wavefront per row i scans every j in ascending order (so the columns
// come out sorted) and compacts the in-range ones with a ballot.
// With cells (cell_of != null): row i belongs to cell c = cell_of[i], whose
// rows are cell_start[c] .. cell_start[c+1]-1 and whose periodic box is
// boxes[3c .. 3c+2]; only rows of the same cell are tested.
__global__ __launch_bounds__(256) void k_neighbours(const double* __restrict__ pos, int n,
                                                    double bx, double by, double bz,
                                                    const int* __restrict__ cell_of,
                                                    const int* __restrict__ cell_start,
                                                    const double* __restrict__ boxes,
                                                    double R2, int* __restrict__ counts,
                                                    const int* __restrict__ row_ptr,
                                                    int* __restrict__ col, int fill) {
#pragma clang fp contract(off)
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int lane = threadIdx.x & 63;
  int jlo = 0, jhi = n;
  if (cell_of) {
    const int c = cell_of[row];
    jlo = cell_start[c];
    jhi = cell_start[c + 1];
    bx = boxes[3 * c];
    by = boxes[3 * c + 1];
    bz = boxes[3 * c + 2];
  }
  const double xi = pos[3 * row], yi = pos[3 * row + 1], zi = pos[3 * row + 2];
  const int base = fill ? row_ptr[row] : 0;
  int cnt = 0;
  for (int j0 = jlo; j0 < jhi; j0 += kWave) {
    const int j = j0 + lane;
    bool ok = false;
    if (j < jhi) {
      double dx = pos[3 * j] - xi;
      double dy = pos[3 * j + 1] - yi;
      double dz = pos[3 * j + 2] - zi;
      dx = dx - bx * rint(dx / bx);
      dy = dy - by * rint(dy / by);
      dz = dz - bz * rint(dz / bz);
      double d2 = dx * dx + dy * dy;
      d2 = d2 + dz * dz;
      ok = d2 <= R2;
    }
    const uint64_t m = __ballot(ok);
    if (fill && ok) col[base + cnt + __popcll(m & ((1ull << lane) - 1ull))] = j;
    cnt += __popcll(m);
  }
  if (!fill && lane == 0) counts[row] = cnt;
}

// ------------------------------------------------------------------ a2
// One workgroup per output row: the union of B's rows k over A's row i is
// accumulated in an LDS bitmap of n bits (optionally intersected with the
// mask row), then counted or emitted in ascending order.
__global__ __launch_bounds__(256) void k_symbolic(
    int n, const int* __restrict__ a_rp, const int* __restrict__ a_col,
    const int* __restrict__ b_rp, const int* __restrict__ b_col,
    const int* __restrict__ m_rp, const int* __restrict__ m_col, int* __restrict__ counts,
    const int* __restrict__ out_rp, int* __restrict__ out_col,
    long long* __restrict__ triples, int fill, const int* __restrict__ wts) {
  extern __shared__ unsigned int sm[];
  __shared__ long long scan[256];
  const int W = (n + 31) >> 5;
  unsigned int* bits = sm;
  unsigned int* mbits = sm + W;
  const int i = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int w = tid; w < W; w += 256) {
    bits[w] = 0u;
    mbits[w] = 0u;
  }
  __syncthreads();
  if (m_rp)
    for (int q = m_rp[i] + tid; q < m_rp[i + 1]; q += 256) {
      const int j = m_col[q];
      atomicOr(&mbits[j >> 5], 1u << (j & 31));
    }
  const int t0 = a_rp[i], t1 = a_rp[i + 1];
  for (int t = t0 + wv; t < t1; t += 4) {
    const int k = a_col[t];
    for (int q = b_rp[k] + lane; q < b_rp[k + 1]; q += kWave) {
      const int j = b_col[q];
      atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
  }
  __syncthreads();
  if (m_rp)
    for (int w = tid; w < W; w += 256) bits[w] &= mbits[w];
  __syncthreads();
  const int chunk = (W + 255) / 256;
  const int w0 = min(W, tid * chunk), w1 = min(W, w0 + chunk);
  long long mine = 0;
  for (int w = w0; w < w1; ++w) mine += __popc(bits[w]);
  scan[tid] = mine;
  __syncthreads();
  if (tid == 0) {
    long long run = 0;
    for (int q = 0; q < 256; ++q) {
      const long long v = scan[q];
      scan[q] = run;
      run += v;
    }
    if (!fill) counts[i] = (int)run;
  }
  __syncthreads();
  if (fill) {
    int p = out_rp[i] + (int)scan[tid];
    for (int w = w0; w < w1; ++w) {
      unsigned int x = bits[w];
      while (x) {
        const int b = __ffs(x) - 1;
        out_col[p++] = (w << 5) + b;
        x &= x - 1u;
      }
    }
  } else if (triples) {
    // kept triples (i,k,j), each weighted by w_i w_k w_j when wts is given
    long long tr = 0;
    for (int t = t0 + wv; t < t1; t += 4) {
      const int k = a_col[t];
      const long long wk = wts ? wts[k] : 1;
      for (int q = b_rp[k] + lane; q < b_rp[k + 1]; q += kWave) {
        const int j = b_col[q];
        const long long hit = (bits[j >> 5] >> (j & 31)) & 1u;
        tr += hit * (wts ? wk * wts[j] : 1);
      }
    }
    __syncthreads();
    scan[tid] = tr;
    __syncthreads();
    if (tid == 0) {
      long long s = 0;
      for (int q = 0; q < 256; ++q) s += scan[q];
      triples[i] = wts ? s * wts[i] : s;
    }
  }
}

// Symmetric half of a pattern (in_half): one thread per row, columns kept in
// their ascending order.
__global__ __launch_bounds__(256) void k_half(int n, const int* __restrict__ rp,
                                              const int* __restrict__ col,
                                              int* __restrict__ counts,
                                              const int* __restrict__ out_rp,
                                              int* __restrict__ out_col) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (!out_col) {
    int c = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) c += in_half(n, i, col[p]) ? 1 : 0;
    counts[i] = c;
    return;
  }
  int q = out_rp[i];
  for (int p = rp[i]; p < rp[i + 1]; ++p)
    if (in_half(n, i, col[p])) out_col[q++] = col[p];
}

// ------------------------------------------------------------------ spatial index
// Largest wrapped cell offset, per axis, between a unit row and the units of
// its columns (only the first row of a unit and the first column of each
// unit count: the others repeat them).  ext[0..2] receive the maxima
// (atomicMax), ext[3] is set when a row unit's first row does not start a
// unit (a pattern qs cannot describe).
__global__ __launch_bounds__(256) void k_ix_extent(int n_units, int qs,
                                                   const int* __restrict__ rp,
                                                   const int* __restrict__ col,
                                                   const int* __restrict__ cell, int g0, int g1,
                                                   int g2, int* __restrict__ ext) {
  const int a = blockIdx.x;
  const int i = a << qs;
  const int m = (1 << qs) - 1;
  const int ca = cell[a];
  int e0 = 0, e1 = 0, e2 = 0;
  for (int p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 256) {
    const int j = col[p];
    if (j & m) continue;
    const int cb = cell[j >> qs];
    int o[3] = {(cb & 1023) - (ca & 1023), ((cb >> 10) & 1023) - ((ca >> 10) & 1023),
                (cb >> 20) - (ca >> 20)};
    const int g[3] = {g0, g1, g2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int v = o[d];
      if (v < 0) v += g[d];
      v = min(v, g[d] - v);   // wrapped distance along the axis
      o[d] = v;
    }
    e0 = max(e0, o[0]);
    e1 = max(e1, o[1]);
    e2 = max(e2, o[2]);
  }
  if (e0) atomicMax(ext + 0, e0);
  if (e1) atomicMax(ext + 1, e1);
  if (e2) atomicMax(ext + 2, e2);
}

// tab[a * stride + window offset of unit b] = position of block (a<<qs, b<<qs).
__global__ __launch_bounds__(256) void k_ix_fill(int n_units, Ix x, const int* __restrict__ col,
                                                 int* __restrict__ tab, int* __restrict__ bad) {
  const int a = blockIdx.x;
  const int i = a << x.qs;
  const int m = (1 << x.qs) - 1;
  const int ca = x.cell[a];
  for (int p = x.rp[i] + threadIdx.x; p < x.rp[i + 1]; p += 256) {
    const int j = col[p];
    if (j & m) continue;
    const int b = j >> x.qs;
    const int o = ix_off(x, ca, x.cell[b], x.slot[b]);
    if (o < 0) {
      atomicOr(bad, 1);
      continue;
    }
    tab[(size_t)a * x.stride + o] = p;
  }
}

// perm[p] = position in PT of the transpose of block p of P; bad[0] set to
// 1 when a block has no transpose.
__global__ __launch_bounds__(256) void k_tmap(int n, const int* __restrict__ rp,
                                              const int* __restrict__ col, Ix xpt,
                                              int* __restrict__ perm, int* __restrict__ bad) {
  const int i = blockIdx.x;
  for (int p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 256) {
    const int q = ix_find(xpt, col[p], i);
    perm[p] = q;
    if (q < 0) bad[0] = 1;
  }
}

// Cluster unions: one workgroup per cluster of m rows; the union of their
// columns is collected in an LDS bitmap, then counted or emitted in
// ascending order together with each row's block position (from the
// pattern's index) or -1, and the packed cell and the slot of the column's
// unit.
__global__ __launch_bounds__(256) void k_cluster_union(int n, int m, const int* __restrict__ rp,
                                                       const int* __restrict__ col, Ix px,
                                                       int* __restrict__ counts,
                                                       const int* __restrict__ out_ptr,
                                                       int* __restrict__ out_col,
                                                       int* __restrict__ out_pos,
                                                       int* __restrict__ out_cell, int fill) {
  extern __shared__ unsigned int bits[];
  __shared__ int scan[256];
  const int W = (n + 31) >> 5;
  const int c = blockIdx.x;
  const int tid = threadIdx.x;
  for (int w = tid; w < W; w += 256) bits[w] = 0u;
  __syncthreads();
  for (int r = 0; r < m; ++r) {
    const int i = c * m + r;
    if (i >= n) break;
    for (int q = rp[i] + tid; q < rp[i + 1]; q += 256) {
      const int j = col[q];
      atomicOr(&bits[j >> 5], 1u << (j & 31));
    }
  }
  __syncthreads();
  const int chunk = (W + 255) / 256;
  const int w0 = min(W, tid * chunk), w1 = min(W, w0 + chunk);
  int mine = 0;
  for (int w = w0; w < w1; ++w) mine += __popc(bits[w]);
  scan[tid] = mine;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int q = 0; q < 256; ++q) {
      const int v = scan[q];
      scan[q] = run;
      run += v;
    }
    if (!fill) counts[c] = run;
  }
  __syncthreads();
  if (!fill) return;
  int t = out_ptr[c] + scan[tid];
  for (int w = w0; w < w1; ++w) {
    unsigned int x = bits[w];
    while (x) {
      const int b = __ffs(x) - 1;
      const int j = (w << 5) + b;
      out_col[t] = j;
      out_cell[2 * (size_t)t] = px.cell[j >> px.qs];
      out_cell[2 * (size_t)t + 1] = px.slot[j >> px.qs];
      for (int r = 0; r < m; ++r) {
        const int i = c * m + r;
        out_pos[(size_t)t * m + r] = i < n ? ix_find(px, i, j) : -1;
      }
      ++t;
      x &= x - 1u;
    }
  }
}

// Work pieces of `piece` columns over the cluster unions.
__global__ __launch_bounds__(256) void k_cluster_items(int nc, int piece,
                                                       const int* __restrict__ cptr,
                                                       int* __restrict__ counts,
                                                       const int* __restrict__ off,
                                                       int* __restrict__ items) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= nc) return;
  const int len = cptr[c + 1] - cptr[c];
  const int k = (len + piece - 1) / piece;
  if (!items) {
    counts[c] = k;
    return;
  }
  const int o = off[c];
  for (int q = 0; q < k; ++q) {
    items[2 * (o + q)] = c;
    items[2 * (o + q) + 1] = cptr[c] + q * piece;
  }
}

// tile4 check, one workgroup per row r: same length and columns as row
// 4(r/4), columns in aligned runs 4b..4b+3.  Any violation sets *bad (a
// vector atomic; the flag only ever goes from 0 to 1).
__global__ __launch_bounds__(256) void k_tile4(int n, const int* __restrict__ rp,
                                               const int* __restrict__ col, int* __restrict__ bad) {
  const int r = blockIdx.x;
  const int r4 = r & ~3;
  const int p0 = rp[r], len = rp[r + 1] - p0;
  const int q0 = rp[r4], len4 = rp[r4 + 1] - q0;
  if (len != len4 || (len & 3) != 0) {
    if (threadIdx.x == 0) atomicOr(bad, 1);
    return;
  }
  for (int t = threadIdx.x; t < len; t += 256) {
    const int j = col[p0 + t];
    const bool ok = j == col[q0 + t] && (j & 3) == (t & 3) && j - (t & 3) == col[p0 + (t & ~3)];
    if (!ok) atomicOr(bad, 1);
  }
}

// Output-grade tile check, one workgroup per row r: every column c of row r
// has the whole run (c & ~3) .. (c & ~3) + 3 in row r & ~3 (the first row
// of r's group).  Any violation sets *bad.

__global__ __launch_bounds__(256) void k_items(int n, const int* __restrict__ rp,
                                               int* __restrict__ counts,
                                               const int* __restrict__ off,
                                               int* __restrict__ items) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int len = rp[i + 1] - rp[i];
  const int c = (len + kWave - 1) / kWave;
  if (!items) {
    counts[i] = c;
    return;
  }
  const int o = off[i];
  for (int q = 0; q < c; ++q) {
    items[2 * (o + q)] = i;
    items[2 * (o + q) + 1] = rp[i] + q * kWave;
  }
}

// ------------------------------------------------------------------ a1
// Counter-based SplitMix64: output number ctr of the stream seeded with seed
// (Steele, Lea & Flood 2014): mix(seed + (ctr + 1) * golden gamma).
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ double rand_entry(uint64_t seed, uint64_t stream, uint64_t a,
                                             uint64_t b, uint64_t e, double scale) {
  const uint64_t ctr = (stream << 56) | (a << 32) | (b << 8) | e;
  const double u = (double)(splitmix64_at(seed, ctr) >> 11) * 0x1.0p-53;
  return scale * (u - 0.5);
}

// Row i of the stored matrix is rows off_of[i] .. off_of[i]+blk-1 of atom
// atom_of[i]'s block (identity maps when atom_of is null): an atom with more
// support functions than blk spans several stored rows, and entries past the
// atom's function count are zero.  The random entries are keyed by the atom
// pair and the element's index in the atom block, so the values do not depend
// on how atoms are split into stored rows.
// Independent cells (cell_of != null): row i belongs to cell c = cell_of[i]
// with periodic box boxes[3c..3c+2] and master seed seeds[c]; atom_of then
// holds each row's atom index within its cell (the counter key) and fun_of
// its atom's function count.
__global__ __launch_bounds__(128) void k_synth(const double* __restrict__ pos, double bx,
                                               double by, double bz,
                                               const int* __restrict__ cell_of,
                                               const double* __restrict__ boxes,
                                               const uint64_t* __restrict__ seeds,
                                               const int* __restrict__ fun_of,
                                               const int* __restrict__ nfun,
                                               const int* __restrict__ atom_of,
                                               const int* __restrict__ off_of, int blk,
                                               const int* __restrict__ rp,
                                               const int* __restrict__ col,
                                               double* __restrict__ val, int kind, double R,
                                               double decay, uint64_t seed, double scale) {
#pragma clang fp contract(off)
  const int i = blockIdx.x;
  const uint64_t stream = kind == 0 ? 1ull : 2ull;
  if (cell_of) {
    const int c = cell_of[i];
    bx = boxes[3 * c];
    by = boxes[3 * c + 1];
    bz = boxes[3 * c + 2];
    seed = seeds[c];
  }
  const double R2 = R * R;
  const int mx = (int)ceil(R / bx) + 1, my = (int)ceil(R / by) + 1, mz = (int)ceil(R / bz) + 1;
  const int ai = atom_of ? atom_of[i] : i;
  const int oi = off_of ? off_of[i] : 0;
  const int ni = fun_of ? fun_of[i] : (nfun ? nfun[ai] : blk);
  for (int p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 128) {
    const int j = col[p];
    const int aj = atom_of ? atom_of[j] : j;
    const int oj = off_of ? off_of[j] : 0;
    const int nj = fun_of ? fun_of[j] : (nfun ? nfun[aj] : blk);
    const double dx = pos[3 * j] - pos[3 * i];
    const double dy = pos[3 * j + 1] - pos[3 * i + 1];
    const double dz = pos[3 * j + 2] - pos[3 * i + 2];
    double w = 0.0;
    for (int tx = -mx; tx <= mx; ++tx)
      for (int ty = -my; ty <= my; ++ty)
        for (int tz = -mz; tz <= mz; ++tz) {
          const double x = dx + (double)tx * bx;
          const double y = dy + (double)ty * by;
          const double z = dz + (double)tz * bz;
          double d2 = x * x + y * y;
          d2 = d2 + z * z;
          if (d2 <= R2) w = w + exp(-(sqrt(d2) / decay));
        }
    double* out = val + (size_t)p * blk * blk;
    for (int r = 0; r < blk; ++r)
      for (int c = 0; c < blk; ++c) {
        const int R = oi + r, C = oj + c;  // element of the atom block
        double v = 0.0;
        if (R < ni && C < nj) {
          double m;
          if (ai == aj) {
            const double a = rand_entry(seed, stream, ai, ai, R * ni + C, scale);
            const double b = rand_entry(seed, stream, ai, ai, C * ni + R, scale);
            m = (a + b) * 0.5;
          } else if (ai < aj) {
            m = rand_entry(seed, stream, ai, aj, R * nj + C, scale);
          } else {
            m = rand_entry(seed, stream, aj, ai, C * ni + R, scale);
          }
          const double wm = w * m;
          if (kind == 0)
            v = (ai == aj && R == C) ? wm + 2.0 : wm;
          else
            v = -wm;
        }
        out[r * blk + c] = v;
      }
  }
}

// Position derivative of a synthetic matrix contracted with a gradient on its
// pattern: for stored row i (atom a = atom_of[i]) and each block (i, j) of
// another atom b,
//   c = sum_rc (G_ij[r][c] - mu GN_ij[r][c] + G_ji[c][r] - mu GN_ji[c][r]) M_ab[R][C]
//   acc_i += sign * c * dw(a,b)/dx_a,  dw/dx_a = sum_T exp(-d_T/decay)/decay (x_b - x_a + T)/d_T
// (R, C: the entries' indices in the atom block, M from the generator's
// counters; G_ji through G's index table; sign -1 for the Hamiltonian,
// whose blocks are -w M).  acc (device [n][3]) accumulates: one workgroup per
// row, fixed order.  Diagonal atom blocks do not depend on the positions.
__global__ __launch_bounds__(128) void k_pos_grad(
    const double* __restrict__ pos, double bx, double by, double bz,
    const int* __restrict__ nfun, const int* __restrict__ atom_of, const int* __restrict__ off_of,
    int blk, int n, const int* __restrict__ rp, const int* __restrict__ col,
    Ix x, const double* __restrict__ G, const double* __restrict__ GN,
    double mu, int kind, double R, double decay, uint64_t seed, double scale,
    double* __restrict__ acc) {
#pragma clang fp contract(off)
  __shared__ double sh[16];
  const int i = blockIdx.x;
  const uint64_t stream = kind == 0 ? 1ull : 2ull;
  const double sign = kind == 0 ? 1.0 : -1.0;
  const double R2 = R * R;
  const int mx = (int)ceil(R / bx) + 1, my = (int)ceil(R / by) + 1, mz = (int)ceil(R / bz) + 1;
  const int ai = atom_of ? atom_of[i] : i;
  const int oi = off_of ? off_of[i] : 0;
  const int ni = nfun ? nfun[ai] : blk;
  double g[3] = {0.0, 0.0, 0.0};
  for (int p = rp[i] + threadIdx.x; p < rp[i + 1]; p += 128) {
    const int j = col[p];
    const int aj = atom_of ? atom_of[j] : j;
    if (aj == ai) continue;
    const int oj = off_of ? off_of[j] : 0;
    const int nj = nfun ? nfun[aj] : blk;
    const int q = ix_find(x, j, i);
    double c = 0.0;
    for (int r = 0; r < blk; ++r)
      for (int cc = 0; cc < blk; ++cc) {
        const int Rr = oi + r, Cc = oj + cc;
        if (Rr >= ni || Cc >= nj) continue;
        const double m = ai < aj ? rand_entry(seed, stream, ai, aj, Rr * nj + Cc, scale)
                                 : rand_entry(seed, stream, aj, ai, Cc * ni + Rr, scale);
        double gv = G[(size_t)p * blk * blk + r * blk + cc];
        if (GN) gv = gv - mu * GN[(size_t)p * blk * blk + r * blk + cc];
        if (q >= 0) {
          double gt = G[(size_t)q * blk * blk + cc * blk + r];
          if (GN) gt = gt - mu * GN[(size_t)q * blk * blk + cc * blk + r];
          gv = gv + gt;
        }
        c = c + gv * m;
      }
    const double dx = pos[3 * j] - pos[3 * i];
    const double dy = pos[3 * j + 1] - pos[3 * i + 1];
    const double dz = pos[3 * j + 2] - pos[3 * i + 2];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int tx = -mx; tx <= mx; ++tx)
      for (int ty = -my; ty <= my; ++ty)
        for (int tz = -mz; tz <= mz; ++tz) {
          const double x = dx + (double)tx * bx;
          const double y = dy + (double)ty * by;
          const double z = dz + (double)tz * bz;
          double d2 = x * x + y * y;
          d2 = d2 + z * z;
          if (d2 <= R2 && d2 > 0.0) {
            const double d = sqrt(d2);
            const double f = exp(-(d / decay)) / decay / d;
            gx = gx + f * x;
            gy = gy + f * y;
            gz = gz + f * z;
          }
        }
    g[0] = g[0] + sign * c * gx;
    g[1] = g[1] + sign * c * gy;
    g[2] = g[2] + sign * c * gz;
  }
  for (int k = 0; k < 3; ++k) {
    double v = g[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) acc[3 * i + k] = acc[3 * i + k] + (sh[0] + sh[1]);
  }
}

// F[seg_atom[s]] = -(sum of acc over rows seg_ptr[s] .. seg_ptr[s+1]-1).
__global__ __launch_bounds__(64) void k_seg_force(int n_seg, const int* __restrict__ seg_ptr,
                                                  const int* __restrict__ seg_atom,
                                                  const double* __restrict__ acc,
                                                  double* __restrict__ F) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= n_seg) return;
  double f[3] = {0.0, 0.0, 0.0};
  for (int r = seg_ptr[s]; r < seg_ptr[s + 1]; ++r)
    for (int k = 0; k < 3; ++k) f[k] += acc[3 * r + k];
  const int a = seg_atom[s];
  for (int k = 0; k < 3; ++k) F[3 * a + k] = -f[k];
}

int read_total_int(const int32_t* dev, int64_t* host, hipStream_t s) {
  int32_t t = 0;
  LNV_HIP(hipMemcpyAsync(&t, dev, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  LNV_HIP(hipStreamSynchronize(s));
  *host = t;
  return LNV_OK;
}

}  // namespace
}  // namespace lnv

using namespace lnv;

extern "C" int lnv_neighbours(const double* pos, int32_t n, const double* box, double R,
                              int32_t* row_ptr, int32_t* col, int64_t cap,
                              int64_t* nnz_out, hipStream_t s) {
  if (!pos || !box || !row_ptr || !nnz_out || n <= 0 || n > LNV_MAX_ATOMS || !(R >= 0.0))
    return LNV_EINVAL;
  if (!(box[0] > 0.0 && box[1] > 0.0 && box[2] > 0.0)) return LNV_EINVAL;
  const double R2 = R * R;
  const int grid = (n + 3) / 4;
  k_neighbours<<<grid, 256, 0, s>>>(pos, n, box[0], box[1], box[2], nullptr, nullptr, nullptr,
                                    R2, row_ptr, nullptr, nullptr, 0);
  LNV_LAUNCH_CHECK();
  k_scan<int32_t><<<1, 1024, 0, s>>>(row_ptr, n);
  LNV_LAUNCH_CHECK();
  LNV_TRY(read_total_int(row_ptr + n, nnz_out, s));
  if (!col) return LNV_OK;
  if (cap < *nnz_out) return LNV_ECAPACITY;
  k_neighbours<<<grid, 256, 0, s>>>(pos, n, box[0], box[1], box[2], nullptr, nullptr, nullptr,
                                    R2, nullptr, row_ptr, col, 1);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_neighbours_cells(const double* pos, int32_t n, int32_t n_cells,
                                    const int32_t* cell_start, const int32_t* cell_of,
                                    const double* boxes, double R, int32_t* row_ptr,
                                    int32_t* col, int64_t cap, int64_t* nnz_out,
                                    hipStream_t s) {
  if (!pos || !cell_start || !cell_of || !boxes || !row_ptr || !nnz_out || n <= 0 ||
      n > LNV_MAX_ATOMS || n_cells <= 0 || !(R >= 0.0))
    return LNV_EINVAL;
  const double R2 = R * R;
  const int grid = (n + 3) / 4;
  k_neighbours<<<grid, 256, 0, s>>>(pos, n, 1.0, 1.0, 1.0, cell_of, cell_start, boxes, R2,
                                    row_ptr, nullptr, nullptr, 0);
  LNV_LAUNCH_CHECK();
  k_scan<int32_t><<<1, 1024, 0, s>>>(row_ptr, n);
  LNV_LAUNCH_CHECK();
  LNV_TRY(read_total_int(row_ptr + n, nnz_out, s));
  if (!col) return LNV_OK;
  if (cap < *nnz_out) return LNV_ECAPACITY;
  k_neighbours<<<grid, 256, 0, s>>>(pos, n, 1.0, 1.0, 1.0, cell_of, cell_start, boxes, R2,
                                    nullptr, row_ptr, col, 1);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_pattern_product(const lnv_pattern* A, const lnv_pattern* B,
                                   const lnv_pattern* mask, int32_t* row_ptr, int32_t* col,
                                   int64_t cap, int64_t* nnz_out, int64_t* row_triples,
                                   int64_t* triples_out, hipStream_t s) {
  if (!A || !B || !row_ptr || !nnz_out) return LNV_EINVAL;
  if (!A->row_ptr || !A->col || !B->row_ptr || !B->col) return LNV_EPATTERN;
  const int n = A->n;
  if (n <= 0 || n > LNV_MAX_ATOMS || B->n != n) return LNV_EPATTERN;
  if (mask && (mask->n != n || !mask->row_ptr || !mask->col)) return LNV_EPATTERN;
  if (triples_out && !row_triples) return LNV_EINVAL;
  const size_t lds = 2 * (size_t)((n + 31) / 32) * sizeof(unsigned int);
  const int* mrp = mask ? mask->row_ptr : nullptr;
  const int* mcol = mask ? mask->col : nullptr;
  k_symbolic<<<n, 256, lds, s>>>(n, A->row_ptr, A->col, B->row_ptr, B->col, mrp, mcol,
                                 row_ptr, nullptr, nullptr,
                                 reinterpret_cast<long long*>(row_triples), 0, nullptr);
  LNV_LAUNCH_CHECK();
  k_scan<int32_t><<<1, 1024, 0, s>>>(row_ptr, n);
  LNV_LAUNCH_CHECK();
  if (row_triples) {
    k_scan<long long><<<1, 1024, 0, s>>>(reinterpret_cast<long long*>(row_triples), n);
    LNV_LAUNCH_CHECK();
  }
  LNV_TRY(read_total_int(row_ptr + n, nnz_out, s));
  if (triples_out) {
    LNV_HIP(hipMemcpyAsync(triples_out, row_triples + n, sizeof(int64_t),
                           hipMemcpyDeviceToHost, s));
    LNV_HIP(hipStreamSynchronize(s));
  }
  if (!col) return LNV_OK;
  if (cap < *nnz_out) return LNV_ECAPACITY;
  k_symbolic<<<n, 256, lds, s>>>(n, A->row_ptr, A->col, B->row_ptr, B->col, mrp, mcol,
                                 nullptr, row_ptr, col, nullptr, 1, nullptr);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_pattern_flops(const lnv_pattern* A, const lnv_pattern* B,
                                 const lnv_pattern* mask, const int32_t* row_fun,
                                 int64_t* flops_out, hipStream_t s) {
  if (!A || !B || !row_fun || !flops_out) return LNV_EINVAL;
  if (!A->row_ptr || !A->col || !B->row_ptr || !B->col) return LNV_EPATTERN;
  const int n = A->n;
  if (n <= 0 || n > LNV_MAX_ATOMS || B->n != n) return LNV_EPATTERN;
  if (mask && (mask->n != n || !mask->row_ptr || !mask->col)) return LNV_EPATTERN;
  const size_t lds = 2 * (size_t)((n + 31) / 32) * sizeof(unsigned int);
  int32_t* counts = nullptr;
  long long* tr = nullptr;
  LNV_HIP(hipMallocAsync(reinterpret_cast<void**>(&counts), sizeof(int32_t) * (n + 1), s));
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&tr), sizeof(long long) * (n + 1), s);
  if (e == hipSuccess) {
    k_symbolic<<<n, 256, lds, s>>>(n, A->row_ptr, A->col, B->row_ptr, B->col,
                                   mask ? mask->row_ptr : nullptr, mask ? mask->col : nullptr,
                                   counts, nullptr, nullptr, tr, 0, row_fun);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    k_scan<long long><<<1, 1024, 0, s>>>(tr, n);
    e = hipGetLastError();
  }
  long long total = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&total, tr + n, sizeof(long long), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (tr) (void)hipFreeAsync(tr, s);
  (void)hipFreeAsync(counts, s);
  if (e != hipSuccess) {
    set_hip_error(e);
    return LNV_EHIP;
  }
  *flops_out = 2 * total;
  return LNV_OK;
}

extern "C" int lnv_pattern_half(const lnv_pattern* P, int32_t* row_ptr, int32_t* col,
                                 int64_t cap, int64_t* nnz_out, hipStream_t s) {
  if (!P || !row_ptr || !nnz_out) return LNV_EINVAL;
  if (!P->row_ptr || !P->col || P->n <= 0) return LNV_EPATTERN;
  const int n = P->n;
  const int grid = (n + 255) / 256;
  k_half<<<grid, 256, 0, s>>>(n, P->row_ptr, P->col, row_ptr, nullptr, nullptr);
  LNV_LAUNCH_CHECK();
  k_scan<int32_t><<<1, 1024, 0, s>>>(row_ptr, n);
  LNV_LAUNCH_CHECK();
  LNV_TRY(read_total_int(row_ptr + n, nnz_out, s));
  if (!col) return LNV_OK;
  if (cap < *nnz_out) return LNV_ECAPACITY;
  k_half<<<grid, 256, 0, s>>>(n, P->row_ptr, P->col, nullptr, row_ptr, col);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_cells(const double* pos, int32_t n_units, const double* box,
                         const int32_t* g, const double* origin, int32_t* cell, int32_t* slot,
                         int32_t* occ_out, hipStream_t s) {
  if (!pos || !box || !g || !origin || !cell || !slot || !occ_out || n_units <= 0)
    return LNV_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (g[d] < 1 || g[d] > 1024 || !(box[d] > 0.0)) return LNV_EINVAL;
  std::vector<double> hp((size_t)n_units * 3);
  LNV_HIP(hipMemcpyAsync(hp.data(), pos, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  LNV_HIP(hipStreamSynchronize(s));
  const int64_t ncell = (int64_t)g[0] * g[1] * g[2];
  if (ncell > ((int64_t)1 << 26)) return LNV_EINVAL;
  std::vector<int32_t> hc(n_units), hs(n_units), fill((size_t)ncell, 0);
  int32_t occ = 0;
  for (int u = 0; u < n_units; ++u) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
      double f = (hp[(size_t)u * 3 + d] - origin[d]) / box[d];
      f -= std::floor(f);
      c[d] = std::min(g[d] - 1, std::max(0, (int)(f * g[d])));
    }
    hc[u] = c[0] | (c[1] << 10) | (c[2] << 20);
    const int64_t k = ((int64_t)c[0] * g[1] + c[1]) * g[2] + c[2];
    hs[u] = fill[(size_t)k]++;
    occ = std::max(occ, fill[(size_t)k]);
  }
  LNV_HIP(hipMemcpyAsync(cell, hc.data(), sizeof(int32_t) * n_units, hipMemcpyHostToDevice, s));
  LNV_HIP(hipMemcpyAsync(slot, hs.data(), sizeof(int32_t) * n_units, hipMemcpyHostToDevice, s));
  LNV_HIP(hipStreamSynchronize(s));
  *occ_out = occ;
  return LNV_OK;
}

extern "C" int lnv_pattern_index(lnv_pattern* P, const int32_t* cell, const int32_t* slot,
                                 const int32_t* g, int32_t occ, int32_t qs, int32_t* tab,
                                 int64_t cap, int64_t* len_out, hipStream_t s) {
  if (!P || !cell || !slot || !g || !len_out || occ <= 0 || (qs != 0 && qs != 2))
    return LNV_EINVAL;
  if (!P->row_ptr || !P->col || P->n <= 0) return LNV_EPATTERN;
  if ((P->n & ((1 << qs) - 1)) != 0) return LNV_EPATTERN;
  for (int d = 0; d < 3; ++d)
    if (g[d] < 1 || g[d] > 1024) return LNV_EINVAL;
  if (qs == 2) {  // atom units describe tile4 patterns only
    int32_t t4 = 0;
    LNV_TRY(lnv_pattern_tile4(P, &t4, s));
    if (t4 != 1) return LNV_EPATTERN;
  }
  const int nu = P->n >> qs;
  // window: the largest wrapped offset along each axis
  int32_t* ext = nullptr;
  LNV_HIP(hipMallocAsync(reinterpret_cast<void**>(&ext), 4 * sizeof(int32_t), s));
  int32_t hext[4] = {0, 0, 0, 0};
  hipError_t e = hipMemsetAsync(ext, 0, 4 * sizeof(int32_t), s);
  if (e == hipSuccess) {
    k_ix_extent<<<nu, 256, 0, s>>>(nu, qs, P->row_ptr, P->col, cell, g[0], g[1], g[2], ext);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hext, ext, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t ef = hipFreeAsync(ext, s);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) {
    set_hip_error(e);
    return LNV_EHIP;
  }
  lnv_index& x = P->ix;
  x.tab = nullptr;
  x.cell = cell;
  x.slot = slot;
  x.occ = occ;
  x.qs = qs;
  int64_t stride = occ;
  for (int d = 0; d < 3; ++d) {
    x.g[d] = g[d];
    x.r[d] = std::min(hext[d], g[d] - 1);
    x.w[d] = std::min(2 * x.r[d] + 1, g[d]);
    stride *= x.w[d];
  }
  x.stride = stride;
  *len_out = (int64_t)nu * stride + 1;   // + the trailing -1 entry
  if (!tab) return LNV_OK;
  if (cap < *len_out) return LNV_ECAPACITY;
  int32_t* bad = nullptr;
  LNV_HIP(hipMallocAsync(reinterpret_cast<void**>(&bad), sizeof(int32_t), s));
  int32_t hbad = 0;
  e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
  if (e == hipSuccess) e = hipMemsetAsync(tab, 0xFF, sizeof(int32_t) * (size_t)*len_out, s);
  if (e == hipSuccess) {
    x.tab = tab;
    k_ix_fill<<<nu, 256, 0, s>>>(nu, make_ix(P), P->col, tab, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t ef2 = hipFreeAsync(bad, s);
  if (e == hipSuccess) e = ef2;
  if (e != hipSuccess) {
    x.tab = nullptr;
    set_hip_error(e);
    return LNV_EHIP;
  }
  if (hbad) {
    x.tab = nullptr;
    return LNV_EPATTERN;
  }
  return LNV_OK;
}

extern "C" int lnv_pattern_tile4(const lnv_pattern* P, int32_t* ok_out, hipStream_t s) {
  if (!P || !ok_out) return LNV_EINVAL;
  if (!P->row_ptr || !P->col || P->n <= 0) return LNV_EPATTERN;
  if (P->n % 4 != 0) {
    *ok_out = 0;
    return LNV_OK;
  }
  int32_t* bad = nullptr;
  LNV_HIP(hipMallocAsync(reinterpret_cast<void**>(&bad), sizeof(int32_t), s));
  int32_t hbad[1] = {1};
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
  if (e == hipSuccess) {
    k_tile4<<<P->n, 256, 0, s>>>(P->n, P->row_ptr, P->col, bad);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  const hipError_t ef = hipFreeAsync(bad, s);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) {
    set_hip_error(e);
    return LNV_EHIP;
  }
  *ok_out = hbad[0] == 0 ? 1 : 0;
  return LNV_OK;
}

extern "C" int lnv_pattern_items(const lnv_pattern* P, int32_t* items, int64_t cap,
                                 int32_t* n_items_out, hipStream_t s) {
  if (!P || !P->row_ptr || P->n <= 0) return LNV_EPATTERN;
  if (!n_items_out) return LNV_EINVAL;
  const int n = P->n;
  int32_t* cnt = nullptr;
  LNV_HIP(hipMallocAsync(reinterpret_cast<void**>(&cnt), sizeof(int32_t) * (n + 1), s));
  const int grid = (n + 255) / 256;
  k_items<<<grid, 256, 0, s>>>(n, P->row_ptr, cnt, nullptr, nullptr);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    k_scan<int32_t><<<1, 1024, 0, s>>>(cnt, n);
    e = hipGetLastError();
  }
  int32_t total = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&total, cnt + n, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  int st = LNV_OK;
  if (e != hipSuccess) {
    set_hip_error(e);
    st = LNV_EHIP;
  } else {
    *n_items_out = total;
    if (items) {
      if (cap < total) {
        st = LNV_ECAPACITY;
      } else {
        k_items<<<grid, 256, 0, s>>>(n, P->row_ptr, nullptr, cnt, items);
        e = hipGetLastError();
        if (e != hipSuccess) {
          set_hip_error(e);
          st = LNV_EHIP;
        }
      }
    }
  }
  hipError_t ef = hipFreeAsync(cnt, s);
  if (st == LNV_OK && ef != hipSuccess) {
    set_hip_error(ef);
    st = LNV_EHIP;
  }
  return st;
}

extern "C" int lnv_synth_blocks(const double* pos, const double* box, const int32_t* nfun,
                                const int32_t* atom_of, const int32_t* off_of, const lnv_bsm* M,
                                int32_t kind, double R, double decay, uint64_t seed,
                                double scale, hipStream_t s) {
  if (!pos || !box || !bsm_ok(M) || (kind != 0 && kind != 1) || !(R >= 0.0) ||
      !(decay > 0.0))
    return LNV_EINVAL;
  if (!M->pat->row_ptr || !M->pat->col) return LNV_EPATTERN;
  if (M->blk <= 0 || M->blk > 16) return LNV_EUNSUPPORTED;
  if ((atom_of == nullptr) != (off_of == nullptr)) return LNV_EINVAL;
  const int n = M->pat->n;
  if (n >= (1 << 24)) return LNV_EUNSUPPORTED;  // counter layout: 24-bit atom ids
  k_synth<<<n, 128, 0, s>>>(pos, box[0], box[1], box[2], nullptr, nullptr, nullptr, nullptr,
                            nfun, atom_of, off_of, M->blk, M->pat->row_ptr, M->pat->col,
                            static_cast<double*>(M->val), kind, R, decay, seed, scale);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_forces(const double* pos, const double* box, const int32_t* nfun,
                          const int32_t* atom_of, const int32_t* off_of, uint64_t seed,
                          double scale, const lnv_bsm* GS, const lnv_bsm* GNS, double mu,
                          double R_S, double decay_S, const lnv_bsm* GH, double R_H,
                          double decay_H, int32_t n_seg, const int32_t* seg_ptr,
                          const int32_t* seg_atom, double* acc, double* F, hipStream_t s) {
  if (!pos || !box || !bsm_ok(GS) || !bsm_ok(GH) || !seg_ptr || !seg_atom || !acc || !F ||
      n_seg <= 0 || !(decay_S > 0.0) || !(decay_H > 0.0))
    return LNV_EINVAL;
  if ((atom_of == nullptr) != (off_of == nullptr)) return LNV_EINVAL;
  if (GNS && (!bsm_ok(GNS) || GNS->pat != GS->pat)) return LNV_EPATTERN;
  const lnv_pattern *ps = GS->pat, *ph = GH->pat;
  if (GS->blk != GH->blk || GS->blk <= 0 || GS->blk > 16) return LNV_EUNSUPPORTED;
  if (ps->n != ph->n || !has_ix(ps) || !has_ix(ph) || !ps->row_ptr || !ph->row_ptr)
    return LNV_EPATTERN;
  const int n = ps->n;
  LNV_HIP(hipMemsetAsync(acc, 0, sizeof(double) * 3 * (size_t)n, s));
  k_pos_grad<<<n, 128, 0, s>>>(pos, box[0], box[1], box[2], nfun, atom_of, off_of, GS->blk, n,
                               ps->row_ptr, ps->col, make_ix(ps), static_cast<const double*>(GS->val),
                               GNS ? static_cast<const double*>(GNS->val) : nullptr, mu, 0, R_S,
                               decay_S, seed, scale, acc);
  LNV_LAUNCH_CHECK();
  k_pos_grad<<<n, 128, 0, s>>>(pos, box[0], box[1], box[2], nfun, atom_of, off_of, GH->blk, n,
                               ph->row_ptr, ph->col, make_ix(ph), static_cast<const double*>(GH->val),
                               nullptr, 0.0, 1, R_H, decay_H, seed, scale, acc);
  LNV_LAUNCH_CHECK();
  k_seg_force<<<(n_seg + 63) / 64, 64, 0, s>>>(n_seg, seg_ptr, seg_atom, acc, F);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_synth_blocks_cells(const double* pos, const int32_t* cell_of,
                                      const double* boxes, const uint64_t* seeds,
                                      const int32_t* atom_of, const int32_t* fun_of,
                                      const int32_t* off_of, const lnv_bsm* M, int32_t kind,
                                      double R, double decay, double scale, hipStream_t s) {
  if (!pos || !cell_of || !boxes || !seeds || !atom_of || !fun_of || !off_of || !bsm_ok(M) ||
      (kind != 0 && kind != 1) || !(R >= 0.0) || !(decay > 0.0))
    return LNV_EINVAL;
  if (!M->pat->row_ptr || !M->pat->col) return LNV_EPATTERN;
  if (M->blk <= 0 || M->blk > 16) return LNV_EUNSUPPORTED;
  const int n = M->pat->n;
  k_synth<<<n, 128, 0, s>>>(pos, 1.0, 1.0, 1.0, cell_of, boxes, seeds, fun_of, nullptr, atom_of,
                            off_of, M->blk, M->pat->row_ptr, M->pat->col,
                            static_cast<double*>(M->val), kind, R, decay, 0ull, scale);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_pattern_transpose_map(const lnv_pattern* P, const lnv_pattern* PT,
                                         int32_t* perm, hipStream_t s) {
  if (!P || !PT || !perm) return LNV_EINVAL;
  if (!P->row_ptr || !P->col || !has_ix(PT) || P->n != PT->n || P->n <= 0 ||
      P->nnzb != PT->nnzb)
    return LNV_EPATTERN;
  int32_t* bad = nullptr;
  LNV_HIP(hipMallocAsync(reinterpret_cast<void**>(&bad), sizeof(int32_t), s));
  hipError_t e = hipMemsetAsync(bad, 0, sizeof(int32_t), s);
  if (e == hipSuccess) {
    k_tmap<<<P->n, 256, 0, s>>>(P->n, P->row_ptr, P->col, make_ix(PT), perm, bad);
    e = hipGetLastError();
  }
  int32_t hbad = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hbad, bad, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipError_t ef = hipFreeAsync(bad, s);
  if (e != hipSuccess) {
    set_hip_error(e);
    return LNV_EHIP;
  }
  if (ef != hipSuccess) {
    set_hip_error(ef);
    return LNV_EHIP;
  }
  return hbad ? LNV_EPATTERN : LNV_OK;
}

extern "C" int lnv_pattern_cluster(const lnv_pattern* P, int32_t m, int32_t g, int32_t* cl_ptr,
                                   int32_t* cl_col, int32_t* cl_pos, int32_t* cl_cell,
                                   int64_t cap, int32_t* cl_items, int64_t items_cap,
                                   int64_t* len_out, int32_t* n_items_out, hipStream_t s) {
  if (!P || !cl_ptr || !len_out || !n_items_out) return LNV_EINVAL;
  if (!((m == 4 && g == 1) || (m == 16 && (g == 4 || g == 8)))) return LNV_EUNSUPPORTED;
  if (!P->row_ptr || !P->col || !has_ix(P) || P->n <= 0 || P->n > LNV_MAX_ATOMS)
    return LNV_EPATTERN;
  const int n = P->n;
  const int nc = (n + m - 1) / m;
  const size_t lds = (size_t)((n + 31) / 32) * sizeof(unsigned int);
  k_cluster_union<<<nc, 256, lds, s>>>(n, m, P->row_ptr, P->col, make_ix(P), cl_ptr, nullptr,
                                       nullptr, nullptr, nullptr, 0);
  LNV_LAUNCH_CHECK();
  k_scan<int32_t><<<1, 1024, 0, s>>>(cl_ptr, nc);
  LNV_LAUNCH_CHECK();
  LNV_TRY(read_total_int(cl_ptr + nc, len_out, s));
  // items: pieces of 64/g columns per cluster
  int32_t* cnt = nullptr;
  LNV_HIP(hipMallocAsync(reinterpret_cast<void**>(&cnt), sizeof(int32_t) * (nc + 1), s));
  const int piece = 64 / g;
  const int gi = (nc + 255) / 256;
  k_cluster_items<<<gi, 256, 0, s>>>(nc, piece, cl_ptr, cnt, nullptr, nullptr);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    k_scan<int32_t><<<1, 1024, 0, s>>>(cnt, nc);
    e = hipGetLastError();
  }
  int32_t nit = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&nit, cnt + nc, sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  int st = LNV_OK;
  if (e != hipSuccess) {
    set_hip_error(e);
    st = LNV_EHIP;
  } else {
    *n_items_out = nit;
    if (cl_col) {
      if (!cl_pos || !cl_items || !cl_cell) {
        st = LNV_EINVAL;
      } else if (cap < *len_out || items_cap < nit) {
        st = LNV_ECAPACITY;
      } else {
        k_cluster_union<<<nc, 256, lds, s>>>(n, m, P->row_ptr, P->col, make_ix(P), nullptr,
                                             cl_ptr, cl_col, cl_pos, cl_cell, 1);
        e = hipGetLastError();
        if (e == hipSuccess) {
          k_cluster_items<<<gi, 256, 0, s>>>(nc, piece, cl_ptr, nullptr, cnt, cl_items);
          e = hipGetLastError();
        }
        if (e != hipSuccess) {
          set_hip_error(e);
          st = LNV_EHIP;
        }
      }
    }
  }
  hipError_t ef = hipFreeAsync(cnt, s);
  if (st == LNV_OK && ef != hipSuccess) {
    set_hip_error(ef);
    st = LNV_EHIP;
  }
  return st;
}
