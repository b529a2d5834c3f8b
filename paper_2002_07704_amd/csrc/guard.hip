// Occupation bounds of L S for the CG runaway guard.
//
// K = 3LSL - 2LSLSL is a density matrix only while the eigenvalues of L S
// (the occupation numbers of the auxiliary matrix, in the support-function
// basis of Sec. II.B) stay near [0, 1]: the McWeeny form maps each
// occupation x to 3x^2 - 2x^3, which has its minimum at 0 and maximum at 1
// and runs away outside.  L S is self-adjoint in the inner product
// <x, y>_S = x^T S y (S symmetric positive definite), so Lanczos in that
// inner product brackets its spectrum: the extreme eigenvalues of the
// tridiagonal matrix of m steps lie inside [lambda_min, lambda_max] and
// converge to them from inside.
//
// One Lanczos step: u = L (S v) (S v kept from the previous step),
// a = (S v)^T u, u -= a v + b_prev v_prev, S u (one multiply), b = sqrt(u^T S u),
// v <- u / b, S v <- S u / b: two block-sparse matrix-vector products and two
// fixed-order reductions.  The start vector is a fixed pseudo-random vector
// (SplitMix64 counter of the row and element), so the estimate is the same
// run to run.  Everything stays on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "internal.h"

namespace lnv {
namespace {

constexpr int kLzMax = 64;      // most Lanczos steps
constexpr int kRedThreads = 1024;

// y = A x for 4x4-blocked A on its pattern: one wavefront per block row i;
// lane l takes the row's blocks l, l + 64, ... in order and the four row
// sums are reduced across the wave by the fixed butterfly (the same
// summation order every run).
__global__ __launch_bounds__(256) void k_bsr_mv(int n, const int* __restrict__ rp,
                                                const int* __restrict__ col,
                                                const double* __restrict__ A,
                                                const double* __restrict__ x,
                                                double* __restrict__ y) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int p = rp[i] + lane; p < rp[i + 1]; p += kWave) {
    const double* a = A + (size_t)p * 16;
    const double* xv = x + (size_t)col[p] * 4;
    const double x0 = xv[0], x1 = xv[1], x2 = xv[2], x3 = xv[3];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      acc[r] = fma(a[r * 4 + 3], x3, fma(a[r * 4 + 2], x2, fma(a[r * 4 + 1], x1,
                                                              fma(a[r * 4], x0, acc[r]))));
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) acc[r] = wave_sum(acc[r]);
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) y[(size_t)i * 4 + r] = acc[r];
  }
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// start vector: entries in [-0.5, 0.5) from a SplitMix64 counter
__global__ __launch_bounds__(256) void k_lz_start(int64_t m, double* __restrict__ v) {
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < m; e += (int64_t)gridDim.x * 256) {
    const uint64_t z = mix64(0x9e3779b97f4a7c15ull * (uint64_t)(e + 1));
    v[e] = (double)(z >> 11) * 0x1.0p-53 - 0.5;
  }
}

// Fixed-order dot product of one workgroup (kRedThreads threads).
__device__ double block_dot(int64_t m, const double* __restrict__ a, const double* __restrict__ b,
                            double* sh) {
  double t = 0.0;
  for (int64_t e = threadIdx.x; e < m; e += kRedThreads) t = fma(a[e], b[e], t);
  return block_sum(t, sh);
}

// Normalise the start vector in the S norm: v = r / |r|_S, Sv = Sr / |r|_S,
// v_prev = 0.  sc[0]: |r|_S (for the check that the start is not zero).
__global__ __launch_bounds__(kRedThreads) void k_lz_init(int64_t m, double* __restrict__ v,
                                                          double* __restrict__ Sv,
                                                          double* __restrict__ vp,
                                                          double* __restrict__ sc) {
  __shared__ double sh[16];
  __shared__ double nrm;
  const double d = block_dot(m, v, Sv, sh);
  if (threadIdx.x == 0) nrm = d > 0.0 ? sqrt(d) : 0.0;
  __syncthreads();
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t e = threadIdx.x; e < m; e += kRedThreads) {
    v[e] *= inv;
    Sv[e] *= inv;
    vp[e] = 0.0;
  }
  if (threadIdx.x == 0) sc[0] = nrm;
}

// a_j = Sv^T u;  u <- u - a_j v - b_{j-1} v_prev
__global__ __launch_bounds__(kRedThreads) void k_lz_alpha(int64_t m, int j,
                                                           const double* __restrict__ v,
                                                           const double* __restrict__ Sv,
                                                           const double* __restrict__ vp,
                                                           double* __restrict__ u,
                                                           double* __restrict__ ab) {
  __shared__ double sh[16];
  __shared__ double a;
  const double d = block_dot(m, Sv, u, sh);
  if (threadIdx.x == 0) a = d;
  __syncthreads();
  const double bp = j > 0 ? ab[kLzMax + j - 1] : 0.0;
  for (int64_t e = threadIdx.x; e < m; e += kRedThreads) u[e] = u[e] - a * v[e] - bp * vp[e];
  if (threadIdx.x == 0) ab[j] = a;
}

// b_j = sqrt(u^T S u);  v_prev <- v, v <- u / b_j, Sv <- Su / b_j
__global__ __launch_bounds__(kRedThreads) void k_lz_beta(int64_t m, int j,
                                                          double* __restrict__ v,
                                                          double* __restrict__ Sv,
                                                          double* __restrict__ vp,
                                                          const double* __restrict__ u,
                                                          const double* __restrict__ Su,
                                                          double* __restrict__ ab) {
  __shared__ double sh[16];
  __shared__ double b;
  const double d = block_dot(m, u, Su, sh);
  if (threadIdx.x == 0) b = d > 0.0 ? sqrt(d) : 0.0;
  __syncthreads();
  const double inv = b > 0.0 ? 1.0 / b : 0.0;
  for (int64_t e = threadIdx.x; e < m; e += kRedThreads) {
    vp[e] = v[e];
    v[e] = u[e] * inv;
    Sv[e] = Su[e] * inv;
  }
  if (threadIdx.x == 0) ab[kLzMax + j] = b;
}

// Number of eigenvalues of the tridiagonal (a[0..k), b[0..k-1)) below x
// (Sturm sequence of the LDL^T pivots).
__device__ int sturm_count(const double* a, const double* b, int k, double x) {
  int cnt = 0;
  double q = 1.0;
  for (int i = 0; i < k; ++i) {
    const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    q = (a[i] - x) - (i > 0 ? bb / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Extreme eigenvalues of the tridiagonal of the first k steps (k stops
// early at a zero b: the Krylov space is exhausted) by bisection inside the
// Gershgorin interval; out[0] = smallest, out[1] = largest.
__global__ void k_lz_extremes(int steps, const double* __restrict__ ab, double* __restrict__ out,
                              const double* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  const double* a = ab;
  const double* b = ab + kLzMax;
  int k = steps;
  for (int i = 0; i < steps - 1; ++i)
    if (!(b[i] > 0.0)) {
      k = i + 1;
      break;
    }
  if (!(sc[0] > 0.0) || k < 1) {
    out[0] = out[1] = NAN;
    return;
  }
  double lo = INFINITY, hi = -INFINITY;
  for (int i = 0; i < k; ++i) {
    const double rad = (i > 0 ? fabs(b[i - 1]) : 0.0) + (i + 1 < k ? fabs(b[i]) : 0.0);
    lo = fmin(lo, a[i] - rad);
    hi = fmax(hi, a[i] + rad);
  }
  // smallest: largest x with count(x) == 0; largest: smallest x with count(x) == k
  double l = lo, h = hi;
  for (int it = 0; it < 200 && h - l > 1e-15 * fmax(1.0, fabs(l) + fabs(h)); ++it) {
    const double mid = 0.5 * (l + h);
    if (sturm_count(a, b, k, mid) == 0) l = mid; else h = mid;
  }
  out[0] = 0.5 * (l + h);
  l = lo;
  h = hi;
  for (int it = 0; it < 200 && h - l > 1e-15 * fmax(1.0, fabs(l) + fabs(h)); ++it) {
    const double mid = 0.5 * (l + h);
    if (sturm_count(a, b, k, mid) < k) l = mid; else h = mid;
  }
  out[1] = 0.5 * (l + h);
}

}  // namespace

int occupation_bounds(const lnv_bsm* L, const lnv_bsm* S, int steps, double* work, double* out,
                      hipStream_t s) {
  const int n = L->pat->n;
  const int64_t m = (int64_t)n * 4;
  double* v = work;
  double* Sv = v + m;
  double* vp = Sv + m;
  double* u = vp + m;
  double* Su = u + m;
  double* ab = Su + m;           // [2 * kLzMax]: a_j, b_j
  double* sc = ab + 2 * kLzMax;  // [1]: |start|_S
  const int mvg = (n + 3) / 4;   // four block rows (wavefronts) per workgroup
  const int vg = (int)((m + 255) / 256 < 1024 ? (m + 255) / 256 : 1024);
  const double* Lv = static_cast<const double*>(L->val);
  const double* Sval = static_cast<const double*>(S->val);
  k_lz_start<<<vg, 256, 0, s>>>(m, v);
  LNV_LAUNCH_CHECK();
  k_bsr_mv<<<mvg, 256, 0, s>>>(n, S->pat->row_ptr, S->pat->col, Sval, v, Sv);
  LNV_LAUNCH_CHECK();
  k_lz_init<<<1, kRedThreads, 0, s>>>(m, v, Sv, vp, sc);
  LNV_LAUNCH_CHECK();
  for (int j = 0; j < steps; ++j) {
    k_bsr_mv<<<mvg, 256, 0, s>>>(n, L->pat->row_ptr, L->pat->col, Lv, Sv, u);
    LNV_LAUNCH_CHECK();
    k_lz_alpha<<<1, kRedThreads, 0, s>>>(m, j, v, Sv, vp, u, ab);
    LNV_LAUNCH_CHECK();
    if (j + 1 == steps) break;
    k_bsr_mv<<<mvg, 256, 0, s>>>(n, S->pat->row_ptr, S->pat->col, Sval, u, Su);
    LNV_LAUNCH_CHECK();
    k_lz_beta<<<1, kRedThreads, 0, s>>>(m, j, v, Sv, vp, u, Su, ab);
    LNV_LAUNCH_CHECK();
  }
  k_lz_extremes<<<1, 64, 0, s>>>(steps, ab, out, sc);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

}  // namespace lnv

using namespace lnv;

extern "C" int64_t lnv_lanczos_len(int32_t n_rows) {
  return n_rows > 0 ? (int64_t)n_rows * 4 * 5 + 2 * kLzMax + 8 : 0;
}

extern "C" int lnv_occupation_bounds(const lnv_bsm* L, const lnv_bsm* S, int32_t steps,
                                     double* work, double* out, hipStream_t s) {
  if (!bsm_ok(L) || !bsm_ok(S) || !work || !out || steps < 1 || steps > kLzMax)
    return LNV_EINVAL;
  if (L->blk != 4 || S->blk != 4) return LNV_EUNSUPPORTED;
  if (L->pat->n != S->pat->n || !L->pat->row_ptr || !L->pat->col || !S->pat->row_ptr ||
      !S->pat->col)
    return LNV_EPATTERN;
  return occupation_bounds(L, S, steps, work, out, s);
}
