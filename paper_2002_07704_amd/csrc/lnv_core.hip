// a4-a7: LNV evaluation and conjugate-gradient step on the device.
//
// Sec. II.C.2: K = 3LSL - 2LSLSL, E = 2 Tr[KH], minimised over the elements
// of the range-restricted L with dE/dL under the electron-number constraint
// N = 2 Tr[KS] = N_e.  With A = LS (stored transposed, SL), X = HLS and
// Z = SLS at natural range, every trace and gradient needs six block-sparse
// products; the three on L's pattern are formed with A^T on the left so the
// left operand's range (that of LS) bounds the contraction.
//
// Every scalar decision (mu, beta, alpha, delta, resets) is taken by a
// one-workgroup kernel from partial sums written by the vector kernels, so a
// CG step is a fixed sequence of launches with no host synchronisation.
// All reductions use a fixed association: results are reproducible bitwise.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <utility>

#include "internal.h"

namespace lnv {

namespace {
thread_local int g_last_hip = 0;
}

void set_hip_error(hipError_t e) { g_last_hip = (int)e; }

namespace {

// ------------------------------------------------------------------ reductions
struct Red {
  int off, count, stride, dst, op;  // op 0: sum, 1: max
  int kind;  // batch stages: 1 partials per work item of L's pattern, 2 per vector workgroup
};
struct RedList {
  Red r[8];
  int nr;
};

enum Stage {
  ST_NONE = 0, ST_EVAL, ST_BETA, ST_PROJ, ST_ALPHA, ST_NCHK, ST_DELTA, ST_INIT, ST_MU, ST_SIGMA,
  ST_PM0, ST_PM
};

// A batch of independent cells minimised together (lnv_batch): cell c owns
// L's work items item_ptr[c] .. item_ptr[c+1]-1 and values val_ptr[c] ..
// val_ptr[c+1]-1 (rows of a cell are consecutive, so both are ranges), its
// scalars at sc + c * LNV_NSCALARS.  The vector kernels give each cell `per`
// workgroups (partial c * per + q); n = 0 is the plain one-system path.
struct Seg {
  int n = 0, per = 0;
  const int* item_ptr = nullptr;
  const int64_t* val_ptr = nullptr;
  const int* row_cell = nullptr;
  const double* n_elec = nullptr;
  const int* row_off = nullptr;     // [n+1] first row of each cell
  const double* n_orb = nullptr;    // [n] orbitals (functions present) of each cell
  int sc_stride = LNV_NSCALARS;     // scalars per cell
};
enum { RK_ALL = 0, RK_ITEMS = 1, RK_VEC = 2, RK_ROWS = 3 };

struct StageArgs {
  double n_elec, n_tol, step_cap;
  int reset;          // host: k % reset_period == 0
  double* en_out;     // ST_EVAL: optional device [2]
  int k;              // ST_BETA: iteration index
  int reset_period;   // ST_BETA: guard repeat window
  int occ_checked;    // ST_BETA: occupation bounds computed this iteration
  double pm_n, pm_theta, pm_tol;   // ST_PM0 / ST_PM: orbitals, occupied states, tolerance
  double* pm_hist;                 // ST_PM: device [4 * pm_hist_len] (c, t1, t2, t3)
  int pm_hist_len;
  int pm_batch;                    // ST_PM: a stopped cell keeps K (coefficients 1, 0, 0)
};

// Runaway guard (ST_BETA): a rise of E beyond this fraction of |E| counts
// as a rise; occupations outside [kOccLo, kOccHi] trip the guard.
constexpr double kRiseTol = 1e-11;
constexpr double kOccLo = -0.5, kOccHi = 1.5;

// Newton's method on a3 x^3 + a2 x^2 + a1 x + a0 from x until the step is
// below 4 ulp of x (at most 100 steps); returns false when it does not settle
// on a root (residual above 1e-12 of the size of the terms).
__device__ bool newton_cubic(double a3, double a2, double a1, double a0, double* x) {
  double v = *x;
  for (int it = 0; it < 100; ++it) {
    const double f = ((a3 * v + a2) * v + a1) * v + a0;
    const double df = (3.0 * a3 * v + 2.0 * a2) * v + a1;
    if (df == 0.0 || !isfinite(f)) break;
    const double nv = v - f / df;
    const bool done = fabs(nv - v) <= 8.9e-16 * fabs(nv);
    v = nv;
    if (done) break;
  }
  const double f = ((a3 * v + a2) * v + a1) * v + a0;
  const double scale = fabs(a3 * v * v * v) + fabs(a2 * v * v) + fabs(a1 * v) + fabs(a0);
  *x = v;
  return isfinite(v) && fabs(f) <= 1e-12 * scale;
}

// Real roots of a3 x^3 + a2 x^2 + a1 x + a0 (leading zero coefficients drop
// the degree).  Candidates: the closed forms (stable quadratic formula;
// Cardano / Viete trigonometric form for the cubic) and, for the root nearest
// zero, Newton's method from the linear estimate -a0/a1.  Every candidate is
// refined by Newton's method to full precision (the closed forms lose the
// small roots to cancellation when the others are large) and kept only when
// it satisfies the polynomial; duplicates are merged.
__device__ int real_roots(double a3, double a2, double a1, double a0, double* r) {
  double cand[4];
  int nc = 0;
  if (a3 == 0.0) {
    if (a2 == 0.0) {
      if (a1 == 0.0) return 0;
      r[0] = -a0 / a1;
      return 1;
    }
    const double disc = a1 * a1 - 4.0 * a2 * a0;
    if (disc < 0.0) return 0;
    const double q = -0.5 * (a1 + copysign(sqrt(disc), a1));
    if (q == 0.0) {
      cand[nc++] = 0.0;
    } else {
      cand[nc++] = q / a2;
      cand[nc++] = a0 / q;
    }
  } else {
    const double B = a2 / a3, C = a1 / a3, D = a0 / a3;
    const double Q = (B * B - 3.0 * C) / 9.0;
    const double R = (2.0 * B * B * B - 9.0 * B * C + 27.0 * D) / 54.0;
    const double Q3 = Q * Q * Q;
    if (R * R < Q3) {
      const double th = acos(R / sqrt(Q3));
      const double s = -2.0 * sqrt(Q);
      const double pi2 = 6.283185307179586476925286766559;
      cand[nc++] = s * cos(th / 3.0) - B / 3.0;
      cand[nc++] = s * cos((th + pi2) / 3.0) - B / 3.0;
      cand[nc++] = s * cos((th - pi2) / 3.0) - B / 3.0;
    } else {
      const double Aq = -copysign(cbrt(fabs(R) + sqrt(R * R - Q3)), R);
      const double Bq = Aq != 0.0 ? Q / Aq : 0.0;
      cand[nc++] = (Aq + Bq) - B / 3.0;
    }
  }
  if (a1 != 0.0) cand[nc++] = -a0 / a1;
  int nr = 0;
  for (int q = 0; q < nc; ++q) {
    double x = cand[q];
    if (!newton_cubic(a3, a2, a1, a0, &x)) continue;
    bool dup = false;
    for (int t = 0; t < nr; ++t)
      if (fabs(r[t] - x) <= 1e-12 * fmax(fabs(x), 1e-300)) dup = true;
    if (!dup && nr < 3) r[nr++] = x;
  }
  return nr;
}

// Local minimum of c0 + c1 a + c2 a^2 + c3 a^3: the root of
// 3 c3 a^2 + 2 c2 a + c1 with positive curvature 2 c2 + 6 c3 a.
__device__ bool cubic_min(double c1, double c2, double c3, double* alpha) {
  if (c3 == 0.0) {
    if (c2 > 0.0) {
      *alpha = -c1 / (2.0 * c2);
      return true;
    }
    return false;
  }
  const double disc = c2 * c2 - 3.0 * c3 * c1;
  if (!(disc > 0.0)) return false;
  const double sq = sqrt(disc);
  *alpha = c2 > 0.0 ? -c1 / (c2 + sq) : (-c2 + sq) / (3.0 * c3);
  return true;
}

// One workgroup per system (a batch: workgroup c takes cell c's partials,
// scalars and electron count).
__global__ __launch_bounds__(256) void k_scalar(const double* __restrict__ partials,
                                                RedList rl, double* __restrict__ sc,
                                                int stage, StageArgs sa, Seg sg) {
  __shared__ double sh[16];
  __shared__ double shm[256];
  const int cell = blockIdx.x;
  if (sg.n > 0) {
    sc += (size_t)cell * sg.sc_stride;
    if (sg.n_elec) {
      sa.n_elec = sg.n_elec[cell];
      sa.pm_theta = 0.5 * sg.n_elec[cell];
    }
    if (sg.n_orb) sa.pm_n = sg.n_orb[cell];
    if (sa.pm_hist) sa.pm_hist += (size_t)cell * 4 * sa.pm_hist_len;
    sa.en_out = nullptr;
  }
  for (int q = 0; q < rl.nr; ++q) {
    Red rd = rl.r[q];
    if (sg.n > 0 && rd.kind == RK_ITEMS) {
      rd.off += sg.item_ptr[cell] * rd.stride;
      rd.count = sg.item_ptr[cell + 1] - sg.item_ptr[cell];
    } else if (sg.n > 0 && rd.kind == RK_VEC) {
      rd.off += cell * sg.per * rd.stride;
      rd.count = sg.per;
    } else if (sg.n > 0 && rd.kind == RK_ROWS) {
      rd.off += sg.row_off[cell] * rd.stride;
      rd.count = sg.row_off[cell + 1] - sg.row_off[cell];
    }
    if (rd.op == 0) {
      // eight independent partial sums per thread, so eight loads are in
      // flight at a time (one workgroup reads every partial of the stage);
      // the order is fixed, so the result is reproducible bit for bit
      double v8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int t = threadIdx.x;
      for (; t + 7 * 256 < rd.count; t += 8 * 256) {
#pragma unroll
        for (int u = 0; u < 8; ++u) v8[u] += partials[rd.off + (size_t)(t + u * 256) * rd.stride];
      }
      for (; t < rd.count; t += 256) v8[0] += partials[rd.off + (size_t)t * rd.stride];
      double v = ((v8[0] + v8[1]) + (v8[2] + v8[3])) + ((v8[4] + v8[5]) + (v8[6] + v8[7]));
      v = block_sum(v, sh);
      if (threadIdx.x == 0) sc[rd.dst] = v;
    } else {
      double v = -INFINITY;
      for (int t = threadIdx.x; t < rd.count; t += 256)
        v = fmax(v, partials[rd.off + (size_t)t * rd.stride]);
      shm[threadIdx.x] = v;
      __syncthreads();
      if (threadIdx.x == 0) {
        double m = shm[0];
        for (int t = 1; t < 256; ++t) m = fmax(m, shm[t]);
        sc[rd.dst] = m;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x != 0 || stage == ST_NONE) return;
  int status = (int)sc[LNV_SC_STATUS];
  switch (stage) {
    case ST_EVAL: {
      const double E = 2.0 * (3.0 * sc[LNV_SC_T0] - 2.0 * sc[LNV_SC_T1]);
      const double N = 2.0 * (3.0 * sc[LNV_SC_T2] - 2.0 * sc[LNV_SC_T3]);
      sc[LNV_SC_E] = E;
      sc[LNV_SC_N] = N;
      const double FF = sc[LNV_SC_FF];
      sc[LNV_SC_MU] = FF != 0.0 ? sc[LNV_SC_GF] / FF : 0.0;
      sc[LNV_SC_FCFC] = FF;
      if (sa.en_out) {
        sa.en_out[0] = E;
        sa.en_out[1] = N;
      }
      if (!isfinite(E) || !isfinite(N) || !isfinite(sc[LNV_SC_MU])) status |= LNV_ST_NONFINITE;
      break;
    }
    case ST_MU: {
      // metric run: mu = <G, F_c> / <F, F_c>
      const double FF = sc[LNV_SC_FF];
      sc[LNV_SC_MU] = FF != 0.0 ? sc[LNV_SC_GF] / FF : 0.0;
      if (!isfinite(sc[LNV_SC_MU])) status |= LNV_ST_NONFINITE;
      break;
    }
    case ST_BETA: {
      // gg = <g, g_c>, ggp = <g, g_c_prev>, gprev = <g_prev, g_c_prev>
      const double gg = sc[LNV_SC_GG], ggp = sc[LNV_SC_GGP], gprev = sc[LNV_SC_GG_PREV];
      // runaway guard: two consecutive rises of E, or occupations of L S
      // outside [-0.5, 1.5], restart the direction (beta = 0); a second trip
      // within one reset period marks the run as running away
      {
        const double E = sc[LNV_SC_E], Ep = sc[LNV_SC_E_PREV];
        double rises = E > Ep + kRiseTol * fmax(1.0, fabs(Ep)) ? sc[LNV_SC_RISES] + 1.0 : 0.0;
        const bool occ_bad = sa.occ_checked &&
                             !(sc[LNV_SC_OCC_MIN] >= kOccLo && sc[LNV_SC_OCC_MAX] <= kOccHi);
        if (rises >= 2.0 || occ_bad) {
          if ((double)sa.k - sc[LNV_SC_GUARD_K] <= (double)sa.reset_period)
            status |= LNV_ST_RUNAWAY;
          status |= LNV_ST_GUARD;
          sc[LNV_SC_FORCE_RESET] = 1.0;
          sc[LNV_SC_GUARD_K] = (double)sa.k;
          rises = 0.0;
        }
        sc[LNV_SC_RISES] = rises;
        sc[LNV_SC_E_PREV] = E;
      }
      double beta = 0.0;
      if (!sa.reset && sc[LNV_SC_FORCE_RESET] == 0.0 && gprev != 0.0)
        beta = fmax(0.0, (gg - ggp) / gprev);
      sc[LNV_SC_BETA] = beta;
      sc[LNV_SC_FORCE_RESET] = 0.0;
      sc[LNV_SC_GNORM] = sqrt(sc[LNV_SC_GGN]);
      sc[LNV_SC_GG_PREV] = gg;
      break;
    }
    case ST_SIGMA: {
      // T[LNV_SC_T4] holds max_a sum_b |S_ab|
      const double m = sc[LNV_SC_T4];
      sc[LNV_SC_SIGMA] = m > 0.0 ? 1.0 / m : 0.0;
      if (!(m > 0.0) || !isfinite(m)) status |= LNV_ST_NONFINITE;
      break;
    }
    case ST_PROJ: {
      const double FF = sc[LNV_SC_FF];
      sc[LNV_SC_T5] = FF != 0.0 ? sc[LNV_SC_DF] / FF : 0.0;
      break;
    }
    case ST_ALPHA: {
      const double c1 = sc[LNV_SC_C1];
      const double c2 = 2.0 * (3.0 * sc[LNV_SC_T0] - 2.0 * (2.0 * sc[LNV_SC_T1] + sc[LNV_SC_T3]));
      const double c3 = -4.0 * sc[LNV_SC_T2];
      sc[LNV_SC_C2] = c2;
      sc[LNV_SC_C3] = c3;
      double a = 0.0;
      if (!cubic_min(c1, c2, c3, &a) || !isfinite(a)) {
        a = 0.0;
        sc[LNV_SC_FORCE_RESET] = 1.0;
        status |= LNV_ST_NO_ALPHA;
      }
      if (!isfinite(c1) || !isfinite(c2) || !isfinite(c3)) status |= LNV_ST_NONFINITE;
      sc[LNV_SC_ALPHA] = a;
      break;
    }
    case ST_NCHK: {
      const double N1 = 2.0 * (3.0 * sc[LNV_SC_T0] - 2.0 * sc[LNV_SC_T1]);
      sc[LNV_SC_N_AFTER] = N1;
      sc[LNV_SC_N0] = N1;
      sc[LNV_SC_N1] = sc[LNV_SC_T2];
      sc[LNV_SC_DELTA] = 0.0;
      sc[LNV_SC_SKIP_NCORR] = fabs(N1 - sa.n_elec) > sa.n_tol * sa.n_elec ? 0.0 : 1.0;
      if (!isfinite(N1)) status |= LNV_ST_NONFINITE;
      break;
    }
    case ST_DELTA: {
      if (sc[LNV_SC_SKIP_NCORR] != 0.0) break;
      sc[LNV_SC_NCORR] += 1.0;
      const double n2 = 2.0 * (3.0 * sc[LNV_SC_T0] - 2.0 * (2.0 * sc[LNV_SC_T1] + sc[LNV_SC_T3]));
      const double n3 = -4.0 * sc[LNV_SC_T2];
      sc[LNV_SC_N2] = n2;
      sc[LNV_SC_N3] = n3;
      double r[3];
      const int nr = real_roots(n3, n2, sc[LNV_SC_N1], sc[LNV_SC_N0] - sa.n_elec, r);
      double d = 0.0;
      if (nr == 0) {
        status |= LNV_ST_NO_DELTA;
      } else {
        d = r[0];
        for (int q = 1; q < nr; ++q)
          if (fabs(r[q]) < fabs(d)) d = r[q];
        if (!(fabs(d) * sqrt(sc[LNV_SC_FCFC]) <= sa.step_cap * sqrt(sc[LNV_SC_LL]))) {
          d = 0.0;
          status |= LNV_ST_DELTA_CAPPED;
        }
      }
      sc[LNV_SC_DELTA] = d;
      break;
    }
    case ST_INIT: {
      const double c2 = 6.0 * sc[LNV_SC_T0];
      const double c3 = -4.0 * sc[LNV_SC_T2];
      double r[3];
      const int nr = real_roots(c3, c2, 0.0, -sa.n_elec, r);
      double lam = 0.0;
      bool found = false;
      for (int q = 0; q < nr; ++q)
        if (r[q] > 0.0 && (!found || r[q] < lam)) {
          lam = r[q];
          found = true;
        }
      if (!found) status |= LNV_ST_NO_DELTA;
      sc[LNV_SC_LAMBDA] = lam;
      // a new minimisation: no previous energy, no guard trip yet
      sc[LNV_SC_E_PREV] = NAN;
      sc[LNV_SC_RISES] = 0.0;
      sc[LNV_SC_GUARD_K] = -1e9;
      break;
    }
    case ST_PM0: {
      // canonical purification start: mu = <T, H>/n, b = ||T||inf ||H||inf,
      // lambda = min(theta/(b - mu), (n - theta)/(mu + b));
      // K0 = ((lambda mu + theta)/n) T - (lambda/n) P_L(T H T)
      const double n = sa.pm_n, th = sa.pm_theta;
      const double mu = sc[LNV_PM_DOT] / n;
      const double b = sc[LNV_PM_NT] * sc[LNV_PM_NH];
      const double lam = fmin(th / (b - mu), (n - th) / (mu + b));
      sc[LNV_PM_MU] = mu;
      sc[LNV_PM_B] = b;
      sc[LNV_PM_LAMBDA] = lam;
      sc[LNV_PM_A0] = (lam * mu + th) / n;
      sc[LNV_PM_A1] = -lam / n;
      sc[LNV_PM_A2] = 0.0;
      sc[LNV_PM_HALF] = 0.5;
      sc[LNV_PM_PREV] = NAN;
      sc[LNV_PM_STOPPED] = 0.0;
      sc[LNV_PM_STEPS] = 0.0;
      return;
    }
    case ST_PM: {
      // one step: c = Tr[rho^2 - rho^3] / Tr[rho - rho^2] from t_p = Tr[rho^p];
      // stop (K kept) when Tr[rho - rho^2] <= tol theta, c is undefined or
      // outside [0, 1], or Tr[rho - rho^2] grew; else the coefficients of
      // K <- a0 K + a1 KSK + a2 KSKSK
      if (sc[LNV_PM_STOPPED] != 0.0) return;
      const int step = (int)sc[LNV_PM_STEPS];
      if (step >= sa.pm_hist_len) {
        sc[LNV_PM_STOPPED] = 1.0;
        if (sa.pm_batch) {
          sc[LNV_PM_A0] = 1.0;
          sc[LNV_PM_A1] = sc[LNV_PM_A2] = 0.0;
        }
        return;
      }
      const double t1 = sc[LNV_PM_T1], t2 = sc[LNV_PM_T2], t3 = sc[LNV_PM_T3];
      const double idem = t1 - t2;
      const double c = idem != 0.0 ? (t2 - t3) / idem : NAN;
      const double prev = sc[LNV_PM_PREV];
      const bool stop = idem <= sa.pm_tol * sa.pm_theta || idem == 0.0 || !(c >= 0.0 && c <= 1.0) ||
                        (!isnan(prev) && idem > prev);
      double* h = sa.pm_hist + 4 * (size_t)step;
      h[0] = stop ? NAN : c;
      h[1] = t1;
      h[2] = t2;
      h[3] = t3;
      sc[LNV_PM_STEPS] = (double)(step + 1);
      sc[LNV_PM_C] = c;
      if (stop) {
        sc[LNV_PM_STOPPED] = 1.0;
        if (sa.pm_batch) {
          // the cell's products still run with the others': keep K
          sc[LNV_PM_A0] = 1.0;
          sc[LNV_PM_A1] = sc[LNV_PM_A2] = 0.0;
        }
        return;
      }
      sc[LNV_PM_PREV] = idem;
      if (c >= 0.5) {
        sc[LNV_PM_A0] = 0.0;
        sc[LNV_PM_A1] = (1.0 + c) / c;
        sc[LNV_PM_A2] = -1.0 / c;
      } else {
        sc[LNV_PM_A0] = (1.0 - 2.0 * c) / (1.0 - c);
        sc[LNV_PM_A1] = (1.0 + c) / (1.0 - c);
        sc[LNV_PM_A2] = -1.0 / (1.0 - c);
      }
      return;
    }
    default:
      break;
  }
  sc[LNV_SC_STATUS] = (double)status;
}

// ------------------------------------------------------------------ per-item kernels
// Workgroup q handles item q of L's pattern: 64 blocks of one row, 4 threads
// per block, thread (b, r) owns row r of block b (4 elements).

// G, F and the trace partials of one evaluation.  The intermediates are of
// type T (FP64, or FP32 in the mixed-precision evaluation); G, F, L and every
// trace are FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_assemble(
    int n, int n_items, const int* __restrict__ items, const int* __restrict__ rp,
    const int* __restrict__ col, Ix lx,
    const double* __restrict__ L, Ix xx,
    const T* __restrict__ X, Ix xtx,
    const T* __restrict__ XT, const T* __restrict__ YT,
    const T* __restrict__ Wv, Ix zx,
    const T* __restrict__ Z, const T* __restrict__ V, double* __restrict__ G,
    double* __restrict__ F, double* __restrict__ partials, int zhalf) {
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rp[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (b < cnt) {
    const int p = c0 + b;
    const int j = col[p];
    const int xp = ix_find(xx, i, j);
    // X^T_ij: stored, or block (j, i) of X transposed
    const int xtp = XT ? ix_find(xtx, i, j) : ix_find(xx, j, i);
    const T* __restrict__ xtv = XT ? XT : X;
    const int ytp = ix_find(lx, j, i);
    // zhalf: Z holds the blocks of its half (in_half) only, Z_ij = Z_ji^T
    const bool zt = zhalf && !in_half(n, i, j);
    const int zp = zt ? ix_find(zx, j, i) : ix_find(zx, i, j);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int e = r * 4 + c, et = c * 4 + r;
      const double x = xp >= 0 ? (double)X[(size_t)xp * 16 + e] : 0.0;
      const double xt = xtp >= 0 ? (double)xtv[(size_t)xtp * 16 + (XT ? e : et)] : 0.0;
      const double yt = (double)YT[(size_t)p * 16 + e];
      const double ytt = ytp >= 0 ? (double)YT[(size_t)ytp * 16 + et] : 0.0;
      const double w = (double)Wv[(size_t)p * 16 + e];
      const double z = zp >= 0 ? (double)Z[(size_t)zp * 16 + (zt ? et : e)] : 0.0;
      const double v = (double)V[(size_t)p * 16 + e];
      const double l = L[(size_t)p * 16 + e];
      const double g = 2.0 * (3.0 * (x + xt) - 2.0 * (yt + ytt + w));
      const double f = 12.0 * (z - v);
      G[(size_t)p * 16 + e] = g;
      F[(size_t)p * 16 + e] = f;
      s[0] = fma(l, x, s[0]);
      s[1] = fma(l, yt, s[1]);
      s[2] = fma(l, z, s[2]);
      s[3] = fma(l, v, s[3]);
      s[4] = fma(f, f, s[4]);
      s[5] = fma(g, f, s[5]);
    }
  }
  // the six partials in one exchange: wave sums, then the four waves' sums
  // added in wave order by one thread each (block_sum's order, one barrier
  // instead of twelve)
  __shared__ double sh6[6][4];
#pragma unroll
  for (int c = 0; c < 6; ++c) s[c] = wave_sum(s[c]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < 6; ++c) sh6[c][threadIdx.x >> 6] = s[c];
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int c = threadIdx.x;
    double t = 0.0;
    for (int q = 0; q < 4; ++q) t += sh6[c][q];
    partials[(size_t)c * n_items + item] = t;
  }
}

// Electron number at the current L: partials <L,Z>, <L,V>, <12(Z-V), F>, <L,L>.
__global__ __launch_bounds__(256) void k_nassemble(
    int n, int n_items, const int* __restrict__ items, const int* __restrict__ rp,
    const int* __restrict__ col, const double* __restrict__ L, Ix zx,
    const double* __restrict__ Z, const double* __restrict__ V,
    const double* __restrict__ Fc, double* __restrict__ partials) {
  __shared__ double sh[16];
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rp[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  double s[4] = {0, 0, 0, 0};
  if (b < cnt) {
    const int p = c0 + b;
    const int j = col[p];
    const int zp = ix_find(zx, i, j);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int e = r * 4 + c;
      const double z = zp >= 0 ? Z[(size_t)zp * 16 + e] : 0.0;
      const double v = V[(size_t)p * 16 + e];
      const double l = L[(size_t)p * 16 + e];
      const double f1 = 12.0 * (z - v);
      s[0] = fma(l, z, s[0]);
      s[1] = fma(l, v, s[1]);
      s[2] = fma(f1, Fc[(size_t)p * 16 + e], s[2]);
      s[3] = fma(l, l, s[3]);
    }
  }
  for (int c = 0; c < 4; ++c) {
    const double t = block_sum(s[c], sh);
    if (threadIdx.x == 0) partials[(size_t)c * n_items + item] = t;
  }
}

// B on its own pattern from A on another pattern of the same atoms: blocks
// present in both are copied, the others set to zero.  Workgroup per row of
// B, 16 threads per block.
__global__ __launch_bounds__(256) void k_remap(int n, const int* __restrict__ b_rp,
                                               const int* __restrict__ b_col,
                                               Ix ax, const double* __restrict__ A,
                                               double* __restrict__ B) {
  const int i = blockIdx.x;
  const int e = threadIdx.x & 15;
  for (int p = b_rp[i] + (threadIdx.x >> 4); p < b_rp[i + 1]; p += 16) {
    const int q = ix_find(ax, i, b_col[p]);
    B[(size_t)p * 16 + e] = q >= 0 ? A[(size_t)q * 16 + e] : 0.0;
  }
}

// Full symmetric matrix F from the blocks U of its half (in_half): F_ij =
// U_ij when only (i, j) is in the half, U_ji^T when only (j, i) is, and
// (U_ij + U_ji^T)/2 when both are (i and j in one row group, the diagonal
// included), so F is exactly symmetric; U's blocks are found through U's own
// index.  Workgroup per item of F, 4 threads per block (thread r writes row r).
template <typename T>
__global__ __launch_bounds__(256) void k_mirror(int n, const int* __restrict__ items,
                                                const int* __restrict__ rpF,
                                                const int* __restrict__ colF, Ix ux,
                                                const T* __restrict__ U, T* __restrict__ F,
                                                const double* __restrict__ skip) {
  if (skip != nullptr && *skip != 0.0) return;
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rpF[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  if (b >= cnt) return;
  const int p = c0 + b;
  const int j = colF[p];
  if (same_group(n, i, j)) {  // both in the half: the symmetric part of the pair
    const int q = ix_find(ux, i, j), qt = ix_find(ux, j, i);
    if (q < 0 || qt < 0) {  // F's pattern not symmetric: poison the block
#pragma unroll
      for (int c = 0; c < 4; ++c) F[(size_t)p * 16 + r * 4 + c] = T(NAN);
      return;
    }
    const T* u = U + (size_t)q * 16;
    const T* ut = U + (size_t)qt * 16;
#pragma unroll
    for (int c = 0; c < 4; ++c)
      F[(size_t)p * 16 + r * 4 + c] = T(0.5) * (u[r * 4 + c] + ut[c * 4 + r]);
    return;
  }
  const bool tr = !in_half(n, i, j);
  const int q = tr ? ix_find(ux, j, i) : ix_find(ux, i, j);
  if (q < 0) {  // F's pattern not symmetric: poison the block
#pragma unroll
    for (int c = 0; c < 4; ++c) F[(size_t)p * 16 + r * 4 + c] = T(NAN);
    return;
  }
  const T* u = U + (size_t)q * 16;
#pragma unroll
  for (int c = 0; c < 4; ++c) F[(size_t)p * 16 + r * 4 + c] = tr ? u[c * 4 + r] : u[r * 4 + c];
}

// Weighted halves of two matrices on L's (symmetric) pattern: for every block
// (i, j) of the half in_half, at position q of U's pattern, dst[q] = w src[p]
// with p its position in the full pattern and w = 1 when (j, i) is in the
// half too (i and j in one row group), 2 otherwise.  For symmetric X and a
// symmetric product Q formed only on the half, sum over the half of
// <dst_q, Q_q> is the full <X, Q>: the blocks left out are the transposes of
// those kept.
__global__ __launch_bounds__(256) void k_half_weighted(int n, const int* __restrict__ items,
                                                       const int* __restrict__ rpF,
                                                       const int* __restrict__ colF, Ix ux,
                                                       const double* __restrict__ src1,
                                                       const double* __restrict__ src2,
                                                       double* __restrict__ dst1,
                                                       double* __restrict__ dst2,
                                                       const double* __restrict__ skip) {
  if (skip != nullptr && *skip != 0.0) return;
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rpF[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  if (b >= cnt) return;
  const int p = c0 + b;
  const int j = colF[p];
  if (!in_half(n, i, j)) return;
  const int q = ix_find(ux, i, j);
  if (q < 0) return;  // U's pattern misses a block of the half: checked on the host
  const double w = same_group(n, i, j) ? 1.0 : 2.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const size_t e = (size_t)r * 4 + c;
    dst1[(size_t)q * 16 + e] = w * src1[(size_t)p * 16 + e];
    dst2[(size_t)q * 16 + e] = w * src2[(size_t)p * 16 + e];
  }
}

// out = a X + b Y + c Z elementwise (Y, Z nullable), grid-stride.
__global__ __launch_bounds__(256) void k_lincomb(int64_t nv, double a, const double* __restrict__ X,
                                                 double b, const double* __restrict__ Y, double c,
                                                 const double* __restrict__ Z,
                                                 double* __restrict__ out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nv;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = a * X[e];
    if (Y) v = fma(b, Y[e], v);
    if (Z) v = fma(c, Z[e], v);
    out[e] = v;
  }
}

// Per-cell energy and electron number of a batch of independent cells from
// the trace partials k_assemble leaves (slots 0..3 = <L,X>, <L,Y>, <L,Z>,
// <L,V> per item of L's pattern): workgroup c sums the items of cell c,
// items cell_item_ptr[c] .. cell_item_ptr[c+1]-1, in a fixed order.
__global__ __launch_bounds__(256) void k_cell_traces(const double* __restrict__ partials,
                                                     int n_items,
                                                     const int* __restrict__ cell_item_ptr,
                                                     double* __restrict__ en) {
  __shared__ double sh[16];
  const int c = blockIdx.x;
  const int q0 = cell_item_ptr[c], q1 = cell_item_ptr[c + 1];
  double t[4];
  for (int k = 0; k < 4; ++k) {
    double v = 0.0;
    for (int q = q0 + threadIdx.x; q < q1; q += blockDim.x) v += partials[(size_t)k * n_items + q];
    t[k] = block_sum(v, sh);
  }
  if (threadIdx.x == 0) {
    en[2 * c] = 2.0 * (3.0 * t[0] - 2.0 * t[1]);
    en[2 * c + 1] = 2.0 * (3.0 * t[2] - 2.0 * t[3]);
  }
}

// <A, B> with B located through B's index table (or at A's positions).
__global__ __launch_bounds__(256) void k_dot_items(
    int n, int n_items, const int* __restrict__ items, const int* __restrict__ rp,
    const int* __restrict__ col, const double* __restrict__ A, Ix bx, int same,
    const double* __restrict__ B, double* __restrict__ partials,
    const double* __restrict__ skip) {
  __shared__ double sh[16];
  if (skip != nullptr && *skip != 0.0) return;
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  double s = 0.0;
  for (int item = blockIdx.x; item < n_items; item += gridDim.x) {
    const int i = items[2 * item], c0 = items[2 * item + 1];
    const int cnt = min(kWave, rp[i + 1] - c0);
    if (b < cnt) {
      const int p = c0 + b;
      const int q = same ? p : ix_find(bx, i, col[p]);
      if (q >= 0)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          s = fma(A[(size_t)p * 16 + r * 4 + c], B[(size_t)q * 16 + r * 4 + c], s);
    }
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// H' = H - mu S on H's pattern (S located through its index table).
__global__ __launch_bounds__(256) void k_hprime(int n, const int* __restrict__ items,
                                                const int* __restrict__ rp,
                                                const int* __restrict__ col,
                                                const double* __restrict__ H, Ix sx,
                                                const double* __restrict__ S,
                                                const double* __restrict__ sc,
                                                double* __restrict__ Hp, Seg sg) {
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rp[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  if (b >= cnt) return;
  const double mu = sc[(sg.n > 0 ? (size_t)sg.row_cell[i] * sg.sc_stride : 0) + LNV_SC_MU];
  const int p = c0 + b;
  const int q = ix_find(sx, i, col[p]);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int e = r * 4 + c;
    const double sv = q >= 0 ? S[(size_t)q * 16 + e] : 0.0;
    Hp[(size_t)p * 16 + e] = H[(size_t)p * 16 + e] - mu * sv;
  }
}

// v * I on the diagonal of L's pattern, zero elsewhere.  The identity is that
// of the orbitals present: a diagonal entry whose S_aa is zero (a padded
// row of an atom split over several stored rows) stays zero, so the
// minimisation never moves such rows.  v = sc[idx] (sc == nullptr: 1).
__global__ __launch_bounds__(256) void k_identity(int n, const int* __restrict__ items,
                                                  const int* __restrict__ rp,
                                                  const int* __restrict__ col, Ix sx,
                                                  const double* __restrict__ S,
                                                  const double* __restrict__ sc, int idx,
                                                  double* __restrict__ D, Seg sg) {
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rp[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  if (b >= cnt) return;
  const int p = c0 + b;
  const bool diag = col[p] == i;
  const double v = sc ? sc[(sg.n > 0 ? (size_t)sg.row_cell[i] * sg.sc_stride : 0) + idx] : 1.0;
  bool present = false;
  if (diag) {
    const int q = ix_find(sx, i, i);
    present = q >= 0 && S[(size_t)q * 16 + r * 5] != 0.0;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
    D[(size_t)p * 16 + r * 4 + c] = (present && r == c) ? v : 0.0;
}

// AT[perm[p]] = A[p]^T for the blocks of item q of A's pattern.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const int* __restrict__ items,
                                                   const int* __restrict__ rp,
                                                   const int* __restrict__ perm,
                                                   const T* __restrict__ A,
                                                   T* __restrict__ AT,
                                                   const double* __restrict__ skip) {
  if (skip != nullptr && *skip != 0.0) return;
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rp[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  if (b >= cnt) return;
  const int p = c0 + b;
  const size_t q = (size_t)perm[p];
  const T* a = A + (size_t)p * 16 + r * 4;
  const T v0 = a[0], v1 = a[1], v2 = a[2], v3 = a[3];
  AT[q * 16 + 0 * 4 + r] = v0;
  AT[q * 16 + 1 * 4 + r] = v1;
  AT[q * 16 + 2 * 4 + r] = v2;
  AT[q * 16 + 3 * 4 + r] = v3;
}

// Elementwise dtype conversion of a value array (grid-stride).
template <typename S, typename D>
__global__ __launch_bounds__(256) void k_convert(int64_t nv, const S* __restrict__ src,
                                                 D* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nv;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = (D)src[e];
}

// ------------------------------------------------------------------ vector kernels
// Fixed grid of kVecGrid workgroups, grid-stride over the nv values of L's
// pattern; partial q of component c goes to partials[c * kVecGrid + q].  A
// batch (Seg) gives cell c the workgroups c * per .. c * per + per - 1, which
// stride over the cell's values with the cell's scalars.

// This workgroup's value range, stride and scalars.
struct VecRange {
  int64_t lo, hi, start, step;
  const double* sc;
};

__device__ __forceinline__ VecRange vec_range(int64_t nv, const double* sc, const Seg& sg) {
  if (sg.n > 0) {
    const int c = blockIdx.x / sg.per, q = blockIdx.x % sg.per;
    const int64_t lo = sg.val_ptr[c];
    return VecRange{lo, sg.val_ptr[c + 1], lo + (int64_t)q * 256 + threadIdx.x,
                    (int64_t)sg.per * 256, sc ? sc + (size_t)c * sg.sc_stride : nullptr};
  }
  return VecRange{0, nv, (int64_t)blockIdx.x * 256 + threadIdx.x, (int64_t)gridDim.x * 256, sc};
}

// g = G - mu F and (metric runs) g_c = G_c - mu F_c;
// partials <g, g_c>, <g, g_c_prev>, <g, g>
__global__ __launch_bounds__(256) void k_vec_g(int64_t nv, const double* __restrict__ G,
                                               const double* __restrict__ F,
                                               const double* __restrict__ Gc,
                                               const double* __restrict__ Fc,
                                               const double* __restrict__ gcprev,
                                               const double* __restrict__ sc,
                                               double* __restrict__ g, double* __restrict__ gc,
                                               double* __restrict__ partials, Seg sg) {
  __shared__ double sh[16];
  const VecRange vr = vec_range(nv, sc, sg);
  const double mu = vr.sc[LNV_SC_MU];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t q = vr.start; q < vr.hi; q += vr.step) {
    const double v = G[q] - mu * F[q];
    g[q] = v;
    double vc = v;
    if (gc) {
      vc = Gc[q] - mu * Fc[q];
      gc[q] = vc;
    }
    s0 = fma(v, vc, s0);
    s1 = fma(v, gcprev[q], s1);
    s2 = fma(v, v, s2);
  }
  double t = block_sum(s0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
  t = block_sum(s1, sh);
  if (threadIdx.x == 0) partials[kVecGrid + blockIdx.x] = t;
  t = block_sum(s2, sh);
  if (threadIdx.x == 0) partials[2 * kVecGrid + blockIdx.x] = t;
}

// metric traces: <F, F_c>, <G, F_c>, <F_c, F_c>
__global__ __launch_bounds__(256) void k_vec_metric_dots(int64_t nv, const double* __restrict__ G,
                                                         const double* __restrict__ F,
                                                         const double* __restrict__ Fc,
                                                         double* __restrict__ partials, Seg sg) {
  __shared__ double sh[16];
  const VecRange vr = vec_range(nv, nullptr, sg);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t q = vr.start; q < vr.hi; q += vr.step) {
    const double fc = Fc[q];
    s0 = fma(F[q], fc, s0);
    s1 = fma(G[q], fc, s1);
    s2 = fma(fc, fc, s2);
  }
  double t = block_sum(s0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
  t = block_sum(s1, sh);
  if (threadIdx.x == 0) partials[kVecGrid + blockIdx.x] = t;
  t = block_sum(s2, sh);
  if (threadIdx.x == 0) partials[2 * kVecGrid + blockIdx.x] = t;
}

// max over orbital rows a of sum_b |S_ab|: one workgroup per atom row,
// thread (b, r) adds row r of blocks b, b+64, ...
__global__ __launch_bounds__(256) void k_rowabs(const int* __restrict__ rp,
                                                const double* __restrict__ S,
                                                double* __restrict__ partials) {
  __shared__ double sh[256];
  const int i = blockIdx.x;
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  double v = 0.0;
  for (int p = rp[i] + b; p < rp[i + 1]; p += 64)
#pragma unroll
    for (int c = 0; c < 4; ++c) v += fabs(S[(size_t)p * 16 + r * 4 + c]);
  sh[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int q = threadIdx.x; q < 256; q += 4) t += sh[q];
    sh[threadIdx.x] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) partials[i] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// sc[idx] * I on the diagonal blocks of a pattern

// D = -g_c + beta D_prev; partial <D, F>
__global__ __launch_bounds__(256) void k_vec_dir(int64_t nv, const double* __restrict__ g,
                                                 const double* __restrict__ Dprev,
                                                 const double* __restrict__ F,
                                                 const double* __restrict__ sc,
                                                 double* __restrict__ D,
                                                 double* __restrict__ partials, Seg sg) {
  __shared__ double sh[16];
  const VecRange vr = vec_range(nv, sc, sg);
  const double beta = vr.sc[LNV_SC_BETA];
  double s0 = 0.0;
  for (int64_t q = vr.start; q < vr.hi; q += vr.step) {
    const double v = beta != 0.0 ? -g[q] + beta * Dprev[q] : -g[q];
    D[q] = v;
    s0 = fma(v, F[q], s0);
  }
  const double t = block_sum(s0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// D <- D - coef F; partial <g, D>
__global__ __launch_bounds__(256) void k_vec_proj(int64_t nv, const double* __restrict__ F,
                                                  const double* __restrict__ g,
                                                  const double* __restrict__ sc,
                                                  double* __restrict__ D,
                                                  double* __restrict__ partials, Seg sg) {
  __shared__ double sh[16];
  const VecRange vr = vec_range(nv, sc, sg);
  const double coef = vr.sc[LNV_SC_T5];
  double s0 = 0.0;
  for (int64_t q = vr.start; q < vr.hi; q += vr.step) {
    const double v = D[q] - coef * F[q];
    D[q] = v;
    s0 = fma(g[q], v, s0);
  }
  const double t = block_sum(s0, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// L += sc[idx] * D (skipped when skip != null and *skip != 0)
__global__ __launch_bounds__(256) void k_vec_axpy(int64_t nv, const double* __restrict__ D,
                                                  const double* __restrict__ sc, int idx,
                                                  const double* __restrict__ skip,
                                                  double* __restrict__ L, Seg sg) {
  if (skip != nullptr && *skip != 0.0) return;
  const VecRange vr = vec_range(nv, sc, sg);
  const double a = vr.sc[idx];
  if (a == 0.0) return;
  for (int64_t q = vr.start; q < vr.hi; q += vr.step) L[q] = L[q] + a * D[q];
}

// out = sc[i0] X + sc[i1] Y + sc[i2] Z (Y, Z nullable; out may alias), the
// association of k_lincomb, per cell of a batch with the cell's scalars;
// skipped when *skip != 0.
__global__ __launch_bounds__(256) void k_lincomb_sc(int64_t nv, const double* __restrict__ sc,
                                                    int i0, int i1, int i2,
                                                    const double* X, const double* Y,
                                                    const double* Z, double* out,
                                                    const double* __restrict__ skip, Seg sg) {
  if (skip != nullptr && *skip != 0.0) return;
  const VecRange vr = vec_range(nv, sc, sg);
  const double a = vr.sc[i0], b = Y ? vr.sc[i1] : 0.0, c = Z ? vr.sc[i2] : 0.0;
  for (int64_t e = vr.start; e < vr.hi; e += vr.step) {
    double v = a * X[e];
    if (Y) v = fma(b, Y[e], v);
    if (Z) v = fma(c, Z[e], v);
    out[e] = v;
  }
}

// Zero the scalar block of each cell (blockIdx.x) except entry keep.
__global__ __launch_bounds__(64) void k_clear_scalars(double* __restrict__ sc, int stride,
                                                      int keep) {
  double* c = sc + (size_t)blockIdx.x * stride;
  for (int q = threadIdx.x; q < stride; q += blockDim.x)
    if (q != keep) c[q] = 0.0;
}

// Y = X + sc[idx] * Y
__global__ __launch_bounds__(256) void k_vec_xpay(int64_t nv, const double* __restrict__ X,
                                                  const double* __restrict__ sc, int idx,
                                                  double* __restrict__ Y) {
  const double a = sc[idx];
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < nv; q += (int64_t)gridDim.x * 256)
    Y[q] = fma(a, Y[q], X[q]);
}

// ------------------------------------------------------------------ host helpers
// n_items_L: the larger of L's n_items and n_cl_items
int64_t slot_len(int n_items_L) {
  const int64_t a = 8 * (int64_t)n_items_L, b = 8 * (int64_t)kVecGrid;
  return a > b ? a : b;
}

int scalar_stage(const double* partials, const RedList& rl, double* sc, int stage,
                 const StageArgs& sa, hipStream_t s, const Seg& sg = Seg{}) {
  k_scalar<<<sg.n > 0 ? sg.n : 1, 256, 0, s>>>(partials, rl, sc, stage, sa, sg);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

RedList reds() {
  RedList r{};
  r.nr = 0;
  return r;
}
void add(RedList& rl, int64_t off, int count, int stride, int dst, int op = 0,
         int kind = RK_ALL) {
  rl.r[rl.nr++] = Red{(int)off, count, stride, dst, op, kind};
}

// Validation of a batch descriptor against L's pattern (host side; the
// device tables themselves are the caller's).
int check_batch(const lnv_batch* b, const lnv_pattern* pl) {
  if (!b || b->n_cells < 1 || !b->item_ptr || !b->val_ptr || !b->row_cell || !b->n_elec ||
      !b->scalars || !b->row_off || !b->n_orb)
    return LNV_EINVAL;
  if (b->n_cells > pl->n) return LNV_EPATTERN;
  if (b->n_cells > kVecGrid) return LNV_EUNSUPPORTED;   // one vector workgroup per cell at least
  return LNV_OK;
}

Seg make_seg(const lnv_batch* b) {
  Seg sg;
  sg.n = b->n_cells;
  sg.per = kVecGrid / b->n_cells;
  sg.item_ptr = b->item_ptr;
  sg.val_ptr = b->val_ptr;
  sg.row_cell = b->row_cell;
  sg.n_elec = b->n_elec;
  sg.row_off = b->row_off;
  sg.n_orb = b->n_orb;
  return sg;
}

// Vector-kernel grid of a batch (cell c: workgroups c * per ...).
int seg_grid(const Seg& sg) { return sg.n > 0 ? sg.n * sg.per : kVecGrid; }

// ix: the pattern must carry its spatial index (for lookups in either
// orientation); items: its row work list.
bool pattern_ready(const lnv_pattern* p, bool ix, bool ix_t, bool items) {
  return p && p->row_ptr && p->col && (!(ix || ix_t) || has_ix(p)) && (!items || p->items);
}

// AT: values of A's dtype.
int transpose_skip_launch(const lnv_bsm* A, const int32_t* perm, void* AT,
                          const double* skip, hipStream_t s) {
  const lnv_pattern* pa = A->pat;
  if (pa->n_items == 0) return LNV_OK;
  if (A->dtype == LNV_F32)
    k_transpose<float><<<pa->n_items, 256, 0, s>>>(pa->items, pa->row_ptr, perm,
                                                   static_cast<const float*>(A->val),
                                                   static_cast<float*>(AT), skip);
  else
    k_transpose<double><<<pa->n_items, 256, 0, s>>>(pa->items, pa->row_ptr, perm,
                                                    static_cast<const double*>(A->val),
                                                    static_cast<double*>(AT), skip);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

int transpose_launch(const lnv_bsm* A, const int32_t* perm, void* AT, hipStream_t s) {
  return transpose_skip_launch(A, perm, AT, nullptr, s);
}

// The intermediates' transposes L.S and X^T are optional as a pair (both
// values NULL): the products then read S.L and X transposed.
bool lean_ws(const lnv_bsm& LS, const lnv_bsm& XT) { return !LS.val && !XT.val; }

// Checks of an evaluation's patterns and intermediates (FP64 or FP32 values,
// per the caller's ok test).
template <typename Ok>
int check_products(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm& SL,
                   const lnv_bsm& LS, const lnv_bsm& X, const lnv_bsm& XT, const lnv_bsm& Z,
                   const int32_t* perm_SL, const int32_t* perm_X, Ok ok) {
  const bool lean = lean_ws(LS, XT);
  if (!ok(&SL) || !ok(&X) || !ok(&Z)) return LNV_EINVAL;
  if (!lean && (!ok(&LS) || !ok(&XT) || !perm_SL || !perm_X)) return LNV_EINVAL;
  const int n = L->pat->n;
  if (S->pat->n != n || H->pat->n != n || SL.pat->n != n || X.pat->n != n || Z.pat->n != n)
    return LNV_EPATTERN;
  if (!lean && (LS.pat->n != n || XT.pat->n != n || SL.pat->nnzb != LS.pat->nnzb ||
                X.pat->nnzb != XT.pat->nnzb))
    return LNV_EPATTERN;
  if (!pattern_ready(L->pat, true, false, true) || !pattern_ready(S->pat, false, false, false) ||
      !pattern_ready(H->pat, false, false, false) || !pattern_ready(SL.pat, lean, false, true) ||
      !pattern_ready(X.pat, true, false, true) || !pattern_ready(Z.pat, true, false, true))
    return LNV_EPATTERN;
  if (!lean && (!pattern_ready(LS.pat, true, false, false) ||
                !pattern_ready(XT.pat, true, false, false)))
    return LNV_EPATTERN;
  return LNV_OK;
}

int check_eval(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm* G,
               const lnv_bsm* F, const lnv_eval_ws* ws) {
  if (!bsm_ok(L) || !bsm_ok(S) || !bsm_ok(H) || !ws || !ws->YT || !ws->W || !ws->V ||
      !ws->partials || !ws->scalars)
    return LNV_EINVAL;
  if ((G && !bsm_ok(G)) || (F && !bsm_ok(F))) return LNV_EINVAL;
  if (L->blk != 4 || S->blk != 4 || H->blk != 4) return LNV_EUNSUPPORTED;
  LNV_TRY(check_products(L, S, H, ws->SL, ws->LS, ws->X, ws->XT, ws->Z, ws->perm_SL, ws->perm_X,
                         [](const lnv_bsm* m) { return bsm_ok(m); }));
  if (G && G->pat != L->pat) return LNV_EPATTERN;
  if (F && F->pat != L->pat) return LNV_EPATTERN;
  if (ws->partials_len < lnv_partials_len(partial_items(L->pat))) return LNV_EINVAL;
  return LNV_OK;
}

// Operands and intermediates of one evaluation, all of one dtype T.
// Zu / Lu (val != NULL): half patterns (in_half) for the symmetric products.
struct EvalOps {
  const lnv_bsm *L, *S, *H;
  const lnv_bsm *SL, *LS, *X, *XT, *Z;
  const int32_t *perm_SL, *perm_X;
  void *YT, *W, *V;
  double* partials;
  double* scalars;
  const lnv_bsm *Zu, *Lu;
  void* Vu;
  const void* SLcarry;   // S.L already formed for this L (copied instead of multiplied)
  bool Zcarry;           // Z = S.L.S already in Z for this L (not formed again)
};

}  // namespace

int transpose_values(const lnv_bsm* A, const int32_t* perm, void* AT, hipStream_t s) {
  return transpose_launch(A, perm, AT, s);
}

bool sym_ready(const lnv_bsm* U, const lnv_bsm* C) {
  return U && U->val && U->pat && U->pat->n == C->pat->n && U->pat->items && U->pat->row_ptr &&
         has_ix(U->pat) && U->dtype == C->dtype && C->pat->items;
}

// C (full symmetric pattern) from the blocks U of its half (skip: as in
// the multiply, a device flag that turns the launch into a no-op).
int mirror_launch(const lnv_bsm* U, const lnv_bsm* C, hipStream_t s, const double* skip) {
  const lnv_pattern *pf = C->pat, *pu = U->pat;
  if (pf->n_items == 0) return LNV_OK;
  if (C->dtype == LNV_F32)
    k_mirror<float><<<pf->n_items, 256, 0, s>>>(pf->n, pf->items, pf->row_ptr, pf->col, make_ix(pu),
                                                static_cast<const float*>(U->val),
                                                static_cast<float*>(C->val), skip);
  else
    k_mirror<double><<<pf->n_items, 256, 0, s>>>(pf->n, pf->items, pf->row_ptr, pf->col, make_ix(pu),
                                                 static_cast<const double*>(U->val),
                                                 static_cast<double*>(C->val), skip);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

namespace {

// C = A.B on C's (symmetric) pattern for a product known to be symmetric.
// With a half buffer U (sym_ready) only the blocks of the half in_half are
// multiplied, into U, and C is filled from them by a transposing copy;
// otherwise C is formed in full.
int sym_product(const lnv_bsm* A, const lnv_bsm* B, const lnv_bsm* C, const lnv_bsm* U,
                hipStream_t s, int transB = 0) {
  if (!sym_ready(U, C))
    return multiply_launch(1.0, A, B, transB, 0.0, C, 1, nullptr, nullptr, nullptr, nullptr, s);
  LNV_TRY(multiply_launch(1.0, A, B, transB, 0.0, U, 1, nullptr, nullptr, nullptr, nullptr, s));
  return mirror_launch(U, C, s);
}

// Two symmetric products C1 = A1.B1, C2 = A2.B2 with the same output pattern
// (halves U1, U2 on one pattern): one paired launch, then the mirrors.
int sym_product_pair(const lnv_bsm* A1, const lnv_bsm* B1, const lnv_bsm* C1, const lnv_bsm* U1,
                     const lnv_bsm* A2, const lnv_bsm* B2, const lnv_bsm* C2, const lnv_bsm* U2,
                     hipStream_t s) {
  if (!sym_ready(U1, C1) || !sym_ready(U2, C2) || U1->pat != U2->pat) {
    LNV_TRY(sym_product(A1, B1, C1, U1, s));
    return sym_product(A2, B2, C2, U2, s);
  }
  LNV_TRY(multiply_pair_launch(A1, B1, U1, A2, B2, U2, 1, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, s));
  LNV_TRY(mirror_launch(U1, C1, s));
  return mirror_launch(U2, C2, s);
}

// The six products (in T), the assembly of G and F and the energy / electron
// traces (FP64, with the FP64 L64 on the left of every trace).
template <typename T>
int eval_products(const lnv_bsm* L64, const EvalOps& o, double* G, double* F, double* EN,
                  hipStream_t s, const Seg& sg = Seg{}) {
  const lnv_pattern* pl = L64->pat;
  const int dt = o.SL->dtype;
  lnv_bsm YT{pl, 4, dt, o.YT}, Wm{pl, 4, dt, o.W}, Vm{pl, 4, dt, o.V};
  if (o.SLcarry) {
    const size_t bytes = (size_t)o.SL->pat->nnzb * 16 * sizeof(T);
    LNV_HIP(hipMemcpyAsync(o.SL->val, o.SLcarry, bytes, hipMemcpyDeviceToDevice, s));
  } else {
    LNV_TRY(multiply_launch(1.0, o.S, o.L, 0, 0.0, o.SL, 1, nullptr, nullptr, nullptr, nullptr,
                            s));
  }
  // L.S and X^T stored (read in their own orientation), or, without them,
  // read transposed from S.L and X
  const bool lean = lean_ws(*o.LS, *o.XT);
  const lnv_bsm* LSop = lean ? o.SL : o.LS;
  const lnv_bsm* XTop = lean ? o.X : o.XT;
  const int tb = lean ? 1 : 0;
  if (!lean) LNV_TRY(transpose_launch(o.SL, o.perm_SL, o.LS->val, s));
  LNV_TRY(multiply_launch(1.0, o.H, LSop, tb, 0.0, o.X, 1, nullptr, nullptr, nullptr, nullptr,
                          s));
  // Z = SLS, W = P_L(SLHLS) and V = P_L(SLSLS) are symmetric (formed on
  // their halves when the workspace carries them); YT = P_L(SLSLH) is not
  const lnv_bsm* Lu = o.Lu;
  lnv_bsm Vu{Lu ? Lu->pat : nullptr, 4, dt, o.Vu};
  // on the atom tiles, Z formed afresh stays on its half: V reads it there
  // (transB = 2) and so does the assembly, and Z is never filled in full
  const bool zhalf = lean && !o.Zcarry && Lu && o.Vu && sym_ready(o.Zu, o.Z) &&
                     sym_ready(&Vu, &Vm) && half_b_ok(o.SL, o.Zu, &Vu);
  if (zhalf)
    LNV_TRY(multiply_launch(1.0, o.S, LSop, tb, 0.0, o.Zu, 1, nullptr, nullptr, nullptr, nullptr,
                            s));
  else if (!o.Zcarry)
    LNV_TRY(sym_product(o.S, LSop, o.Z, o.Zu, s, tb));
  if (!lean) LNV_TRY(transpose_launch(o.X, o.perm_X, o.XT->val, s));
  LNV_TRY(multiply_launch(1.0, o.SL, XTop, tb, 0.0, &YT, 1, nullptr, nullptr, nullptr, nullptr,
                          s));
  if (zhalf) {
    LNV_TRY(sym_product(o.SL, o.X, &Wm, Lu, s));
    LNV_TRY(sym_product(o.SL, o.Zu, &Vm, &Vu, s, 2));
  } else {
    LNV_TRY(sym_product_pair(o.SL, o.X, &Wm, Lu, o.SL, o.Z, &Vm, Lu ? &Vu : nullptr, s));
  }
  const lnv_bsm* Zr = zhalf ? o.Zu : o.Z;
  const int ni = pl->n_items;
  double* part = o.partials;
  k_assemble<T><<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, make_ix(pl),
                                   static_cast<const double*>(L64->val), make_ix(o.X->pat),
                                   static_cast<const T*>(o.X->val),
                                   lean ? make_ix(o.X->pat) : make_ix(o.XT->pat),
                                   lean ? nullptr : static_cast<const T*>(o.XT->val),
                                   static_cast<const T*>(o.YT), static_cast<const T*>(o.W),
                                   make_ix(Zr->pat), static_cast<const T*>(Zr->val),
                                   static_cast<const T*>(o.V), G, F, part, zhalf ? 1 : 0);
  LNV_LAUNCH_CHECK();
  RedList rl = reds();
  add(rl, 0 * (int64_t)ni, ni, 1, LNV_SC_T0, 0, RK_ITEMS);
  add(rl, 1 * (int64_t)ni, ni, 1, LNV_SC_T1, 0, RK_ITEMS);
  add(rl, 2 * (int64_t)ni, ni, 1, LNV_SC_T2, 0, RK_ITEMS);
  add(rl, 3 * (int64_t)ni, ni, 1, LNV_SC_T3, 0, RK_ITEMS);
  add(rl, 4 * (int64_t)ni, ni, 1, LNV_SC_FF, 0, RK_ITEMS);
  add(rl, 5 * (int64_t)ni, ni, 1, LNV_SC_GF, 0, RK_ITEMS);
  StageArgs sa{};
  sa.en_out = EN;
  return scalar_stage(part, rl, o.scalars, ST_EVAL, sa, s, sg);
}

int eval_core(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, double* G, double* F,
              double* EN, const lnv_eval_ws* ws, hipStream_t s,
              const double* sl_carry = nullptr, bool z_carry = false,
              double* scalars = nullptr, const Seg& sg = Seg{}) {
  EvalOps o{L,       S,           H,          &ws->SL,     &ws->LS, &ws->X,
            &ws->XT, &ws->Z,      ws->perm_SL, ws->perm_X,  ws->YT,  ws->W,
            ws->V,   ws->partials, scalars ? scalars : ws->scalars, &ws->Zu,    &ws->Lu, ws->Vu,
            sl_carry, z_carry};
  return eval_products<double>(L, o, G, F, EN, s, sg);
}

int convert_launch(const lnv_bsm* A, lnv_bsm* B, hipStream_t s) {
  const int64_t nv = A->pat->nnzb * (int64_t)A->blk * A->blk;
  if (nv == 0) return LNV_OK;
  int64_t g = (nv + 255) / 256;
  const int grid = (int)(g < 4 * kVecGrid ? g : 4 * kVecGrid);
  if (A->dtype == LNV_F64 && B->dtype == LNV_F32)
    k_convert<double, float><<<grid, 256, 0, s>>>(nv, static_cast<const double*>(A->val),
                                                  static_cast<float*>(B->val));
  else if (A->dtype == LNV_F32 && B->dtype == LNV_F64)
    k_convert<float, double><<<grid, 256, 0, s>>>(nv, static_cast<const float*>(A->val),
                                                  static_cast<double*>(B->val));
  else if (A->dtype == LNV_F64)
    k_convert<double, double><<<grid, 256, 0, s>>>(nv, static_cast<const double*>(A->val),
                                                   static_cast<double*>(B->val));
  else
    k_convert<float, float><<<grid, 256, 0, s>>>(nv, static_cast<const float*>(A->val),
                                                 static_cast<float*>(B->val));
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

bool f32_ok(const lnv_bsm* M) { return bsm_ok_any(M) && M->dtype == LNV_F32 && M->blk == 4; }

int check_eval32(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm* G,
                 const lnv_bsm* F, const lnv_eval32_ws* ws) {
  if (!bsm_ok(L) || !bsm_ok(S) || !bsm_ok(H) || !ws || !G || !F || !bsm_ok(G) || !bsm_ok(F))
    return LNV_EINVAL;
  if (!ws->YT || !ws->W || !ws->V || !ws->partials || !ws->scalars) return LNV_EINVAL;
  if (!f32_ok(&ws->L) || !f32_ok(&ws->S) || !f32_ok(&ws->H)) return LNV_EINVAL;
  if (L->blk != 4 || S->blk != 4 || H->blk != 4) return LNV_EUNSUPPORTED;
  if (ws->L.pat != L->pat || ws->S.pat != S->pat || ws->H.pat != H->pat) return LNV_EPATTERN;
  if (G->pat != L->pat || F->pat != L->pat) return LNV_EPATTERN;
  LNV_TRY(check_products(L, S, H, ws->SL, ws->LS, ws->X, ws->XT, ws->Z, ws->perm_SL, ws->perm_X,
                         [](const lnv_bsm* m) { return f32_ok(m); }));
  if (ws->partials_len < lnv_partials_len(partial_items(L->pat))) return LNV_EINVAL;
  return LNV_OK;
}

int vec_grid() { return kVecGrid; }

}  // namespace
}  // namespace lnv

using namespace lnv;

extern "C" const char* lnv_strerror(int st) {
  switch (st) {
    case LNV_OK: return "success";
    case LNV_EINVAL: return "invalid argument";
    case LNV_ECAPACITY: return "output capacity too small";
    case LNV_EPATTERN: return "incompatible or incomplete sparsity pattern";
    case LNV_EHIP: return "HIP runtime error";
    case LNV_ENUMERIC: return "non-finite value or no admissible root";
    case LNV_EUNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

extern "C" int lnv_last_hip_error(void) { return g_last_hip; }

extern "C" int lnv_sync_check(hipStream_t s) {
  LNV_HIP(hipStreamSynchronize(s));
  LNV_HIP(hipGetLastError());
  return LNV_OK;
}

extern "C" int lnv_cg_check(const double* scalars, int32_t* status_out, hipStream_t s) {
  if (!scalars) return LNV_EINVAL;
  double st = 0.0;
  LNV_HIP(hipMemcpyAsync(&st, scalars + LNV_SC_STATUS, sizeof(double), hipMemcpyDeviceToHost, s));
  LNV_HIP(hipStreamSynchronize(s));
  const int bits = (int)st;
  if (status_out) *status_out = bits;
  return (bits & (LNV_ST_NONFINITE | LNV_ST_RUNAWAY)) ? LNV_ENUMERIC : LNV_OK;
}

extern "C" int64_t lnv_partials_len(int32_t n_items_L) {
  return (int64_t)LNV_NSLOTS * slot_len(n_items_L);
}

extern "C" int lnv_bsm_multiply_dot(double alpha, const lnv_bsm* A, const lnv_bsm* B,
                                    int32_t transB, double beta, lnv_bsm* C, int32_t store,
                                    const lnv_bsm* M1, const lnv_bsm* M2, double* partials,
                                    double* out, hipStream_t s) {
  if (!bsm_ok_any(C)) return LNV_EINVAL;
  if ((M1 && (!bsm_ok_any(M1) || M1->pat != C->pat)) ||
      (M2 && (!bsm_ok_any(M2) || M2->pat != C->pat)))
    return LNV_EPATTERN;
  if ((M1 && M1->dtype != C->dtype) || (M2 && M2->dtype != C->dtype)) return LNV_EUNSUPPORTED;
  if ((M1 || M2) && (!partials || !out)) return LNV_EINVAL;
  if (M2 && !M1) return LNV_EINVAL;
  const void* m1 = M1 ? M1->val : nullptr;
  const void* m2 = M2 ? M2->val : nullptr;
  LNV_TRY(multiply_launch(alpha, A, B, transB, beta, C, store, m1, m2, partials, nullptr, s));
  if (!M1) return LNV_OK;
  const int ni = multiply_nparts(A, B, transB, C);
  // reduce the interleaved partials into out[0..1] (fixed order)
  RedList rl = reds();
  add(rl, 0, ni, 2, 0);
  if (M2) add(rl, 1, ni, 2, 1);
  StageArgs sa{};
  k_scalar<<<1, 256, 0, s>>>(partials, rl, out, ST_NONE, sa, Seg{});
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

// Scratch of lnv_bsm_multiply_dot_noalloc: the trace partials of the
// multiply's work pieces, in device memory the library holds for the life of
// the process (one copy per GPU, each at its own address).  Host code names
// it only through hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[LNV_NOALLOC_PARTIALS];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of this GPU's scratch (the current device), looked up on
// the first call made with that device current.
int scratch_address(double** out) {
  int dev = -1;
  LNV_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return LNV_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    LNV_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return LNV_EHIP;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return LNV_OK;
}
}  // namespace

extern "C" int lnv_bsm_multiply_dot_noalloc(double alpha, const lnv_bsm* A, const lnv_bsm* B,
                                            int32_t transB, double beta, lnv_bsm* C,
                                            int32_t store, const lnv_bsm* M1, const lnv_bsm* M2,
                                            double* out, hipStream_t s) {
  if (!M1 || !out) return LNV_EINVAL;
  if (!bsm_ok_any(A) || !bsm_ok_any(B) || !bsm_ok_any(C)) return LNV_EINVAL;
  if (timing_on()) return LNV_EUNSUPPORTED;   // the timing creates events
  // every work piece writes its two partials before the reduction reads
  // them, so nothing in the scratch needs clearing between calls
  const int64_t need = 2 * (int64_t)multiply_nparts(A, B, transB, C);
  if (need > LNV_NOALLOC_PARTIALS) return LNV_ECAPACITY;
  double* part = nullptr;
  LNV_TRY(scratch_address(&part));
  return lnv_bsm_multiply_dot(alpha, A, B, transB, beta, C, store, M1, M2, part, out, s);
}

extern "C" int lnv_bsm_dot(const lnv_bsm* A, const lnv_bsm* B, double* partials, double* out,
                           hipStream_t s) {
  if (!bsm_ok(A) || !bsm_ok(B) || !partials || !out) return LNV_EINVAL;
  if (A->blk != 4 || B->blk != 4) return LNV_EUNSUPPORTED;
  const lnv_pattern *pa = A->pat, *pb = B->pat;
  if (pa->n != pb->n) return LNV_EPATTERN;
  const bool same = pa == pb;
  if (!pattern_ready(pa, false, false, true) || (!same && !has_ix(pb))) return LNV_EPATTERN;
  const int ni = pa->n_items;
  if (ni == 0) {
    LNV_HIP(hipMemsetAsync(out, 0, sizeof(double), s));
    return LNV_OK;
  }
  const int grid = ni < LNV_DOT_PARTIALS ? ni : LNV_DOT_PARTIALS;
  k_dot_items<<<grid, 256, 0, s>>>(pa->n, ni, pa->items, pa->row_ptr, pa->col,
                                   static_cast<const double*>(A->val), make_ix(pb), same ? 1 : 0,
                                   static_cast<const double*>(B->val), partials, nullptr);
  LNV_LAUNCH_CHECK();
  RedList rl = reds();
  add(rl, 0, grid, 1, 0);
  StageArgs sa{};
  k_scalar<<<1, 256, 0, s>>>(partials, rl, out, ST_NONE, sa, Seg{});
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_eval(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, lnv_bsm* G,
                        lnv_bsm* F, double* EN, lnv_eval_ws* ws, hipStream_t s) {
  if (!G || !F) return LNV_EINVAL;
  LNV_TRY(check_eval(L, S, H, G, F, ws));
  ws->carry = 0;   // Z (and S.L) now belong to this L
  return eval_core(L, S, H, static_cast<double*>(G->val), static_cast<double*>(F->val), EN, ws,
                   s);
}

extern "C" int lnv_eval_mixed(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, lnv_bsm* G,
                              lnv_bsm* F, double* EN, const lnv_eval32_ws* ws, hipStream_t s) {
  LNV_TRY(check_eval32(L, S, H, G, F, ws));
  lnv_bsm L32 = ws->L, S32 = ws->S, H32 = ws->H;
  LNV_TRY(convert_launch(L, &L32, s));
  LNV_TRY(convert_launch(S, &S32, s));
  LNV_TRY(convert_launch(H, &H32, s));
  EvalOps o{&L32,    &S32,         &H32,        &ws->SL,     &ws->LS, &ws->X,
            &ws->XT, &ws->Z,       ws->perm_SL, ws->perm_X,  ws->YT,  ws->W,
            ws->V,   ws->partials, ws->scalars, &ws->Zu,     &ws->Lu, ws->Vu};
  return eval_products<float>(L, o, static_cast<double*>(G->val), static_cast<double*>(F->val),
                              EN, s);
}

extern "C" int lnv_bsm_lincomb(double a, const lnv_bsm* X, double b, const lnv_bsm* Y, double c,
                               const lnv_bsm* Z, lnv_bsm* out, hipStream_t s) {
  if (!bsm_ok(X) || !bsm_ok(out) || (Y && !bsm_ok(Y)) || (Z && !bsm_ok(Z))) return LNV_EINVAL;
  const int64_t nb = X->pat->nnzb;
  if (out->pat->nnzb != nb || (Y && Y->pat->nnzb != nb) || (Z && Z->pat->nnzb != nb) ||
      X->blk != out->blk || (Y && Y->blk != X->blk) || (Z && Z->blk != X->blk))
    return LNV_EPATTERN;
  const int64_t nv = nb * X->blk * X->blk;
  if (nv == 0) return LNV_OK;
  k_lincomb<<<vec_grid(), 256, 0, s>>>(nv, a, static_cast<const double*>(X->val), b,
                                       Y ? static_cast<const double*>(Y->val) : nullptr, c,
                                       Z ? static_cast<const double*>(Z->val) : nullptr,
                                       static_cast<double*>(out->val));
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_bsm_remap(const lnv_bsm* A, lnv_bsm* B, hipStream_t s) {
  if (!bsm_ok(A) || !bsm_ok(B)) return LNV_EINVAL;
  if (A->blk != 4 || B->blk != 4) return LNV_EUNSUPPORTED;
  if (A->pat->n != B->pat->n || !has_ix(A->pat) || !B->pat->row_ptr || !B->pat->col)
    return LNV_EPATTERN;
  k_remap<<<B->pat->n, 256, 0, s>>>(B->pat->n, B->pat->row_ptr, B->pat->col, make_ix(A->pat),
                                    static_cast<const double*>(A->val),
                                    static_cast<double*>(B->val));
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_bsm_norm_inf(const lnv_bsm* A, double* partials, double* out, hipStream_t s) {
  if (!bsm_ok(A) || !partials || !out) return LNV_EINVAL;
  if (A->blk != 4) return LNV_EUNSUPPORTED;
  const lnv_pattern* pa = A->pat;
  if (!pa->row_ptr) return LNV_EPATTERN;
  k_rowabs<<<pa->n, 256, 0, s>>>(pa->row_ptr, static_cast<const double*>(A->val), partials);
  LNV_LAUNCH_CHECK();
  RedList rl = reds();
  add(rl, 0, pa->n, 1, 0, 1);
  StageArgs sa{};
  k_scalar<<<1, 256, 0, s>>>(partials, rl, out, ST_NONE, sa, Seg{});
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_cell_traces(const lnv_pattern* PL, const lnv_eval_ws* ws, int32_t n_cells,
                               const int32_t* cell_item_ptr, double* EN_cells, hipStream_t s) {
  if (!PL || !ws || !ws->partials || !cell_item_ptr || !EN_cells || n_cells <= 0)
    return LNV_EINVAL;
  if (PL->n_items <= 0) return LNV_EPATTERN;
  k_cell_traces<<<n_cells, 256, 0, s>>>(ws->partials, PL->n_items, cell_item_ptr, EN_cells);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_bsm_convert(const lnv_bsm* A, lnv_bsm* B, hipStream_t s) {
  if (!bsm_ok_any(A) || !bsm_ok_any(B)) return LNV_EINVAL;
  if (A->blk != B->blk) return LNV_EPATTERN;
  if (A->pat != B->pat && A->pat->nnzb != B->pat->nnzb) return LNV_EPATTERN;
  return convert_launch(A, B, s);
}

namespace {

int check_cg(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm* T,
             const lnv_cg_ws* ws) {
  if (!ws) return LNV_EINVAL;
  LNV_TRY(check_eval(L, S, H, nullptr, nullptr, &ws->ev));
  if (lean_ws(ws->ev.LS, ws->ev.XT)) return LNV_EINVAL;   // the step's scratch buffers
  if (!ws->SL2 || !ws->Hp || !ws->G || !ws->F || !ws->g || !ws->gc_prev || !ws->D ||
      !ws->D_prev)
    return LNV_EINVAL;
  if (!pattern_ready(S->pat, true, false, false) || !pattern_ready(H->pat, false, false, true))
    return LNV_EPATTERN;
  if (ws->ev.X.pat->nnzb < ws->ev.Z.pat->nnzb) return LNV_EINVAL;  // Z_F reuses X's buffer
  if (T) {
    if (!bsm_ok(T) || T->pat != L->pat || T->blk != 4) return LNV_EPATTERN;
    if (!ws->Gc || !ws->Fc || !ws->gc || !bsm_ok(&ws->LL)) return LNV_EINVAL;
    if (ws->LL.pat->n != L->pat->n || !pattern_ready(ws->LL.pat, false, false, true))
      return LNV_EPATTERN;
  }
  return LNV_OK;
}

// Partial sums of the traces T0..T3 written by cubic_traces: trace t is the
// sum of n[t] partials at off[t], off[t] + stride[t], ...
struct TraceParts {
  int64_t off[4];
  int n[4];
  int stride[4];
};

// Traces of the cubic along direction P at the current L, with M the
// (symmetric) matrix the trace is taken against: H' = H - mu S for the
// energy line, S for the electron number (m_is_s).  With A_P^T = S P (into
// apt), A_P = its transpose (into ap) and X_P = M A_P:
//   T0 = <P, X_P>           = Tr[P M P S]
//   T1 = Tr[L S P S P M],   T2 = Tr[P S P S P M],   T3 = Tr[P S L S P M]
// (the energy's cubic has c2 = 2(3 T0 - 2(2 T1 + T3)), c3 = -4 T2; T1 = T3
// when M = S).  Q = A_P^T X_P = S P M P S is symmetric, and by cyclic shifts
// and transposition of the traces of products of symmetric matrices
//   T3 = <L, Q>,  T2 = <P, Q>,  T1 = <P, S L X_P>  (S L = SLcur).
// With the workspace's half of L's pattern (ev.Lu, ev.Vu) Q is formed only
// on the half, traced against weighted halves of L and P (k_half_weighted),
// and S L X_P on L's pattern reads X_P as stored; without it, the products
// P_L(X_P A_P) (as P_L(A_P^T X_P^T), X_P^T transposed into XPT unless
// M = S) and P_L(X_P A) are formed in full.
int cubic_traces(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* M, bool m_is_s,
                 const double* P, const lnv_eval_ws& ev, double* apt, double* ap,
                 const lnv_bsm* SLcur, lnv_bsm XP, const lnv_bsm* XPT, double* partials,
                 int64_t slot, const double* skip, TraceParts* tp, hipStream_t s) {
  const lnv_pattern* pl = L->pat;
  lnv_bsm Pm{pl, 4, LNV_F64, const_cast<double*>(P)};
  lnv_bsm APT{ev.SL.pat, 4, LNV_F64, apt};
  lnv_bsm AP{ev.LS.pat, 4, LNV_F64, ap};
  LNV_TRY(multiply_launch(1.0, S, &Pm, 0, 0.0, &APT, 1, nullptr, nullptr, nullptr, skip, s));
  LNV_TRY(transpose_skip_launch(&APT, ev.perm_SL, ap, skip, s));
  if (m_is_s && XP.pat == ev.Z.pat && sym_ready(&ev.Zu, &XP)) {
    // M = S: X_P = S P S is symmetric, formed from its half
    LNV_TRY(multiply_launch(1.0, M, &AP, 0, 0.0, &ev.Zu, 1, nullptr, nullptr, nullptr, skip, s));
    LNV_TRY(mirror_launch(&ev.Zu, &XP, s, skip));
  } else {
    LNV_TRY(multiply_launch(1.0, M, &AP, 0, 0.0, &XP, 1, nullptr, nullptr, nullptr, skip, s));
  }
  const int ni = pl->n_items;
  // one workgroup per item: partial q belongs to item q
  k_dot_items<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, P, make_ix(XP.pat),
                                 0, static_cast<const double*>(XP.val), partials + 0 * slot, skip);
  LNV_LAUNCH_CHECK();
  tp->off[0] = 0;
  tp->n[0] = ni;
  tp->stride[0] = 1;
  // C of the trace-only products: written between contraction slabs, so it
  // needs a buffer of its own (ev.YT is dead outside the evaluation)
  lnv_bsm scratchC{pl, 4, LNV_F64, ev.YT};
  const lnv_pattern* pu = ev.Lu.pat;
  // the half (in_half) of L's pattern holds every block of a row group and
  // one block of each other pair: between half and all of L's blocks
  const bool half = pu && ev.Lu.val && ev.Vu && pu->n == pl->n && has_ix(pu) && pu->row_ptr &&
                    pu->col && pl->items && ev.Lu.dtype == LNV_F64 &&
                    2 * pu->nnzb >= pl->nnzb + pl->n && pu->nnzb <= pl->nnzb &&
                    (m_is_s || SLcur);
  if (half) {
    lnv_bsm Qh{pu, 4, LNV_F64, ev.YT};
    const int nq = multiply_nparts(&APT, &XP, 0, &Qh);
    const int nr = m_is_s ? 0 : multiply_nparts(SLcur, &XP, 0, &scratchC);
    if (2 * (int64_t)nq <= slot && 2 * (int64_t)nr <= slot) {
      double* Lh = static_cast<double*>(ev.Lu.val);
      double* Ph = static_cast<double*>(ev.Vu);
      k_half_weighted<<<ni, 256, 0, s>>>(pl->n, pl->items, pl->row_ptr, pl->col, make_ix(pu),
                                         static_cast<const double*>(L->val), P, Lh, Ph, skip);
      LNV_LAUNCH_CHECK();
      // <L, Q> -> T3 (even partials), <P, Q> -> T2 (odd)
      LNV_TRY(multiply_launch(1.0, &APT, &XP, 0, 0.0, &Qh, 0, Lh, Ph, partials + 1 * slot, skip,
                              s));
      tp->off[3] = 1 * slot;
      tp->off[2] = 1 * slot + 1;
      tp->n[2] = tp->n[3] = nq;
      tp->stride[2] = tp->stride[3] = 2;
      if (m_is_s) {
        tp->off[1] = tp->off[3];
        tp->n[1] = nq;
        tp->stride[1] = 2;
        return LNV_OK;
      }
      // T1 = <P, S L X_P>
      LNV_TRY(multiply_launch(1.0, SLcur, &XP, 0, 0.0, &scratchC, 0, P, nullptr,
                              partials + 2 * slot, skip, s));
      tp->off[1] = 2 * slot;
      tp->n[1] = nr;
      tp->stride[1] = 2;
      return LNV_OK;
    }
  }
  const lnv_bsm* B = &XP;
  if (XPT && !m_is_s) {
    LNV_TRY(transpose_skip_launch(&XP, ev.perm_X, static_cast<double*>(XPT->val), skip, s));
    B = XPT;
  } else if (!m_is_s) {
    return LNV_EINVAL;   // X_P^T needs a buffer
  }
  const int np = multiply_nparts(&APT, B, 0, &scratchC);
  tp->off[1] = 1 * slot;
  tp->off[2] = 1 * slot + 1;
  tp->off[3] = 2 * slot;
  for (int t = 1; t < 4; ++t) {
    tp->n[t] = np;
    tp->stride[t] = 2;
  }
  if (SLcur && multiply_nparts(SLcur, B, 0, &scratchC) != np) return LNV_EPATTERN;
  if (!SLcur) {
    tp->off[3] = tp->off[1];   // T3 = T1 when M = S
    return multiply_launch(1.0, &APT, B, 0, 0.0, &scratchC, 0,
                           static_cast<const double*>(L->val), P, partials + 1 * slot, skip, s);
  }
  // both trace products in one launch (the second's second trace, <P, .>
  // again, lands in the unused odd partials of its slot)
  return multiply_pair_launch(&APT, B, &scratchC, SLcur, B, &scratchC, 0,
                              static_cast<const double*>(L->val), P, partials + 1 * slot, P, P,
                              partials + 2 * slot, skip, s);
}

// out = P_L(T V T) through the natural-range intermediate on pat(L.L) (in
// ws->LL).  With an index table on pat(L.L) it is formed as P_L(T (V T)):
// the restricted product then contracts over T's short rows (range R_L)
// with the natural-range V T on the right, the orientation in which nearly
// every lane of a 64-column piece finds its block; (T V) T would contract
// over the long rows of T V against T's short rows (about a tenth of the
// lanes busy).  The triples are the same either way.
int metric_apply(const lnv_bsm* T, const double* V, double* out, lnv_cg_ws* ws, hipStream_t s) {
  const lnv_pattern* pl = T->pat;
  lnv_bsm Vm{pl, 4, LNV_F64, const_cast<double*>(V)};
  lnv_bsm Om{pl, 4, LNV_F64, out};
  // P_L(T V T) is symmetric for symmetric T and V
  if (has_ix(ws->LL.pat)) {
    LNV_TRY(multiply_launch(1.0, &Vm, T, 0, 0.0, &ws->LL, 1, nullptr, nullptr, nullptr, nullptr,
                            s));
    return sym_product(T, &ws->LL, &Om, &ws->ev.Lu, s);
  }
  LNV_TRY(multiply_launch(1.0, T, &Vm, 0, 0.0, &ws->LL, 1, nullptr, nullptr, nullptr, nullptr, s));
  return sym_product(&ws->LL, T, &Om, &ws->ev.Lu, s);
}

// out1 = P_L(T V1 T), out2 = P_L(T V2 T) as paired launches: the natural
// intermediates (V1 T, V2 T; or T V1, T V2) into LL and into X's buffer
// (free between the evaluation and the line search) when pat(L.L) fits
// there, the halves into Lu's and Vu's buffers; otherwise one after the
// other.
int metric_apply_pair(const lnv_bsm* T, const double* V1, double* out1, const double* V2,
                      double* out2, lnv_cg_ws* ws, hipStream_t s) {
  const lnv_eval_ws& ev = ws->ev;
  const lnv_pattern* pl = T->pat;
  const bool room = ws->LL.pat && ev.X.pat && ws->LL.pat->nnzb <= ev.X.pat->nnzb && ev.X.val &&
                    ev.Vu && ev.Lu.val && ev.Lu.pat;
  if (!room) {
    LNV_TRY(metric_apply(T, V1, out1, ws, s));
    return metric_apply(T, V2, out2, ws, s);
  }
  lnv_bsm V1m{pl, 4, LNV_F64, const_cast<double*>(V1)}, V2m{pl, 4, LNV_F64, const_cast<double*>(V2)};
  lnv_bsm O1{pl, 4, LNV_F64, out1}, O2{pl, 4, LNV_F64, out2};
  lnv_bsm LL2{ws->LL.pat, 4, LNV_F64, ev.X.val};
  lnv_bsm U2{ev.Lu.pat, 4, LNV_F64, ev.Vu};
  if (has_ix(ws->LL.pat)) {
    LNV_TRY(multiply_pair_launch(&V1m, T, &ws->LL, &V2m, T, &LL2, 1, nullptr, nullptr, nullptr,
                                 nullptr, nullptr, nullptr, nullptr, s));
    return sym_product_pair(T, &ws->LL, &O1, &ev.Lu, T, &LL2, &O2, &U2, s);
  }
  LNV_TRY(multiply_pair_launch(T, &V1m, &ws->LL, T, &V2m, &LL2, 1, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, s));
  return sym_product_pair(&ws->LL, T, &O1, &ev.Lu, &LL2, T, &O2, &U2, s);
}

// The metric products of a mixed-precision step in FP32 (the metric is a
// preconditioner: the projection keeps <D, F> = 0 in FP64 whatever the
// precision of F_c, and the line search and electron-number correction stay
// FP64).  T, G, F are rounded to FP32 into buffers the FP32 evaluation has
// finished with (its L copy, YT, W), the natural intermediates G T and F T
// go to its X and XT, the halves to its Lu and Vu, the mirrored results to
// YT and W (G and F in FP32 are dead by then), and G_c, F_c come back in
// FP64.  LNV_EUNSUPPORTED when a buffer or table does not fit: the caller
// then forms the products in FP64.
int metric_apply_pair32(const lnv_bsm* T, const double* G, double* Gc, const double* F,
                        double* Fc, const lnv_cg_ws* ws, const lnv_eval32_ws* w32,
                        hipStream_t s) {
  const lnv_pattern* pl = T->pat;
  const lnv_pattern* pll = ws->LL.pat;
  const lnv_pattern* pu = w32->Lu.pat;
  if (!pll || !has_ix(pll) || !w32->X.val || !w32->XT.val || !w32->X.pat || !w32->XT.pat ||
      pll->nnzb > w32->X.pat->nnzb || pll->nnzb > w32->XT.pat->nnzb || !pu || !w32->Lu.val ||
      !w32->Vu || !w32->YT || !w32->W || !w32->L.val || w32->L.pat != pl || pu->n != pl->n ||
      w32->Lu.dtype != LNV_F32)
    return LNV_EUNSUPPORTED;
  lnv_bsm T32{pl, 4, LNV_F32, w32->L.val};
  lnv_bsm G64{pl, 4, LNV_F64, const_cast<double*>(G)}, F64{pl, 4, LNV_F64, const_cast<double*>(F)};
  lnv_bsm G32{pl, 4, LNV_F32, w32->YT}, F32{pl, 4, LNV_F32, w32->W};
  LNV_TRY(convert_launch(T, &T32, s));
  LNV_TRY(convert_launch(&G64, &G32, s));
  LNV_TRY(convert_launch(&F64, &F32, s));
  lnv_bsm GT{pll, 4, LNV_F32, w32->X.val}, FT{pll, 4, LNV_F32, w32->XT.val};
  LNV_TRY(multiply_pair_launch(&G32, &T32, &GT, &F32, &T32, &FT, 1, nullptr, nullptr, nullptr,
                               nullptr, nullptr, nullptr, nullptr, s));
  lnv_bsm U1{pu, 4, LNV_F32, w32->Lu.val}, U2{pu, 4, LNV_F32, w32->Vu};
  LNV_TRY(sym_product_pair(&T32, &GT, &G32, &U1, &T32, &FT, &F32, &U2, s));
  lnv_bsm Gc64{pl, 4, LNV_F64, Gc}, Fc64{pl, 4, LNV_F64, Fc};
  LNV_TRY(convert_launch(&G32, &Gc64, s));
  return convert_launch(&F32, &Fc64, s);
}

}  // namespace

namespace {

// Hotelling's iteration; sc: the scalar block(s) (a batch: sigma per cell,
// from each cell's rows).
int hotelling_impl(const lnv_bsm* S, lnv_bsm* T, int32_t n_iter, lnv_cg_ws* ws, double* sc,
                   const Seg& sg, hipStream_t s) {
  if (!bsm_ok(S) || !bsm_ok(T) || !ws || n_iter < 0) return LNV_EINVAL;
  if (S->blk != 4 || T->blk != 4) return LNV_EUNSUPPORTED;
  const lnv_eval_ws& ev = ws->ev;
  if (!ws->Gc || !ev.partials || !sc || !bsm_ok(&ev.SL)) return LNV_EINVAL;
  const lnv_pattern* pt = T->pat;
  if (S->pat->n != pt->n || ev.SL.pat->n != pt->n) return LNV_EPATTERN;
  if (!pattern_ready(pt, true, false, true) || !pattern_ready(S->pat, true, false, false) ||
      !pattern_ready(ev.SL.pat, true, false, true))
    return LNV_EPATTERN;
  if (ev.partials_len < pt->n) return LNV_EINVAL;
  ws->ev.carry = 0;
  double* part = ev.partials;
  const size_t bytes = sizeof(double) * (size_t)pt->nnzb * 16;
  k_rowabs<<<S->pat->n, 256, 0, s>>>(S->pat->row_ptr, static_cast<const double*>(S->val), part);
  LNV_LAUNCH_CHECK();
  RedList rl = reds();
  add(rl, 0, S->pat->n, 1, LNV_SC_T4, 1, RK_ROWS);
  StageArgs sa{};
  LNV_TRY(scalar_stage(part, rl, sc, ST_SIGMA, sa, s, sg));
  k_identity<<<pt->n_items, 256, 0, s>>>(pt->n, pt->items, pt->row_ptr, pt->col, make_ix(S->pat),
                                         static_cast<const double*>(S->val), sc, LNV_SC_SIGMA,
                                         static_cast<double*>(T->val), sg);
  LNV_LAUNCH_CHECK();
  // T_{n+1} = 2 T_n - T_n (S T_n) on T's pattern; ST lives on pat(S.T)
  lnv_bsm ST{ev.SL.pat, 4, LNV_F64, ev.SL.val};
  double* cur = static_cast<double*>(T->val);
  double* nxt = ws->Gc;
  for (int it = 0; it < n_iter; ++it) {
    lnv_bsm Tc{pt, 4, LNV_F64, cur};
    lnv_bsm Tn{pt, 4, LNV_F64, nxt};
    LNV_TRY(multiply_launch(1.0, S, &Tc, 0, 0.0, &ST, 1, nullptr, nullptr, nullptr, nullptr, s));
    LNV_HIP(hipMemcpyAsync(nxt, cur, bytes, hipMemcpyDeviceToDevice, s));
    LNV_TRY(multiply_launch(-1.0, &Tc, &ST, 0, 2.0, &Tn, 1, nullptr, nullptr, nullptr, nullptr, s));
    std::swap(cur, nxt);
  }
  if (cur != T->val) LNV_HIP(hipMemcpyAsync(T->val, cur, bytes, hipMemcpyDeviceToDevice, s));
  return LNV_OK;
}

}  // namespace

extern "C" int lnv_hotelling(const lnv_bsm* S, lnv_bsm* T, int32_t n_iter, lnv_cg_ws* ws,
                             hipStream_t s) {
  if (!ws) return LNV_EINVAL;
  return hotelling_impl(S, T, n_iter, ws, ws->ev.scalars, Seg{}, s);
}

namespace {

int check_pm(const lnv_bsm* K, const lnv_pm_ws* ws) {
  if (!bsm_ok(K) || !ws || !ws->K2 || !ws->K3 || !ws->KT || !ws->perm_L || !ws->partials ||
      !ws->scalars || !ws->hist || ws->hist_len < 0 || !bsm_ok(&ws->SK))
    return LNV_EINVAL;
  if (K->blk != 4 || ws->SK.blk != 4) return LNV_EUNSUPPORTED;
  const lnv_pattern* pl = K->pat;
  if (!pattern_ready(pl, true, false, true)) return LNV_EPATTERN;
  if (ws->partials_len < lnv_partials_len(partial_items(pl))) return LNV_EINVAL;
  return LNV_OK;
}

}  // namespace

namespace {

// Purification start and step; a batch (sg.n > 0) takes n_orb and n_elec per
// cell from sg, reduces per cell (scalars and history per cell at stride
// LNV_PM_NSCALARS and 4 hist_len) and never skips a launch: a stopped cell
// gets the coefficients (1, 0, 0), which leave its K unchanged.
int pm_start_impl(lnv_bsm* K, const lnv_bsm* T, const lnv_bsm* H, lnv_bsm* HT, double n_orb,
                  double n_elec, lnv_pm_ws* ws, const Seg& sg, hipStream_t s) {
  LNV_TRY(check_pm(K, ws));
  if (!bsm_ok(T) || !bsm_ok(H) || !bsm_ok(HT) || (sg.n == 0 && !(n_orb > 0.0 && n_elec > 0.0)))
    return LNV_EINVAL;
  const lnv_pattern* pl = K->pat;
  if (T->pat != pl) return LNV_EPATTERN;
  if (!pattern_ready(H->pat, true, false, false) || !H->pat->row_ptr) return LNV_EPATTERN;
  const int ni = pl->n_items;
  const int64_t slot = slot_len(partial_items(pl));
  if ((int64_t)H->pat->n > slot || (int64_t)pl->n > slot) return LNV_EINVAL;
  double* part = ws->partials;
  double* sc = ws->scalars;
  // <T, H>, ||T||inf, ||H||inf
  k_dot_items<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col,
                                 static_cast<const double*>(T->val), make_ix(H->pat), 0,
                                 static_cast<const double*>(H->val), part, nullptr);
  LNV_LAUNCH_CHECK();
  k_rowabs<<<pl->n, 256, 0, s>>>(pl->row_ptr, static_cast<const double*>(T->val), part + slot);
  LNV_LAUNCH_CHECK();
  k_rowabs<<<H->pat->n, 256, 0, s>>>(H->pat->row_ptr, static_cast<const double*>(H->val),
                                     part + 2 * slot);
  LNV_LAUNCH_CHECK();
  RedList rl = reds();
  add(rl, 0, ni, 1, LNV_PM_DOT, 0, RK_ITEMS);
  add(rl, slot, pl->n, 1, LNV_PM_NT, 1, RK_ROWS);
  add(rl, 2 * slot, H->pat->n, 1, LNV_PM_NH, 1, RK_ROWS);
  StageArgs sa{};
  sa.pm_n = n_orb;
  sa.pm_theta = 0.5 * n_elec;
  LNV_TRY(scalar_stage(part, rl, sc, ST_PM0, sa, s, sg));
  // K0 = a0 T + a1 P_L(T (H T))
  lnv_bsm K2{pl, 4, LNV_F64, ws->K2};
  LNV_TRY(multiply_launch(1.0, H, T, 0, 0.0, HT, 1, nullptr, nullptr, nullptr, nullptr, s));
  LNV_TRY(multiply_launch(1.0, T, HT, 0, 0.0, &K2, 1, nullptr, nullptr, nullptr, nullptr, s));
  const int64_t nv = pl->nnzb * 16;
  k_lincomb_sc<<<seg_grid(sg), 256, 0, s>>>(nv, sc, LNV_PM_A0, LNV_PM_A1, LNV_PM_A2,
                                            static_cast<const double*>(T->val), ws->K2, nullptr,
                                            static_cast<double*>(K->val), nullptr, sg);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

int pm_step_impl(lnv_bsm* K, const lnv_bsm* S, double n_elec, double tol, lnv_pm_ws* ws,
                 const Seg& sg, hipStream_t s) {
  LNV_TRY(check_pm(K, ws));
  if (!bsm_ok(S) || (sg.n == 0 && !(n_elec > 0.0)) || !(tol >= 0.0)) return LNV_EINVAL;
  const lnv_pattern* pl = K->pat;
  if (!pattern_ready(S->pat, true, false, false)) return LNV_EPATTERN;
  const int ni = pl->n_items;
  const int64_t slot = slot_len(partial_items(pl));
  const int64_t nv = pl->nnzb * 16;
  double* part = ws->partials;
  double* sc = ws->scalars;
  // one system: a stopped purification turns every launch into a no-op
  const double* stopped = sg.n > 0 ? nullptr : sc + LNV_PM_STOPPED;
  double* Kv = static_cast<double*>(K->val);
  lnv_bsm K2{pl, 4, LNV_F64, ws->K2}, K3{pl, 4, LNV_F64, ws->K3};
  // S K, K S K = P_L(K . SK), K S K S K = P_L(KSK . SK)
  LNV_TRY(multiply_launch(1.0, S, K, 0, 0.0, &ws->SK, 1, nullptr, nullptr, nullptr, stopped, s));
  LNV_TRY(multiply_launch(1.0, K, &ws->SK, 0, 0.0, &K2, 1, nullptr, nullptr, nullptr, stopped,
                          s));
  LNV_TRY(multiply_launch(1.0, &K2, &ws->SK, 0, 0.0, &K3, 1, nullptr, nullptr, nullptr, stopped,
                          s));
  // t_p = <K (SK)^(p-1), S>
  const double* Ms[3] = {Kv, ws->K2, ws->K3};
  for (int p = 0; p < 3; ++p) {
    k_dot_items<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, Ms[p],
                                   make_ix(S->pat), 0, static_cast<const double*>(S->val),
                                   part + p * slot, stopped);
    LNV_LAUNCH_CHECK();
  }
  RedList rl = reds();
  add(rl, 0, ni, 1, LNV_PM_T1, 0, RK_ITEMS);
  add(rl, slot, ni, 1, LNV_PM_T2, 0, RK_ITEMS);
  add(rl, 2 * slot, ni, 1, LNV_PM_T3, 0, RK_ITEMS);
  StageArgs sa{};
  sa.pm_theta = 0.5 * n_elec;
  sa.pm_tol = tol;
  sa.pm_hist = ws->hist;
  sa.pm_hist_len = ws->hist_len;
  sa.pm_batch = sg.n > 0;
  // a stopped purification leaves its scalars alone (the stage returns first)
  LNV_TRY(scalar_stage(part, rl, sc, ST_PM, sa, s, sg));
  const int vg = seg_grid(sg);
  k_lincomb_sc<<<vg, 256, 0, s>>>(nv, sc, LNV_PM_A0, LNV_PM_A1, LNV_PM_A2, Kv, ws->K2, ws->K3,
                                  Kv, stopped, sg);
  LNV_LAUNCH_CHECK();
  // K <- (K + K^T)/2
  LNV_TRY(transpose_skip_launch(K, ws->perm_L, ws->KT, stopped, s));
  k_lincomb_sc<<<vg, 256, 0, s>>>(nv, sc, LNV_PM_HALF, LNV_PM_HALF, 0, Kv, ws->KT, nullptr, Kv,
                                  stopped, sg);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

}  // namespace

extern "C" int lnv_pm_start(lnv_bsm* K, const lnv_bsm* T, const lnv_bsm* H, lnv_bsm* HT,
                            double n_orb, double n_elec, lnv_pm_ws* ws, hipStream_t s) {
  return pm_start_impl(K, T, H, HT, n_orb, n_elec, ws, Seg{}, s);
}

extern "C" int lnv_pm_step(lnv_bsm* K, const lnv_bsm* S, double n_elec, double tol,
                           lnv_pm_ws* ws, hipStream_t s) {
  return pm_step_impl(K, S, n_elec, tol, ws, Seg{}, s);
}

extern "C" int lnv_cg_init(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* T, double n_elec,
                           lnv_cg_ws* ws, hipStream_t s) {
  if (!bsm_ok(L) || !bsm_ok(S) || !ws || !(n_elec > 0.0)) return LNV_EINVAL;
  if (L->blk != 4 || S->blk != 4) return LNV_EUNSUPPORTED;
  const lnv_eval_ws& ev = ws->ev;
  if (!ev.partials || !ev.scalars || !ws->D || !ws->D_prev || !ws->gc_prev || !ws->SL2)
    return LNV_EINVAL;
  if (!bsm_ok(&ev.SL) || !bsm_ok(&ev.LS) || !bsm_ok(&ev.X) || !bsm_ok(&ev.Z) || !ev.perm_SL)
    return LNV_EINVAL;
  if (!pattern_ready(L->pat, true, false, true) || !pattern_ready(ev.SL.pat, false, false, true) ||
      !pattern_ready(ev.LS.pat, true, false, false) || !pattern_ready(ev.Z.pat, true, false, true) ||
      !pattern_ready(S->pat, true, false, false))
    return LNV_EPATTERN;
  if (T && (!bsm_ok(T) || T->pat != L->pat || T->blk != 4)) return LNV_EPATTERN;
  if (ev.partials_len < lnv_partials_len(partial_items(L->pat))) return LNV_EINVAL;
  ws->ev.carry = 0;   // SL2 and Z are scratch here
  const lnv_pattern* pl = L->pat;
  const int64_t nv = pl->nnzb * 16;
  const int ni = pl->n_items;
  const int64_t slot = slot_len(partial_items(pl));
  double* part = ev.partials;
  double* sc = ev.scalars;
  // keep sigma (from lnv_hotelling) and the counters across the reset
  LNV_HIP(hipMemsetAsync(sc, 0, sizeof(double) * LNV_SC_SIGMA, s));
  LNV_HIP(hipMemsetAsync(sc + LNV_SC_GGN, 0, sizeof(double), s));
  LNV_HIP(hipMemsetAsync(sc + LNV_SC_NCORR + 1, 0,
                         sizeof(double) * (LNV_NSCALARS - LNV_SC_NCORR - 1), s));
  LNV_HIP(hipMemsetAsync(ws->gc_prev, 0, sizeof(double) * nv, s));
  LNV_HIP(hipMemsetAsync(ws->D_prev, 0, sizeof(double) * nv, s));
  LNV_HIP(hipMemsetAsync(L->val, 0, sizeof(double) * nv, s));
  if (T) {
    LNV_HIP(hipMemcpyAsync(ws->D, T->val, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
  } else {
    k_identity<<<ni, 256, 0, s>>>(pl->n, pl->items, pl->row_ptr, pl->col, make_ix(S->pat),
                                  static_cast<const double*>(S->val), nullptr, 0, ws->D, Seg{});
    LNV_LAUNCH_CHECK();
  }
  // N(lambda T) = 6 Tr[TSTS] lambda^2 - 4 Tr[TSTSTS] lambda^3 at L = 0:
  // A_D^T = S T, Z_D = S A_D = S T S,  <T, Z_D> and <T, P_L(Z_D A_D)>.
  lnv_bsm ZD{ev.Z.pat, 4, LNV_F64, ev.Z.val};
  TraceParts tp{};
  LNV_TRY(cubic_traces(L, S, S, true, ws->D, ev, ws->SL2, static_cast<double*>(ev.LS.val), nullptr,
                       ZD, nullptr, part, slot, nullptr, &tp, s));
  RedList rl = reds();
  add(rl, tp.off[0], tp.n[0], tp.stride[0], LNV_SC_T0);
  add(rl, tp.off[2], tp.n[2], tp.stride[2], LNV_SC_T2);
  StageArgs sa{};
  sa.n_elec = n_elec;
  LNV_TRY(scalar_stage(part, rl, sc, ST_INIT, sa, s));
  k_vec_axpy<<<vec_grid(), 256, 0, s>>>(nv, ws->D, sc, LNV_SC_LAMBDA, nullptr,
                                        static_cast<double*>(L->val), Seg{});
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_cg_step(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm* T,
                           double n_elec, int64_t k, const lnv_opts* opts, lnv_cg_ws* ws,
                           hipStream_t s) {
  if (!opts || opts->reset_period <= 0 || !(n_elec > 0.0) || k < 0) return LNV_EINVAL;
  LNV_TRY(check_cg(L, S, H, T, ws));
  const lnv_eval_ws& ev = ws->ev;
  const lnv_pattern* pl = L->pat;
  const lnv_pattern* ph = H->pat;
  const int64_t nv = pl->nnzb * 16;
  const int ni = pl->n_items;
  const int64_t slot = slot_len(partial_items(pl));
  double* part = ev.partials;
  double* sc = ev.scalars;
  double* Lv = static_cast<double*>(L->val);
  const bool metric = T != nullptr;
  StageArgs sa{};
  sa.n_elec = n_elec;
  sa.n_tol = opts->n_tol;
  sa.step_cap = opts->step_cap;
  sa.reset = (k % opts->reset_period) == 0;
  sa.k = (int)k;
  sa.reset_period = opts->reset_period;

  // 1. E, N, G, F (FP64, or FP32 products); metric gradients G_c, F_c; mu
  // k > 0: L is the previous step's result, whose S.L and S.L.S that step
  // left in SL2 and Z (ev.carry set, and cleared by any other call that
  // writes them); formed afresh at the resets (k % reset_period == 0) so
  // that the rounding of the carried sums does not build up
  const bool carry = k > 0 && k % opts->reset_period != 0 && ev.carry != 0;
  ws->ev.carry = 0;   // until this step has left S.L and S.L.S of its final L
  if (opts->eval32) {
    const lnv_eval32_ws* w32 = opts->eval32;
    lnv_bsm Gm{pl, 4, LNV_F64, ws->G}, Fm{pl, 4, LNV_F64, ws->F};
    LNV_TRY(check_eval32(L, S, H, &Gm, &Fm, w32));
    if (w32->SL.pat != ev.SL.pat) return LNV_EPATTERN;
    lnv_bsm L32 = w32->L, S32 = w32->S, H32 = w32->H;
    LNV_TRY(convert_launch(L, &L32, s));
    LNV_TRY(convert_launch(S, &S32, s));
    LNV_TRY(convert_launch(H, &H32, s));
    EvalOps o{&L32,     &S32,     &H32,         &w32->SL,     &w32->LS, &w32->X,
              &w32->XT, &w32->Z,  w32->perm_SL, w32->perm_X,  w32->YT,  w32->W,
              w32->V,   part,     sc,           &w32->Zu,     &w32->Lu, w32->Vu};
    LNV_TRY(eval_products<float>(L, o, ws->G, ws->F, nullptr, s));
    // S.L in FP64 for the line search: the carried one, else the FP32 product widened
    if (carry) {
      LNV_HIP(hipMemcpyAsync(ev.SL.val, ws->SL2, sizeof(double) * (size_t)ev.SL.pat->nnzb * 16,
                             hipMemcpyDeviceToDevice, s));
    } else {
      lnv_bsm SL64 = ev.SL;
      LNV_TRY(convert_launch(&w32->SL, &SL64, s));
    }
  } else {
    LNV_TRY(eval_core(L, S, H, ws->G, ws->F, nullptr, &ev, s, carry ? ws->SL2 : nullptr, carry));
  }
  // occupation bounds of L S for the runaway guard (every occ_every-th step)
  if (opts->occ_every > 0 && ws->lanczos && k % opts->occ_every == 0) {
    const int steps = opts->occ_iter > 0 ? (opts->occ_iter < 64 ? opts->occ_iter : 64) : 16;
    LNV_TRY(occupation_bounds(L, S, steps, ws->lanczos, sc + LNV_SC_OCC_MIN, s));
    sa.occ_checked = 1;
  }
  const double* Gc = ws->G;
  const double* Fc = ws->F;
  double* gcur = ws->g;
  if (metric) {
    int st = LNV_EUNSUPPORTED;
    if (opts->eval32)
      st = metric_apply_pair32(T, ws->G, ws->Gc, ws->F, ws->Fc, ws, opts->eval32, s);
    if (st == LNV_EUNSUPPORTED)
      LNV_TRY(metric_apply_pair(T, ws->G, ws->Gc, ws->F, ws->Fc, ws, s));
    else
      LNV_TRY(st);
    Gc = ws->Gc;
    Fc = ws->Fc;
    gcur = ws->gc;
    k_vec_metric_dots<<<kVecGrid, 256, 0, s>>>(nv, ws->G, ws->F, ws->Fc, part, Seg{});
    LNV_LAUNCH_CHECK();
    RedList rl = reds();
    add(rl, 0, kVecGrid, 1, LNV_SC_FF);
    add(rl, kVecGrid, kVecGrid, 1, LNV_SC_GF);
    add(rl, 2 * kVecGrid, kVecGrid, 1, LNV_SC_FCFC);
    LNV_TRY(scalar_stage(part, rl, sc, ST_MU, sa, s));
  }
  // 2-3. g = G - mu F, g_c = G_c - mu F_c, Polak-Ribiere beta with resets
  k_vec_g<<<kVecGrid, 256, 0, s>>>(nv, ws->G, ws->F, Gc, Fc, ws->gc_prev, sc, ws->g,
                                   metric ? ws->gc : nullptr, part, Seg{});
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0, kVecGrid, 1, LNV_SC_GG);
    add(rl, kVecGrid, kVecGrid, 1, LNV_SC_GGP);
    add(rl, 2 * kVecGrid, kVecGrid, 1, LNV_SC_GGN);
    LNV_TRY(scalar_stage(part, rl, sc, ST_BETA, sa, s));
  }
  // 4. D = -g_c + beta D_prev, projected: D <- D - (<D,F>/<F,F_c>) F_c
  k_vec_dir<<<kVecGrid, 256, 0, s>>>(nv, gcur, ws->D_prev, ws->F, sc, ws->D, part, Seg{});
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0, kVecGrid, 1, LNV_SC_DF);
    LNV_TRY(scalar_stage(part, rl, sc, ST_PROJ, sa, s));
  }
  k_vec_proj<<<kVecGrid, 256, 0, s>>>(nv, Fc, ws->g, sc, ws->D, part, Seg{});
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0, kVecGrid, 1, LNV_SC_C1);
    LNV_TRY(scalar_stage(part, rl, sc, ST_NONE, sa, s));
  }
  // 5. exact cubic line minimisation of E - mu N along D
  k_hprime<<<ph->n_items, 256, 0, s>>>(ph->n, ph->items, ph->row_ptr, ph->col,
                                       static_cast<const double*>(H->val), make_ix(S->pat),
                                       static_cast<const double*>(S->val), sc, ws->Hp, Seg{});
  LNV_LAUNCH_CHECK();
  lnv_bsm Hp{ph, 4, LNV_F64, ws->Hp};
  lnv_bsm XD{ev.X.pat, 4, LNV_F64, ev.X.val};
  lnv_bsm XDT{ev.XT.pat, 4, LNV_F64, ev.XT.val};
  TraceParts tp{};
  LNV_TRY(cubic_traces(L, S, &Hp, false, ws->D, ev, ws->SL2, static_cast<double*>(ev.LS.val),
                       &ev.SL, XD, &XDT, part, slot, nullptr, &tp, s));
  {
    RedList rl = reds();
    for (int t = 0; t < 4; ++t) add(rl, tp.off[t], tp.n[t], tp.stride[t], LNV_SC_T0 + t);
    LNV_TRY(scalar_stage(part, rl, sc, ST_ALPHA, sa, s));
  }
  k_vec_axpy<<<kVecGrid, 256, 0, s>>>(nv, ws->D, sc, LNV_SC_ALPHA, nullptr, Lv, Seg{});
  LNV_LAUNCH_CHECK();
  // 6. electron number at the new L; cubic correction along F_c when needed
  lnv_bsm SL2{ev.SL.pat, 4, LNV_F64, ws->SL2};
  lnv_bsm Vm{pl, 4, LNV_F64, ev.V};
  const int64_t nsl = ev.SL.pat->nnzb * 16;
  if (opts->eval32 && !carry) {
    // the FP64 S.L of this step was widened from an FP32 product
    LNV_TRY(multiply_launch(1.0, S, L, 0, 0.0, &SL2, 1, nullptr, nullptr, nullptr, nullptr, s));
  } else {
    // S.L_new = S.L + alpha S.D: this step's FP64 S.L and the line search's
    // S.D, which it left in SL2
    k_vec_xpay<<<kVecGrid, 256, 0, s>>>(nsl, static_cast<const double*>(ev.SL.val), sc,
                                        LNV_SC_ALPHA, ws->SL2);
    LNV_LAUNCH_CHECK();
  }
  LNV_TRY(transpose_launch(&SL2, ev.perm_SL, static_cast<double*>(ev.LS.val), s));
  lnv_bsm Vu{ev.Lu.pat, 4, LNV_F64, ev.Vu};
  LNV_TRY(sym_product(S, &ev.LS, &ev.Z, &ev.Zu, s));
  LNV_TRY(sym_product(&SL2, &ev.Z, &Vm, &Vu, s));
  k_nassemble<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, Lv, make_ix(ev.Z.pat),
                                 static_cast<const double*>(ev.Z.val), ev.V, Fc, part);
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0 * (int64_t)ni, ni, 1, LNV_SC_T0);
    add(rl, 1 * (int64_t)ni, ni, 1, LNV_SC_T1);
    add(rl, 2 * (int64_t)ni, ni, 1, LNV_SC_T2);
    add(rl, 3 * (int64_t)ni, ni, 1, LNV_SC_LL);
    LNV_TRY(scalar_stage(part, rl, sc, ST_NCHK, sa, s));
  }
  const double* skip = sc + LNV_SC_SKIP_NCORR;
  // the old S.L buffer (ev.SL) is free now: A_F^T = S F_c goes there (A_F in
  // ev.LS), the products with A_new use S.L_new in SL2, and Z_F = S F_c S
  // reuses X's buffer.
  lnv_bsm ZF{ev.Z.pat, 4, LNV_F64, ev.X.val};
  LNV_TRY(cubic_traces(L, S, S, true, Fc, ev, static_cast<double*>(ev.SL.val),
                       static_cast<double*>(ev.LS.val), &SL2, ZF, nullptr, part, slot, skip, &tp,
                       s));
  {
    RedList rl = reds();
    for (int t = 0; t < 4; ++t) add(rl, tp.off[t], tp.n[t], tp.stride[t], LNV_SC_T0 + t);
    // the reductions read stale partials when skipped; ST_DELTA ignores them
    LNV_TRY(scalar_stage(part, rl, sc, ST_DELTA, sa, s));
  }
  k_vec_axpy<<<kVecGrid, 256, 0, s>>>(nv, Fc, sc, LNV_SC_DELTA, skip, Lv, Seg{});
  LNV_LAUNCH_CHECK();
  // S.L and S.L.S of the final L for the next step: + delta S.F_c (A_F^T,
  // in ev.SL) and + delta S.F_c.S (Z_F, in X's buffer)
  k_vec_axpy<<<kVecGrid, 256, 0, s>>>(nsl, static_cast<const double*>(ev.SL.val), sc,
                                      LNV_SC_DELTA, skip, ws->SL2, Seg{});
  LNV_LAUNCH_CHECK();
  k_vec_axpy<<<kVecGrid, 256, 0, s>>>(ev.Z.pat->nnzb * 16, static_cast<const double*>(ev.X.val),
                                      sc, LNV_SC_DELTA, skip, static_cast<double*>(ev.Z.val), Seg{});
  LNV_LAUNCH_CHECK();
  if (metric)
    std::swap(ws->gc, ws->gc_prev);
  else
    std::swap(ws->g, ws->gc_prev);
  std::swap(ws->D, ws->D_prev);
  ws->ev.carry = 1;
  return LNV_OK;
}

// ------------------------------------------------------------------ batches of cells
namespace {


// The traces T0..T3 of cubic_traces for a batch: every product is stored
// and traced per work item of L's pattern (k_dot_items), so each partial
// belongs to one cell (a fused trace partial of the multiply covers a piece
// of a row cluster, which may straddle two cells).  T0 = <P, X_P>,
// Q = P_L(A_P^T X_P^T) = P_L(S P S P M): T1 = <L, Q>, T2 = <P, Q>;
// T3 = <P, P_L(S L X_P^T)> = Tr[P S L S P M] (T3 = T1 when M = S).
// Partials: T_t at partials + t * slot, one per item.
int cubic_traces_batch(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* M, bool m_is_s,
                       const double* P, const lnv_eval_ws& ev, double* apt, double* ap,
                       const lnv_bsm* SLcur, lnv_bsm XP, const lnv_bsm* XPT, double* partials,
                       int64_t slot, hipStream_t s) {
  const lnv_pattern* pl = L->pat;
  const int ni = pl->n_items;
  lnv_bsm Pm{pl, 4, LNV_F64, const_cast<double*>(P)};
  lnv_bsm APT{ev.SL.pat, 4, LNV_F64, apt};
  lnv_bsm AP{ev.LS.pat, 4, LNV_F64, ap};
  LNV_TRY(multiply_launch(1.0, S, &Pm, 0, 0.0, &APT, 1, nullptr, nullptr, nullptr, nullptr, s));
  LNV_TRY(transpose_launch(&APT, ev.perm_SL, ap, s));
  LNV_TRY(multiply_launch(1.0, M, &AP, 0, 0.0, &XP, 1, nullptr, nullptr, nullptr, nullptr, s));
  const lnv_bsm* B = &XP;
  if (!m_is_s) {
    if (!XPT || !SLcur) return LNV_EINVAL;
    LNV_TRY(transpose_launch(&XP, ev.perm_X, static_cast<double*>(XPT->val), s));
    B = XPT;
  }
  const Ix lx = make_ix(pl);
  k_dot_items<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, P, make_ix(XP.pat),
                                 0, static_cast<const double*>(XP.val), partials, nullptr);
  LNV_LAUNCH_CHECK();
  lnv_bsm Q{pl, 4, LNV_F64, ev.YT};
  LNV_TRY(multiply_launch(1.0, &APT, B, 0, 0.0, &Q, 1, nullptr, nullptr, nullptr, nullptr, s));
  k_dot_items<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col,
                                 static_cast<const double*>(L->val), lx, 1,
                                 static_cast<const double*>(ev.YT), partials + 1 * slot, nullptr);
  LNV_LAUNCH_CHECK();
  k_dot_items<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, P, lx, 1,
                                 static_cast<const double*>(ev.YT), partials + 2 * slot, nullptr);
  LNV_LAUNCH_CHECK();
  if (m_is_s) return LNV_OK;
  lnv_bsm R{pl, 4, LNV_F64, ev.W};
  LNV_TRY(multiply_launch(1.0, SLcur, B, 0, 0.0, &R, 1, nullptr, nullptr, nullptr, nullptr, s));
  k_dot_items<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, P, lx, 1,
                                 static_cast<const double*>(ev.W), partials + 3 * slot, nullptr);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

// Reductions T0..T3 of cubic_traces_batch (T3 from T1's partials when M = S).
RedList batch_trace_reds(int ni, int64_t slot, bool m_is_s) {
  RedList rl = reds();
  add(rl, 0, ni, 1, LNV_SC_T0, 0, RK_ITEMS);
  add(rl, 1 * slot, ni, 1, LNV_SC_T1, 0, RK_ITEMS);
  add(rl, 2 * slot, ni, 1, LNV_SC_T2, 0, RK_ITEMS);
  add(rl, (m_is_s ? 1 : 3) * slot, ni, 1, LNV_SC_T3, 0, RK_ITEMS);
  return rl;
}

int check_batch_cg(const lnv_bsm* L, const lnv_bsm* S, const lnv_batch* b, lnv_cg_ws* ws) {
  if (!bsm_ok(L) || !bsm_ok(S) || !ws) return LNV_EINVAL;
  if (L->blk != 4 || S->blk != 4) return LNV_EUNSUPPORTED;
  LNV_TRY(check_batch(b, L->pat));
  const lnv_eval_ws& ev = ws->ev;
  if (!ev.partials || !ws->D || !ws->D_prev || !ws->gc_prev || !ws->SL2 || !ev.YT || !ev.W)
    return LNV_EINVAL;
  if (!bsm_ok(&ev.SL) || !bsm_ok(&ev.LS) || !bsm_ok(&ev.X) || !bsm_ok(&ev.Z) || !ev.perm_SL)
    return LNV_EINVAL;
  if (!pattern_ready(L->pat, true, false, true) || !pattern_ready(ev.SL.pat, false, false, true) ||
      !pattern_ready(ev.LS.pat, true, false, false) || !pattern_ready(ev.Z.pat, true, false, true) ||
      !pattern_ready(S->pat, true, false, false))
    return LNV_EPATTERN;
  if (ev.partials_len < lnv_partials_len(partial_items(L->pat))) return LNV_EINVAL;
  return LNV_OK;
}

}  // namespace

extern "C" int lnv_hotelling_batch(const lnv_bsm* S, lnv_bsm* T, int32_t n_iter,
                                   const lnv_batch* b, lnv_cg_ws* ws, hipStream_t s) {
  if (!T || !bsm_ok(T)) return LNV_EINVAL;
  LNV_TRY(check_batch(b, T->pat));
  return hotelling_impl(S, T, n_iter, ws, b->scalars, make_seg(b), s);
}

extern "C" int lnv_pm_start_batch(lnv_bsm* K, const lnv_bsm* T, const lnv_bsm* H, lnv_bsm* HT,
                                  const lnv_batch* b, lnv_pm_ws* ws, hipStream_t s) {
  if (!K || !bsm_ok(K)) return LNV_EINVAL;
  LNV_TRY(check_batch(b, K->pat));
  Seg sg = make_seg(b);
  sg.sc_stride = LNV_PM_NSCALARS;
  return pm_start_impl(K, T, H, HT, 0.0, 0.0, ws, sg, s);
}

extern "C" int lnv_pm_step_batch(lnv_bsm* K, const lnv_bsm* S, const lnv_batch* b, double tol,
                                 lnv_pm_ws* ws, hipStream_t s) {
  if (!K || !bsm_ok(K)) return LNV_EINVAL;
  LNV_TRY(check_batch(b, K->pat));
  Seg sg = make_seg(b);
  sg.sc_stride = LNV_PM_NSCALARS;
  return pm_step_impl(K, S, 0.0, tol, ws, sg, s);
}

extern "C" int lnv_cg_init_batch(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* T,
                                 const lnv_batch* b, lnv_cg_ws* ws, hipStream_t s) {
  LNV_TRY(check_batch_cg(L, S, b, ws));
  if (T && (!bsm_ok(T) || T->pat != L->pat || T->blk != 4)) return LNV_EPATTERN;
  const lnv_eval_ws& ev = ws->ev;
  ws->ev.carry = 0;
  const lnv_pattern* pl = L->pat;
  const int64_t nv = pl->nnzb * 16;
  const int ni = pl->n_items;
  const int64_t slot = slot_len(partial_items(pl));
  const Seg sg = make_seg(b);
  double* part = ev.partials;
  double* sc = b->scalars;
  // every cell's scalars but its sigma (from lnv_hotelling_batch) start at zero
  k_clear_scalars<<<b->n_cells, 64, 0, s>>>(sc, LNV_NSCALARS, LNV_SC_SIGMA);
  LNV_LAUNCH_CHECK();
  LNV_HIP(hipMemsetAsync(ws->gc_prev, 0, sizeof(double) * nv, s));
  LNV_HIP(hipMemsetAsync(ws->D_prev, 0, sizeof(double) * nv, s));
  LNV_HIP(hipMemsetAsync(L->val, 0, sizeof(double) * nv, s));
  if (T) {
    LNV_HIP(hipMemcpyAsync(ws->D, T->val, sizeof(double) * nv, hipMemcpyDeviceToDevice, s));
  } else {
    k_identity<<<ni, 256, 0, s>>>(pl->n, pl->items, pl->row_ptr, pl->col, make_ix(S->pat),
                                  static_cast<const double*>(S->val), nullptr, 0, ws->D, sg);
    LNV_LAUNCH_CHECK();
  }
  // per cell: N(lambda P) = 6 Tr[PSPS] lambda^2 - 4 Tr[PSPSPS] lambda^3 at L = 0, P = T or I
  lnv_bsm ZD{ev.Z.pat, 4, LNV_F64, ev.Z.val};
  LNV_TRY(cubic_traces_batch(L, S, S, true, ws->D, ev, ws->SL2, static_cast<double*>(ev.LS.val),
                             nullptr, ZD, nullptr, part, slot, s));
  StageArgs sa{};
  LNV_TRY(scalar_stage(part, batch_trace_reds(ni, slot, true), sc, ST_INIT, sa, s, sg));
  k_vec_axpy<<<seg_grid(sg), 256, 0, s>>>(nv, ws->D, sc, LNV_SC_LAMBDA, nullptr,
                                          static_cast<double*>(L->val), sg);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_cg_step_batch(lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H,
                                 const lnv_bsm* T, const lnv_batch* b, int64_t k,
                                 const lnv_opts* opts, lnv_cg_ws* ws, hipStream_t s) {
  if (!opts || opts->reset_period <= 0 || k < 0) return LNV_EINVAL;
  if (opts->eval32) return LNV_EUNSUPPORTED;
  LNV_TRY(check_batch_cg(L, S, b, ws));
  LNV_TRY(check_cg(L, S, H, T, ws));
  const lnv_eval_ws& ev = ws->ev;
  const lnv_pattern* pl = L->pat;
  const lnv_pattern* ph = H->pat;
  const int64_t nv = pl->nnzb * 16;
  const int ni = pl->n_items;
  const int64_t slot = slot_len(partial_items(pl));
  const Seg sg = make_seg(b);
  const int vg = seg_grid(sg);
  const bool metric = T != nullptr;
  double* part = ev.partials;
  double* sc = b->scalars;
  double* Lv = static_cast<double*>(L->val);
  StageArgs sa{};
  sa.n_tol = opts->n_tol;
  sa.step_cap = opts->step_cap;
  sa.reset = (k % opts->reset_period) == 0;
  sa.k = (int)k;
  sa.reset_period = opts->reset_period;
  ws->ev.carry = 0;   // S.L and S.L.S are formed afresh every step here
  // 1. per cell E, N, G, F; metric gradients G_c = P_L(T G T), F_c = P_L(T F T);
  // mu = <G,F_c>/<F,F_c>
  LNV_TRY(eval_core(L, S, H, ws->G, ws->F, nullptr, &ev, s, nullptr, false, sc, sg));
  const double* Gc = ws->G;
  const double* Fc = ws->F;
  double* gcur = ws->g;
  if (metric) {
    LNV_TRY(metric_apply_pair(T, ws->G, ws->Gc, ws->F, ws->Fc, ws, s));
    Gc = ws->Gc;
    Fc = ws->Fc;
    gcur = ws->gc;
    k_vec_metric_dots<<<vg, 256, 0, s>>>(nv, ws->G, ws->F, ws->Fc, part, sg);
    LNV_LAUNCH_CHECK();
    RedList rl = reds();
    add(rl, 0, vg, 1, LNV_SC_FF, 0, RK_VEC);
    add(rl, kVecGrid, vg, 1, LNV_SC_GF, 0, RK_VEC);
    add(rl, 2 * kVecGrid, vg, 1, LNV_SC_FCFC, 0, RK_VEC);
    LNV_TRY(scalar_stage(part, rl, sc, ST_MU, sa, s, sg));
  }
  // 2-3. g = G - mu F (g_c = G_c - mu F_c), PR+ beta per cell
  k_vec_g<<<vg, 256, 0, s>>>(nv, ws->G, ws->F, Gc, Fc, ws->gc_prev, sc, ws->g,
                             metric ? ws->gc : nullptr, part, sg);
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0, vg, 1, LNV_SC_GG, 0, RK_VEC);
    add(rl, kVecGrid, vg, 1, LNV_SC_GGP, 0, RK_VEC);
    add(rl, 2 * kVecGrid, vg, 1, LNV_SC_GGN, 0, RK_VEC);
    LNV_TRY(scalar_stage(part, rl, sc, ST_BETA, sa, s, sg));
  }
  // 4. D = -g_c + beta D_prev, projected on <D, F> = 0 along F_c
  k_vec_dir<<<vg, 256, 0, s>>>(nv, gcur, ws->D_prev, ws->F, sc, ws->D, part, sg);
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0, vg, 1, LNV_SC_DF, 0, RK_VEC);
    LNV_TRY(scalar_stage(part, rl, sc, ST_PROJ, sa, s, sg));
  }
  k_vec_proj<<<vg, 256, 0, s>>>(nv, Fc, ws->g, sc, ws->D, part, sg);
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0, vg, 1, LNV_SC_C1, 0, RK_VEC);
    LNV_TRY(scalar_stage(part, rl, sc, ST_NONE, sa, s, sg));
  }
  // 5. exact cubic line minimisation of E - mu N along D, per cell
  k_hprime<<<ph->n_items, 256, 0, s>>>(ph->n, ph->items, ph->row_ptr, ph->col,
                                       static_cast<const double*>(H->val), make_ix(S->pat),
                                       static_cast<const double*>(S->val), sc, ws->Hp, sg);
  LNV_LAUNCH_CHECK();
  lnv_bsm Hp{ph, 4, LNV_F64, ws->Hp};
  lnv_bsm XD{ev.X.pat, 4, LNV_F64, ev.X.val};
  lnv_bsm XDT{ev.XT.pat, 4, LNV_F64, ev.XT.val};
  LNV_TRY(cubic_traces_batch(L, S, &Hp, false, ws->D, ev, ws->SL2,
                             static_cast<double*>(ev.LS.val), &ev.SL, XD, &XDT, part, slot, s));
  LNV_TRY(scalar_stage(part, batch_trace_reds(ni, slot, false), sc, ST_ALPHA, sa, s, sg));
  k_vec_axpy<<<vg, 256, 0, s>>>(nv, ws->D, sc, LNV_SC_ALPHA, nullptr, Lv, sg);
  LNV_LAUNCH_CHECK();
  // 6. electron number at the new L; the cubic correction along F_c per cell
  // (cells within tolerance keep delta = 0)
  lnv_bsm SL2{ev.SL.pat, 4, LNV_F64, ws->SL2};
  lnv_bsm Vm{pl, 4, LNV_F64, ev.V};
  lnv_bsm Vu{ev.Lu.pat, 4, LNV_F64, ev.Vu};
  LNV_TRY(multiply_launch(1.0, S, L, 0, 0.0, &SL2, 1, nullptr, nullptr, nullptr, nullptr, s));
  LNV_TRY(transpose_launch(&SL2, ev.perm_SL, static_cast<double*>(ev.LS.val), s));
  LNV_TRY(sym_product(S, &ev.LS, &ev.Z, &ev.Zu, s));
  LNV_TRY(sym_product(&SL2, &ev.Z, &Vm, &Vu, s));
  k_nassemble<<<ni, 256, 0, s>>>(pl->n, ni, pl->items, pl->row_ptr, pl->col, Lv, make_ix(ev.Z.pat),
                                 static_cast<const double*>(ev.Z.val), ev.V, Fc, part);
  LNV_LAUNCH_CHECK();
  {
    RedList rl = reds();
    add(rl, 0 * (int64_t)ni, ni, 1, LNV_SC_T0, 0, RK_ITEMS);
    add(rl, 1 * (int64_t)ni, ni, 1, LNV_SC_T1, 0, RK_ITEMS);
    add(rl, 2 * (int64_t)ni, ni, 1, LNV_SC_T2, 0, RK_ITEMS);
    add(rl, 3 * (int64_t)ni, ni, 1, LNV_SC_LL, 0, RK_ITEMS);
    LNV_TRY(scalar_stage(part, rl, sc, ST_NCHK, sa, s, sg));
  }
  lnv_bsm ZF{ev.Z.pat, 4, LNV_F64, ev.X.val};
  LNV_TRY(cubic_traces_batch(L, S, S, true, Fc, ev, static_cast<double*>(ev.SL.val),
                             static_cast<double*>(ev.LS.val), nullptr, ZF, nullptr, part, slot,
                             s));
  LNV_TRY(scalar_stage(part, batch_trace_reds(ni, slot, true), sc, ST_DELTA, sa, s, sg));
  k_vec_axpy<<<vg, 256, 0, s>>>(nv, Fc, sc, LNV_SC_DELTA, nullptr, Lv, sg);
  LNV_LAUNCH_CHECK();
  if (metric)
    std::swap(ws->gc, ws->gc_prev);
  else
    std::swap(ws->g, ws->gc_prev);
  std::swap(ws->D, ws->D_prev);
  return LNV_OK;
}

extern "C" int lnv_bsm_transpose(const lnv_bsm* A, const int32_t* perm, lnv_bsm* AT,
                                 hipStream_t s) {
  if (!bsm_ok_any(A) || !bsm_ok_any(AT) || !perm) return LNV_EINVAL;
  if (A->blk != 4 || AT->blk != 4 || A->dtype != AT->dtype) return LNV_EUNSUPPORTED;
  if (A->pat->n != AT->pat->n || A->pat->nnzb != AT->pat->nnzb || !A->pat->items ||
      !A->pat->row_ptr)
    return LNV_EPATTERN;
  return transpose_launch(A, perm, AT->val, s);
}
