// Adjoint of the LNV energy: dE/dH and dE/dS at a given L.
//
// Sec. II.C.2 writes the density matrix as K = 3LSL - 2LSLSL (Eq. 4) and the
// band energy as E = 2 Tr[KH].  Differentiating each stored entry of H and of
// S (L, S, H symmetric) gives
//   dE/dH = 2 K                           on H's pattern,
//   dE/dS = 2 [3 LHL - 2 (LSLHL + LHLSL)] on S's pattern.
// Both are formed from natural-range intermediates that are recomputed here
// rather than kept from the evaluation (SL = S.L, LSL = L.SL, HL = H.L):
//   dE/dH = P_H(6 L.SL - 4 LSL.SL)
//   dE/dS = P_S(6 L.HL) - 4 (Y + Y^T),   Y = P_S(LSL.HL),  Y^T = P_S(LHLSL)
// and, for forces at a constrained minimum, the electron-number derivative
//   dN/dS = 12 (LSL - LSLSL) = P_S(12 L.SL - 12 LSL.SL)   (N = 2 Tr[KS])
// so every product reads its right operand in stored orientation and the
// transposed term costs one gather on S's own (symmetric) pattern.  LSL, the
// two-term symmetric combinations of dH and dN/dS and L.HL are formed from
// the blocks of their symmetric halves when the workspace provides the
// buffers.  With the transposes LS = (SL)^T and LH = (HL)^T in the workspace,
// the restricted products with the long-range L.S.L are taken with it on the
// right: P(LS.LSL) (the same L S L S L as LSL.SL) and Y^T = P_S(LH.LSL) (dS
// needs only Y + Y^T).  The contraction then runs over the rows of LS or LH
// (ranges R_L + R_S, R_L + R_H) instead of those of L.S.L (2 R_L + R_S),
// and nearly every lane of a 64-column piece finds its block.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace lnv {
namespace {

// dS_p += c (Y_p + Y_q^T), q = position of block (j, i) in S's pattern.
// Workgroup per item of S's pattern: 64 blocks, 4 threads per block, thread
// (b, r) owns row r of block b.
__global__ __launch_bounds__(256) void k_sym_update(int n, const int* __restrict__ items,
                                                    const int* __restrict__ rp,
                                                    const int* __restrict__ col,
                                                    Ix x,
                                                    const double* __restrict__ Y, double c,
                                                    double* __restrict__ dS) {
  const int item = blockIdx.x;
  const int i = items[2 * item], c0 = items[2 * item + 1];
  const int cnt = min(kWave, rp[i + 1] - c0);
  const int b = threadIdx.x >> 2, r = threadIdx.x & 3;
  if (b >= cnt) return;
  const int p = c0 + b;
  const int q = ix_find(x, col[p], i);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double yt = q >= 0 ? Y[(size_t)q * 16 + k * 4 + r] : 0.0;
    const size_t e = (size_t)p * 16 + r * 4 + k;
    dS[e] = fma(c, Y[e] + yt, dS[e]);
  }
}

bool has(const lnv_pattern* p, bool lut, bool items) {
  return p && p->row_ptr && p->col && (!lut || has_ix(p)) && (!items || p->items);
}

int check_adjoint(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, const lnv_bsm* dS,
                  const lnv_bsm* dH, const lnv_bsm* dNS, const lnv_adj_ws* ws) {
  if (!bsm_ok(L) || !bsm_ok(S) || !bsm_ok(H) || !ws) return LNV_EINVAL;
  if (!dS && !dH && !dNS) return LNV_EINVAL;
  if ((dS && !bsm_ok(dS)) || (dH && !bsm_ok(dH)) || (dNS && !bsm_ok(dNS))) return LNV_EINVAL;
  if (dNS && (dNS->blk != 4 || dNS->pat != S->pat || !has(S->pat, false, true)))
    return LNV_EPATTERN;
  if (!bsm_ok(&ws->SL) || !bsm_ok(&ws->LSL)) return LNV_EINVAL;
  if (dS && (!bsm_ok(&ws->HL) || !ws->YS)) return LNV_EINVAL;
  if (L->blk != 4 || S->blk != 4 || H->blk != 4 || ws->SL.blk != 4 || ws->LSL.blk != 4 ||
      (dS && (dS->blk != 4 || ws->HL.blk != 4)) || (dH && dH->blk != 4))
    return LNV_EUNSUPPORTED;
  const int n = L->pat->n;
  if (S->pat->n != n || H->pat->n != n || ws->SL.pat->n != n || ws->LSL.pat->n != n ||
      (dS && ws->HL.pat->n != n))
    return LNV_EPATTERN;
  if ((dS && dS->pat != S->pat) || (dH && dH->pat != H->pat)) return LNV_EPATTERN;
  if (!has(L->pat, true, false) || !has(S->pat, false, false) ||
      !has(ws->SL.pat, true, true) || !has(ws->LSL.pat, false, true))
    return LNV_EPATTERN;
  if (dS && (!has(S->pat, true, true) || !has(ws->HL.pat, true, true) ||
             !has(H->pat, false, false)))
    return LNV_EPATTERN;
  if (dH && !has(H->pat, false, true)) return LNV_EPATTERN;
  // optional transposes: checked only when given
  if (ws->LS.val) {
    if (!bsm_ok(&ws->LS) || !ws->perm_SL) return LNV_EINVAL;
    if (ws->LS.blk != 4) return LNV_EUNSUPPORTED;
    if (ws->LS.pat->n != n || !has(ws->LS.pat, false, false) || !has_ix(ws->LSL.pat))
      return LNV_EPATTERN;
  }
  if (ws->LH.val && dS) {
    if (!bsm_ok(&ws->LH) || !ws->perm_HL) return LNV_EINVAL;
    if (ws->LH.blk != 4) return LNV_EUNSUPPORTED;
    if (ws->LH.pat->n != n || !has(ws->LH.pat, false, false) || !has_ix(ws->LSL.pat))
      return LNV_EPATTERN;
  }
  return LNV_OK;
}

}  // namespace
}  // namespace lnv

using namespace lnv;

extern "C" int lnv_adjoint(const lnv_bsm* L, const lnv_bsm* S, const lnv_bsm* H, lnv_bsm* dS,
                           lnv_bsm* dH, lnv_bsm* dNS, const lnv_adj_ws* ws, hipStream_t s) {
  LNV_TRY(check_adjoint(L, S, H, dS, dH, dNS, ws));
  const bool use_ls = ws->LS.val != nullptr;
  const bool use_lh = ws->LH.val != nullptr && dS != nullptr;
  LNV_TRY(multiply_launch(1.0, S, L, 0, 0.0, &ws->SL, 1, nullptr, nullptr, nullptr, nullptr, s));
  if (use_ls) LNV_TRY(transpose_values(&ws->SL, ws->perm_SL, ws->LS.val, s));
  // LSL = L S L is symmetric: the blocks of its half, then the mirror
  if (sym_ready(&ws->LSLu, &ws->LSL)) {
    LNV_TRY(multiply_launch(1.0, L, &ws->SL, 0, 0.0, &ws->LSLu, 1, nullptr, nullptr, nullptr,
                            nullptr, s));
    LNV_TRY(mirror_launch(&ws->LSLu, &ws->LSL, s));
  } else {
    LNV_TRY(multiply_launch(1.0, L, &ws->SL, 0, 0.0, &ws->LSL, 1, nullptr, nullptr, nullptr,
                            nullptr, s));
  }
  // a L.SL + b LSL.SL on the symmetric output pattern of D (= a LSL + b LSLSL)
  auto two_terms = [&](double a, double b, lnv_bsm* D, const lnv_bsm* U) -> int {
    const lnv_bsm* out = sym_ready(U, D) ? U : D;
    if (use_ls)
      LNV_TRY(multiply_launch(b, &ws->LS, &ws->LSL, 0, 0.0, out, 1, nullptr, nullptr, nullptr,
                              nullptr, s));
    else
      LNV_TRY(multiply_launch(b, &ws->LSL, &ws->SL, 0, 0.0, out, 1, nullptr, nullptr, nullptr,
                              nullptr, s));
    LNV_TRY(multiply_launch(a, L, &ws->SL, 0, 1.0, out, 1, nullptr, nullptr, nullptr, nullptr,
                            s));
    return out == U ? mirror_launch(U, D, s) : LNV_OK;
  };
  if (dH) LNV_TRY(two_terms(6.0, -4.0, dH, &ws->Hu));
  if (dNS) LNV_TRY(two_terms(12.0, -12.0, dNS, &ws->Su));
  if (dS) {
    const lnv_pattern* ps = S->pat;
    lnv_bsm Y{ps, 4, LNV_F64, ws->YS};
    LNV_TRY(multiply_launch(1.0, H, L, 0, 0.0, &ws->HL, 1, nullptr, nullptr, nullptr, nullptr, s));
    if (use_lh) {
      // Y^T = P_S(LH.LSL): k_sym_update takes Y + Y^T either way
      LNV_TRY(transpose_values(&ws->HL, ws->perm_HL, ws->LH.val, s));
      LNV_TRY(multiply_launch(1.0, &ws->LH, &ws->LSL, 0, 0.0, &Y, 1, nullptr, nullptr, nullptr,
                              nullptr, s));
    } else {
      LNV_TRY(multiply_launch(1.0, &ws->LSL, &ws->HL, 0, 0.0, &Y, 1, nullptr, nullptr, nullptr,
                              nullptr, s));
    }
    // 6 L H L is symmetric; Y = LSLHL is not
    if (sym_ready(&ws->Su, dS)) {
      LNV_TRY(multiply_launch(6.0, L, &ws->HL, 0, 0.0, &ws->Su, 1, nullptr, nullptr, nullptr,
                              nullptr, s));
      LNV_TRY(mirror_launch(&ws->Su, dS, s));
    } else {
      LNV_TRY(multiply_launch(6.0, L, &ws->HL, 0, 0.0, dS, 1, nullptr, nullptr, nullptr, nullptr,
                              s));
    }
    if (ps->n_items > 0) {
      k_sym_update<<<ps->n_items, 256, 0, s>>>(ps->n, ps->items, ps->row_ptr, ps->col, make_ix(ps),
                                               ws->YS, -4.0, static_cast<double*>(dS->val));
      LNV_LAUNCH_CHECK();
    }
  }
  return LNV_OK;
}
