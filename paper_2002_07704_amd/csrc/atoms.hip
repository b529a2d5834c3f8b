// Atoms with their own number of support functions (Sec. II.B): the layout of
// atom blocks in 4x4-blocked stored rows, and the conversion between
// variable-size atom blocks and that storage.
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace lnv {
namespace {

constexpr int kMaxFun = 64;  // largest support-function count of one atom

// Row positions: the position of each stored row's atom.
__global__ void k_rows_pos(int n_rows, const int* __restrict__ atom_of,
                           const double* __restrict__ atom_pos, double* __restrict__ row_pos) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rows) return;
  const int a = atom_of[r];
#pragma unroll
  for (int d = 0; d < 3; ++d) row_pos[3 * r + d] = atom_pos[3 * a + d];
}

// Pack: one workgroup per stored row r of B, threads over (block, element).  Element
// (s, t) of stored block (r, c) is element (off_of[r] + s, off_of[c] + t) of
// atom block (atom_of[r], atom_of[c]) of A, zero past either atom's functions
// or when A has no such block.
template <typename T>
__global__ void k_pack(int n_rows, const int* __restrict__ b_rp, const int* __restrict__ b_col,
                       T* __restrict__ b_val, const int* __restrict__ a_rp,
                       const int* __restrict__ a_col, const long long* __restrict__ a_off,
                       const T* __restrict__ a_val, const int* __restrict__ nfun,
                       const int* __restrict__ atom_of, const int* __restrict__ off_of) {
  const int r = blockIdx.x;
  if (r >= n_rows) return;
  const int i = atom_of[r], oi = off_of[r], ni = nfun[i];
  const int q0 = b_rp[r], q1 = b_rp[r + 1];
  const int a0 = a_rp[i], a1 = a_rp[i + 1];
  for (int e = threadIdx.x; e < (q1 - q0) * 16; e += blockDim.x) {
    const int q = q0 + e / 16, s = (e % 16) / 4, t = e % 4;
    const int c = b_col[q];
    const int j = atom_of[c], oj = off_of[c], nj = nfun[j];
    T v = 0;
    if (oi + s < ni && oj + t < nj) {
      // binary search for atom j in A's row i
      int lo = a0, hi = a1;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a_col[mid] < j) lo = mid + 1;
        else hi = mid;
      }
      if (lo < a1 && a_col[lo] == j) v = a_val[a_off[lo] + (long long)(oi + s) * nj + (oj + t)];
    }
    b_val[(size_t)q * 16 + s * 4 + t] = v;
  }
}

// Unpack: one workgroup per atom row i of A, threads over (block, element).
// Element (x, y) of atom block (i, j) is element (x & 3, y & 3) of stored
// block (row_start[i] + x/4, row_start[j] + y/4) of B (zero when B has no
// such block).
template <typename T>
__global__ void k_unpack(int n_atoms, const int* __restrict__ a_rp, const int* __restrict__ a_col,
                         const long long* __restrict__ a_off, T* __restrict__ a_val,
                         const int* __restrict__ nfun, const int* __restrict__ row_start, Ix bx,
                         const T* __restrict__ b_val) {
  const int i = blockIdx.x;
  if (i >= n_atoms) return;
  const int ni = nfun[i], ri = row_start[i];
  for (int p = a_rp[i]; p < a_rp[i + 1]; ++p) {
    const int j = a_col[p], nj = nfun[j], rj = row_start[j];
    T* out = a_val + a_off[p];
    for (int e = threadIdx.x; e < ni * nj; e += blockDim.x) {
      const int x = e / nj, y = e % nj;
      const int pos = ix_find(bx, ri + x / 4, rj + y / 4);
      out[e] = pos < 0 ? T(0) : b_val[(size_t)pos * 16 + (x & 3) * 4 + (y & 3)];
    }
  }
}

bool vbsm_ok(const lnv_vbsm* A) {
  return A && A->atoms && A->row_ptr && A->col && A->val_off && A->val && A->nnz >= 0 &&
         (A->dtype == LNV_F64 || A->dtype == LNV_F32) && A->atoms->n_atoms > 0 &&
         A->atoms->nfun && A->atoms->row_start && A->atoms->atom_of && A->atoms->off_of;
}

}  // namespace
}  // namespace lnv

using namespace lnv;

extern "C" int lnv_atoms_layout(const int32_t* nfun, int32_t n_atoms, const int32_t* order,
                                int32_t* row_start, int32_t* atom_of, int32_t* off_of,
                                int64_t cap, int32_t* n_rows_out, hipStream_t s) {
  if (!nfun || n_atoms <= 0 || !row_start || !n_rows_out || cap < 0) return LNV_EINVAL;
  if ((atom_of == nullptr) != (off_of == nullptr)) return LNV_EINVAL;
  std::vector<int32_t> nf(n_atoms), ord(n_atoms);
  LNV_HIP(hipMemcpyAsync(nf.data(), nfun, sizeof(int32_t) * n_atoms, hipMemcpyDeviceToHost, s));
  if (order)
    LNV_HIP(hipMemcpyAsync(ord.data(), order, sizeof(int32_t) * n_atoms, hipMemcpyDeviceToHost,
                           s));
  LNV_HIP(hipStreamSynchronize(s));
  if (!order)
    for (int a = 0; a < n_atoms; ++a) ord[a] = a;
  std::vector<char> seen(n_atoms, 0);
  for (int q = 0; q < n_atoms; ++q) {
    const int a = ord[q];
    if (a < 0 || a >= n_atoms || seen[a]) return LNV_EINVAL;  // not a permutation
    seen[a] = 1;
    if (nf[a] < 1 || nf[a] > kMaxFun) return LNV_EUNSUPPORTED;
  }
  long long rows = 0;
  std::vector<int32_t> start(n_atoms + 1), ao, oo;
  for (int q = 0; q < n_atoms; ++q) {
    const int a = ord[q];
    start[a] = (int32_t)rows;
    rows += (nf[a] + 3) / 4;
  }
  if (rows > LNV_MAX_ATOMS) return LNV_EUNSUPPORTED;
  start[n_atoms] = (int32_t)rows;
  *n_rows_out = (int32_t)rows;
  if (atom_of) {
    if (cap < rows) return LNV_ECAPACITY;
    ao.resize(rows);
    oo.resize(rows);
    for (int q = 0; q < n_atoms; ++q) {
      const int a = ord[q];
      for (int u = 0; u < (nf[a] + 3) / 4; ++u) {
        ao[start[a] + u] = a;
        oo[start[a] + u] = 4 * u;
      }
    }
    LNV_HIP(hipMemcpyAsync(atom_of, ao.data(), sizeof(int32_t) * rows, hipMemcpyHostToDevice, s));
    LNV_HIP(hipMemcpyAsync(off_of, oo.data(), sizeof(int32_t) * rows, hipMemcpyHostToDevice, s));
  }
  LNV_HIP(hipMemcpyAsync(row_start, start.data(), sizeof(int32_t) * (n_atoms + 1),
                         hipMemcpyHostToDevice, s));
  LNV_HIP(hipStreamSynchronize(s));
  return LNV_OK;
}

extern "C" int lnv_atoms_rows(const lnv_atoms* A, const double* atom_pos, double* row_pos,
                              hipStream_t s) {
  if (!A || !A->atom_of || !atom_pos || !row_pos || A->n_rows <= 0) return LNV_EINVAL;
  k_rows_pos<<<(A->n_rows + 255) / 256, 256, 0, s>>>(A->n_rows, A->atom_of, atom_pos, row_pos);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_vbsm_offsets(const lnv_atoms* A, const int32_t* row_ptr, const int32_t* col,
                                int64_t nnz, int64_t* val_off, int64_t* len_out,
                                hipStream_t s) {
  if (!A || !A->nfun || A->n_atoms <= 0 || !row_ptr || (nnz > 0 && !col) || !val_off ||
      nnz < 0)
    return LNV_EINVAL;
  const int n = A->n_atoms;
  std::vector<int32_t> rp(n + 1), cl(nnz), nf(n);
  LNV_HIP(hipMemcpyAsync(rp.data(), row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
  if (nnz > 0)
    LNV_HIP(hipMemcpyAsync(cl.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
  LNV_HIP(hipMemcpyAsync(nf.data(), A->nfun, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
  LNV_HIP(hipStreamSynchronize(s));
  if (rp[0] != 0 || rp[n] != nnz) return LNV_EPATTERN;
  std::vector<int64_t> off(nnz + 1);
  int64_t o = 0;
  for (int i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return LNV_EPATTERN;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
      if (cl[p] < 0 || cl[p] >= n) return LNV_EPATTERN;
      off[p] = o;
      o += (int64_t)nf[i] * nf[cl[p]];
    }
  }
  off[nnz] = o;
  if (len_out) *len_out = o;
  LNV_HIP(hipMemcpyAsync(val_off, off.data(), sizeof(int64_t) * (nnz + 1), hipMemcpyHostToDevice,
                         s));
  LNV_HIP(hipStreamSynchronize(s));
  return LNV_OK;
}

extern "C" int lnv_vbsm_pack(const lnv_vbsm* A, lnv_bsm* B, hipStream_t s) {
  if (!vbsm_ok(A) || !bsm_ok_any(B)) return LNV_EINVAL;
  if (B->blk != 4 || B->dtype != A->dtype) return LNV_EUNSUPPORTED;
  const lnv_pattern* pb = B->pat;
  if (!pb->row_ptr || !pb->col || pb->n != A->atoms->n_rows) return LNV_EPATTERN;
  const lnv_atoms* at = A->atoms;
  if (A->dtype == LNV_F64)
    k_pack<double><<<pb->n, 256, 0, s>>>(pb->n, pb->row_ptr, pb->col, static_cast<double*>(B->val),
                                         A->row_ptr, A->col,
                                         reinterpret_cast<const long long*>(A->val_off),
                                         static_cast<const double*>(A->val), at->nfun,
                                         at->atom_of, at->off_of);
  else
    k_pack<float><<<pb->n, 256, 0, s>>>(pb->n, pb->row_ptr, pb->col, static_cast<float*>(B->val),
                                        A->row_ptr, A->col,
                                        reinterpret_cast<const long long*>(A->val_off),
                                        static_cast<const float*>(A->val), at->nfun, at->atom_of,
                                        at->off_of);
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}

extern "C" int lnv_vbsm_unpack(const lnv_bsm* B, lnv_vbsm* A, hipStream_t s) {
  if (!vbsm_ok(A) || !bsm_ok_any(B)) return LNV_EINVAL;
  if (B->blk != 4 || B->dtype != A->dtype) return LNV_EUNSUPPORTED;
  const lnv_pattern* pb = B->pat;
  if (!has_ix(pb) || pb->n != A->atoms->n_rows) return LNV_EPATTERN;
  const lnv_atoms* at = A->atoms;
  const Ix bx = make_ix(pb);
  if (A->dtype == LNV_F64)
    k_unpack<double><<<at->n_atoms, 256, 0, s>>>(
        at->n_atoms, A->row_ptr, A->col, reinterpret_cast<const long long*>(A->val_off),
        static_cast<double*>(A->val), at->nfun, at->row_start, bx,
        static_cast<const double*>(B->val));
  else
    k_unpack<float><<<at->n_atoms, 256, 0, s>>>(
        at->n_atoms, A->row_ptr, A->col, reinterpret_cast<const long long*>(A->val_off),
        static_cast<float*>(A->val), at->nfun, at->row_start, bx,
        static_cast<const float*>(B->val));
  LNV_LAUNCH_CHECK();
  return LNV_OK;
}
