"""Geometry, range patterns and synthetic matrices for the oracle.

Test infrastructure only (see the package docstring).

Range rule (Sec. II.C.2): a matrix element A_{ia,jb} is kept only when the
distance between atoms i and j does not exceed the cutoff R_c of that matrix.
Under periodic boundary conditions (Sec. II.C.1) the distance is taken to the
nearest periodic image, computed per axis as

    dx = (x_j - x_i) - box * rint((x_j - x_i) / box)
    d2 = (dx*dx + dy*dy) + dz*dz            (left to right, no fused multiply-add)

and the pair is in range iff d2 <= R*R.  The pattern keeps (i, j) once even when
several images are within range; the synthetic matrix element sums over all of
them (Gamma-point folding of a translation-invariant operator).

Synthetic S and H replace the grid integrals of Eq. (2) (which need
pseudopotentials and basis sets that are not part of this work):

    S_ij = w_S(i,j) M^S_ij + 2 I delta_ij,   w_S = sum_T exp(-d_T / 3.0)
    H_ij = -(w_H(i,j) M^H_ij),               w_H = sum_T exp(-d_T / 2.5)

where the sums run over the periodic images T of j with d_T^2 <= R^2 (images
enumerated with integer offsets t in [-m, m]^3, tx outermost, m = ceil(R/box)+1),
and M_ij is a seeded random block: for i <= j, element e = r*n_j + c equals
scale*(u - 0.5) with u the SplitMix64 uniform of counter (stream, i, j, e);
M_ji = M_ij^T; diagonal blocks are symmetrised as (R + R^T) * 0.5.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

import lnv_workloads as W


# ---------------------------------------------------------------- patterns
def neighbours(pos, box, R, rows=None):
    """Brute-force CSR neighbour list: row_ptr [n+1], col (ascending, self kept).

    If `rows` is given, only those rows are built and a list of arrays is
    returned instead.
    """
    pos = np.asarray(pos, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    n = pos.shape[0]
    R2 = float(R) * float(R)
    want = range(n) if rows is None else rows
    out = []
    blk = 256
    want = list(want)
    for s in range(0, len(want), blk):
        ii = np.asarray(want[s:s + blk])
        d = pos[None, :, :] - pos[ii][:, None, :]
        d = d - box * np.rint(d / box)
        d2 = (d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1]) + d[..., 2] * d[..., 2]
        for r in range(len(ii)):
            out.append(np.nonzero(d2[r] <= R2)[0].astype(np.int32))
    if rows is not None:
        return out
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum([len(c) for c in out])
    col = np.concatenate(out) if out else np.zeros(0, np.int32)
    return row_ptr.astype(np.int32), col.astype(np.int32)


def pattern_matrix(row_ptr, col, n):
    """0/1 scipy CSR matrix of an atom pattern."""
    return sp.csr_matrix((np.ones(len(col), dtype=np.int64), np.asarray(col),
                          np.asarray(row_ptr)), shape=(n, n))


def pattern_product(A, B, mask=None):
    """Natural pattern pat(A.B) (boolean product), optionally intersected with
    `mask`; also returns the number of (i,k,j) triples feeding the kept blocks."""
    P = (A @ B).tocsr()
    if mask is not None:
        P = P.multiply(mask).tocsr()
    P.sort_indices()
    triples = int(P.sum())
    P.data[:] = 1
    return P, triples


# ---------------------------------------------------------------- orbitals
def offsets(nfun):
    off = np.zeros(len(nfun) + 1, dtype=np.int64)
    off[1:] = np.cumsum(nfun)
    return off


def block_mask(row_ptr, col, nfun):
    """Dense 0/1 orbital mask of an atom pattern."""
    off = offsets(nfun)
    n = len(nfun)
    M = np.zeros((off[-1], off[-1]))
    for i in range(n):
        for j in col[row_ptr[i]:row_ptr[i + 1]]:
            M[off[i]:off[i + 1], off[j]:off[j + 1]] = 1.0
    return M


def dense_to_blocks(A, row_ptr, col, nfun, pad=None):
    """Stored blocks of a dense matrix on a pattern: [nnzb, p, p] with p = pad
    (zero padded) or, for uniform nfun, the block size."""
    off = offsets(nfun)
    p = pad or int(np.max(nfun))
    n = len(nfun)
    out = np.zeros((len(col), p, p))
    for i in range(n):
        for t in range(row_ptr[i], row_ptr[i + 1]):
            j = col[t]
            out[t, :nfun[i], :nfun[j]] = A[off[i]:off[i + 1], off[j]:off[j + 1]]
    return out


def blocks_to_dense(V, row_ptr, col, nfun):
    off = offsets(nfun)
    n = len(nfun)
    A = np.zeros((off[-1], off[-1]))
    for i in range(n):
        for t in range(row_ptr[i], row_ptr[i + 1]):
            j = col[t]
            A[off[i]:off[i + 1], off[j]:off[j + 1]] = V[t, :nfun[i], :nfun[j]]
    return A


# ---------------------------------------------------------------- synthetic S, H
def image_weight(dx, box, R, decay):
    """sum over images of exp(-d_T/decay) for displacement(s) dx [..., 3]."""
    dx = np.asarray(dx, dtype=np.float64)
    R2 = float(R) * float(R)
    m = [int(math.ceil(R / b)) + 1 for b in box]
    w = np.zeros(dx.shape[:-1])
    for tx in range(-m[0], m[0] + 1):
        for ty in range(-m[1], m[1] + 1):
            for tz in range(-m[2], m[2] + 1):
                x = dx[..., 0] + float(tx) * box[0]
                y = dx[..., 1] + float(ty) * box[1]
                z = dx[..., 2] + float(tz) * box[2]
                d2 = (x * x + y * y) + z * z
                ok = d2 <= R2
                w = w + np.where(ok, np.exp(-(np.sqrt(d2) / decay)), 0.0)
    return w


def random_block(seed, stream, i, j, ni, nj, scale):
    """M_ij (ni x nj): counter-based uniforms, transposed for i > j and
    symmetrised on the diagonal."""
    a, b = (i, j) if i <= j else (j, i)
    na, nb = (ni, nj) if i <= j else (nj, ni)
    e = np.arange(na * nb)
    u = W.uniform01(seed, stream, a, b, e).reshape(na, nb)
    Mab = scale * (u - 0.5)
    if i == j:
        return (Mab + Mab.T) * 0.5
    return Mab if i <= j else Mab.T


def synth_blocks(w, kind, row_ptr, col, pad=None):
    """Stored blocks [nnzb, p, p] of the synthetic S (kind='S') or H ('H').

    Entry by entry this is random_block's definition (pinned against it in
    the tests); the uniforms of all blocks of one row with the same column
    block size are drawn in one vectorised call."""
    stream, decay, R = ((W.STREAM_S, 3.0, w.R_S) if kind == "S"
                        else (W.STREAM_H, 2.5, w.R_H))
    n = w.n
    nf = np.asarray(w.nfun)
    p = pad or int(nf.max())
    out = np.zeros((len(col), p, p))
    for i in range(n):
        r0 = row_ptr[i]
        js = np.asarray(col[r0:row_ptr[i + 1]], dtype=np.int64)
        dx = w.pos[js] - w.pos[i]
        wt = image_weight(dx, w.box, R, decay)
        ni = int(nf[i])
        for nj in np.unique(nf[js]):
            nj = int(nj)
            sel = np.nonzero(nf[js] == nj)[0]
            j = js[sel]
            r = np.arange(ni)[:, None]
            c = np.arange(nj)[None, :]
            M = np.empty((len(j), ni, nj))
            up, lo, dg = j > i, j < i, j == i
            if up.any():       # M_ij = scale (U(i, j, r*nj + c) - 1/2)
                M[up] = w.scale * (W.uniform01(w.seed, stream, i, j[up][:, None, None],
                                               (r * nj + c)[None]) - 0.5)
            if lo.any():       # M_ij = M_ji^T, M_ji = scale (U(j, i, c*ni + r) - 1/2)
                M[lo] = w.scale * (W.uniform01(w.seed, stream, j[lo][:, None, None], i,
                                               (c * ni + r)[None]) - 0.5)
            if dg.any():       # (R + R^T) / 2 on the diagonal block
                Mab = w.scale * (W.uniform01(w.seed, stream, i, i, r * ni + c) - 0.5)
                M[dg] = (Mab + Mab.T) * 0.5
            blk = wt[sel][:, None, None] * M
            if kind == "S":
                if dg.any():
                    blk[dg] += 2.0 * np.eye(ni)
            else:
                blk = -blk
            out[r0 + sel, :ni, :nj] = blk
    return out


class System:
    """Dense view of one workload: patterns, masks, S and H."""

    def __init__(self, w, R_L=None):
        self.w = w
        self.n = w.n
        self.nfun = w.nfun
        self.R_L = w.R_L if R_L is None else R_L
        self.pat = {}
        for name, R in (("S", w.R_S), ("H", w.R_H), ("L", self.R_L)):
            self.pat[name] = neighbours(w.pos, w.box, R)
        self.Sb = synth_blocks(w, "S", *self.pat["S"])
        self.Hb = synth_blocks(w, "H", *self.pat["H"])
        self.S = blocks_to_dense(self.Sb, *self.pat["S"], self.nfun)
        self.H = blocks_to_dense(self.Hb, *self.pat["H"], self.nfun)
        self.maskL = block_mask(*self.pat["L"], self.nfun)
        self.maskS = block_mask(*self.pat["S"], self.nfun)
        self.maskH = block_mask(*self.pat["H"], self.nfun)

    def blocks(self, A, name):
        return dense_to_blocks(A, *self.pat[name], self.nfun)
