"""Row-wise oracle for cells too large for dense matrices -- test infrastructure.

The same quantities as `lnv.evaluate` (Sec. II.C.2: K = 3LSL - 2LSLSL,
E = 2Tr[KH], N = 2Tr[KS], G = dE/dL, F = dN/dL) for the orbital rows of a few
sampled atoms i: each product chain is applied to the n_i x N_orb row panel
of its leftmost factor with scipy sparse matrices, so the cost is a handful of
panel-times-sparse products per sampled atom.

  G_i = 2 [3 (SLH + HLS) - 2 (SLSLH + SLHLS + HLSLS)]_i  on L's row i
  F_i = 12 [SLS - SLSLS]_i                                 on L's row i
  e_i = 2 sum_{a in i} (KH)_aa,   n_i = 2 sum_{a in i} (KS)_aa
so that sum_i e_i = E and sum_i n_i = N.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import structure as st


def bsr(blocks, row_ptr, col, nfun):
    """scipy CSR orbital matrix from stored blocks [nnzb, p, p] (block (i, j)
    is the leading nfun[i] x nfun[j] corner)."""
    nfun = np.asarray(nfun)
    n = len(nfun)
    b = int(nfun[0])
    if np.all(nfun == b):
        M = sp.bsr_matrix((np.ascontiguousarray(blocks[:, :b, :b]), np.asarray(col),
                           np.asarray(row_ptr)), shape=(n * b, n * b))
        return M.tocsr()
    off = st.offsets(nfun)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    col = np.asarray(col)
    parts_r, parts_c, parts_v = [], [], []
    for ni in np.unique(nfun):
        for nj in np.unique(nfun):
            sel = np.nonzero((nfun[rows] == ni) & (nfun[col] == nj))[0]
            if len(sel) == 0:
                continue
            rr = off[rows[sel]][:, None, None] + np.arange(ni)[None, :, None]
            cc = off[col[sel]][:, None, None] + np.arange(nj)[None, None, :]
            parts_r.append(np.broadcast_to(rr, (len(sel), ni, nj)).ravel())
            parts_c.append(np.broadcast_to(cc, (len(sel), ni, nj)).ravel())
            parts_v.append(blocks[sel, :ni, :nj].ravel())
    N = int(off[-1])
    M = sp.coo_matrix((np.concatenate(parts_v), (np.concatenate(parts_r),
                                                 np.concatenate(parts_c))), shape=(N, N))
    return M.tocsr()


class RowOracle:
    def __init__(self, w, Sb, Hb, Lb, patS, patH, patL):
        self.w = w
        self.nfun = w.nfun
        self.off = st.offsets(w.nfun)
        self.S = bsr(Sb, *patS, w.nfun)
        self.H = bsr(Hb, *patH, w.nfun)
        self.L = bsr(Lb, *patL, w.nfun)
        self.patL = patL

    def _panel(self, M, i):
        a, b = self.off[i], self.off[i + 1]
        return M[a:b].toarray()

    def row(self, i):
        """(e_i, n_i, G row blocks [m, n_i, p], F row blocks, columns of L's
        row); block t holds atom col[t]'s n_j columns, zero padded to
        p = max nfun."""
        S, H, L = self.S, self.H, self.L

        def chain(P, *mats):
            for M in mats:
                P = np.asarray(P @ M)
            return P

        Si, Hi, Li = self._panel(S, i), self._panel(H, i), self._panel(L, i)
        SL = chain(Si, L)
        HL = chain(Hi, L)
        SLH = chain(SL, H)
        HLS = chain(HL, S)
        SLS = chain(SL, S)
        SLSL = chain(SLS, L)
        SLSLH = chain(SLSL, H)
        SLHLS = chain(SLH, L, S)
        HLSLS = chain(HLS, L, S)
        SLSLS = chain(SLSL, S)
        LS = chain(Li, S)
        LSL = chain(LS, L)
        LSLSL = chain(LSL, S, L)
        Ki = 3.0 * LSL - 2.0 * LSLSL
        Gi = 2.0 * (3.0 * (SLH + HLS) - 2.0 * (SLSLH + SLHLS + HLSLS))
        Fi = 12.0 * (SLS - SLSLS)
        e = 2.0 * float(np.sum(Ki * Hi))
        nn = 2.0 * float(np.sum(Ki * Si))
        rp, col = self.patL
        cols = col[rp[i]:rp[i + 1]]
        b = self.off[i + 1] - self.off[i]
        p = int(np.max(self.nfun))
        Gb = np.zeros((len(cols), b, p))
        Fb = np.zeros((len(cols), b, p))
        for t, j in enumerate(cols):
            nj = self.off[j + 1] - self.off[j]
            Gb[t, :, :nj] = Gi[:, self.off[j]:self.off[j + 1]]
            Fb[t, :, :nj] = Fi[:, self.off[j]:self.off[j + 1]]
        return e, nn, Gb, Fb, cols


def reach(w):
    """Distance from a row's atom within which `RowOracle.row` reads matrix
    rows: the chain M1 M2 ... Mm applied to row i of M1 reads the rows of
    M(k+1) within R1 + ... + Rk of atom i (minimum-image distances obey the
    triangle inequality), and the longest chains are S.L.H.L.S and H.L.S.L.S
    (in G) and L.S.L.S.L (in K): R_H + R_S + 2 R_L."""
    return w.R_H + w.R_S + 2.0 * w.R_L


def region_patterns(w, atoms):
    """Range patterns (S, H, L) whose rows are those of the full patterns for
    every atom within reach(w) + 1 bohr of the given atoms and empty
    elsewhere: a RowOracle on them gives exactly the rows of those atoms, at
    a fraction of the set-up cost of the full patterns on large cells.
    Returns ((pS, pH, pL), number of rows kept)."""
    d = w.pos[None, :, :] - w.pos[np.asarray(atoms)][:, None, :]
    d = d - w.box * np.rint(d / w.box)
    near = np.nonzero(((d * d).sum(-1) <= (reach(w) + 1.0) ** 2).any(0))[0]
    out = []
    for R in (w.R_S, w.R_H, w.R_L):
        cols = st.neighbours(w.pos, w.box, R, rows=near)
        lens = np.zeros(w.n, dtype=np.int64)
        lens[near] = [len(c) for c in cols]
        rp = np.zeros(w.n + 1, dtype=np.int64)
        rp[1:] = np.cumsum(lens)
        out.append((rp.astype(np.int32), np.concatenate(cols).astype(np.int32)))
    return tuple(out), len(near)

