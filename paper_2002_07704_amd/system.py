"""Device-resident LNV system: patterns, matrices and workspaces.

Builds, on one GPU, everything the hot path needs for one geometry -- range
patterns of S, H and L (Sec. II.C.2), the synthetic S and H, the natural
patterns of the products S.L, H.L.S and S.L.S with their index tables and
work lists -- then exposes the evaluation and CG calls of liblnv.  Torch is
used for device memory and the stream only; every step runs in the library's
HIP kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses
from ctypes import byref, c_double, c_int32, c_int64

import numpy as np
import torch

from . import lib as L_

BLK = 4


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Cells:
    """The spatial cells of a system's units (rows, or with qs = 2 the atoms
    of four rows): lnv_cells on a g[0] x g[1] x g[2] grid of the box.  Every
    pattern of the system indexes its blocks through them (lnv_index)."""

    def __init__(self, pos_units, box, g, qs, dev, origin=None):
        pos_units = np.ascontiguousarray(pos_units, dtype=np.float64)
        self.n_units = int(pos_units.shape[0])
        self.qs = int(qs)
        self.g = tuple(int(x) for x in g)
        self.box = tuple(float(b) for b in box)
        self.origin = tuple(float(o) for o in (origin if origin is not None else
                                               [b / gg / 8.0 for b, gg in zip(self.box, self.g)]))
        pos_d = torch.as_tensor(pos_units, device=dev)
        self.cell = torch.empty(self.n_units, dtype=torch.int32, device=dev)
        self.slot = torch.empty(self.n_units, dtype=torch.int32, device=dev)
        occ = c_int32(0)
        L_.call("lnv_cells", _ptr(pos_d), self.n_units, (c_double * 3)(*self.box),
                (c_int32 * 3)(*self.g), (c_double * 3)(*self.origin), _ptr(self.cell),
                _ptr(self.slot), byref(occ), _stream())
        self.occ = int(occ.value)

    @staticmethod
    def single(n_units, dev):
        """One cell holding every unit (the index is then the dense n x n
        table): for patterns that come without positions."""
        return Cells(np.zeros((n_units, 3)), (1.0, 1.0, 1.0), (1, 1, 1), 0, dev,
                     origin=(0.0, 0.0, 0.0))

    @staticmethod
    def choose_grid(pos_units, box, ranges, max_g=1024):
        """Grid of the spatial index: the coarsest cells (edge box/g per
        axis) whose summed table sizes, over patterns with the given ranges,
        stay within a quarter of the smallest -- per row unit, (window cells)
        x (fullest cell's count), the window reaching floor(R/edge) + 1 cells
        each way, at most the whole axis.  One cell per axis is the dense
        table; coarser windows span more axes, where a lookup needs no
        window arithmetic (on the 4096-atom cell the dense table, 1.14x the
        smallest, makes the CG iteration 4% faster)."""
        pos = np.asarray(pos_units, dtype=np.float64)
        box = np.asarray(box, dtype=np.float64)
        costs = []
        kmax = int(min(max_g, max(1, np.floor(box.min() / 2.0))))
        for k in range(1, kmax + 1):
            g = np.maximum(1, np.round(box / (box.min() / k))).astype(np.int64)
            if np.any(g > max_g):
                break
            edge = box / g
            c = np.minimum((np.mod(pos / box, 1.0) * g).astype(np.int64), g - 1)
            key = (c[:, 0] * g[1] + c[:, 1]) * g[2] + c[:, 2]
            occ = int(np.bincount(key).max())
            cost = 0
            for R in ranges:
                w = np.minimum(2 * (np.floor(R / edge) + 1) + 1, g)
                cost += int(np.prod(w)) * occ
            costs.append((tuple(int(x) for x in g), cost))
        low = min(c for _, c in costs)
        return next(g for g, c in costs if c <= 1.25 * low)


class Pattern:
    """Atom-block CSR pattern on the device plus its optional tables."""

    def __init__(self, n, row_ptr, col, cells=None):
        self.n = int(n)
        self.row_ptr = row_ptr
        self.col = col
        self.cells = cells      # the system's Cells (for the spatial index)
        self.ix_tab = None      # lnv_index table (device)
        self.items = None
        self.triples = None
        self.cl = None          # (m, g, cl_ptr, cl_col, cl_pos, cl_items, cl_cell)
        self.tile4 = 0          # lnv_pattern_tile4 grade (1 tile4, 0)
        self.struct = L_.LnvPattern()
        self._sync()

    @property
    def nnzb(self):
        return int(self.col.numel())

    @property
    def has_index(self):
        return self.ix_tab is not None

    def _sync(self):
        s = self.struct
        s.n = self.n
        s.nnzb = self.nnzb
        s.row_ptr = self.row_ptr.data_ptr()
        s.col = self.col.data_ptr() if self.col.numel() else self.row_ptr.data_ptr()
        s.ix.tab = self.ix_tab.data_ptr() if self.ix_tab is not None else None
        s.items = self.items.data_ptr() if self.items is not None else None
        s.n_items = 0 if self.items is None else self.items.numel() // 2
        if self.cl is not None:
            m, g, cptr, ccol, cpos, citems, ccell = self.cl
            s.cl_m, s.cl_g, s.n_cl_items = m, g, citems.numel() // 2
            s.cl_ptr, s.cl_col = cptr.data_ptr(), ccol.data_ptr()
            s.cl_pos, s.cl_items = cpos.data_ptr(), citems.data_ptr()
            s.cl_cell = ccell.data_ptr()
        else:
            s.cl_m = s.cl_g = s.n_cl_items = 0
        s.tile4 = self.tile4

    def check_tile4(self):
        """lnv_pattern_tile4: may the atom-tile multiply read and write this
        pattern by tiles (1: 4 rows per atom, columns in aligned runs of 4)?"""
        ok = c_int32(0)
        L_.call("lnv_pattern_tile4", byref(self.struct), byref(ok), _stream())
        self.tile4 = int(ok.value)
        self._sync()
        return self.tile4

    def build_index(self):
        """The spatial index of the pattern over its system's cells
        (lnv_pattern_index, two-phase); idempotent."""
        if self.ix_tab is not None:
            return self
        if self.cells is None:
            self.cells = Cells.single(self.n, self.row_ptr.device)
        c = self.cells
        ln = c_int64(0)
        g = (c_int32 * 3)(*c.g)
        L_.call("lnv_pattern_index", byref(self.struct), _ptr(c.cell), _ptr(c.slot), g, c.occ,
                c.qs, None, 0, byref(ln), _stream())
        tab = torch.empty(ln.value, dtype=torch.int32, device=self.row_ptr.device)
        L_.call("lnv_pattern_index", byref(self.struct), _ptr(c.cell), _ptr(c.slot), g, c.occ,
                c.qs, _ptr(tab), tab.numel(), byref(ln), _stream())
        self.ix_tab = tab
        self._sync()
        return self

    def index_bytes(self):
        return 0 if self.ix_tab is None else self.ix_tab.numel() * 4

    def build_items(self):
        cnt = c_int32(0)
        L_.call("lnv_pattern_items", byref(self.struct), None, 0, byref(cnt), _stream())
        self.items = torch.empty(max(1, 2 * cnt.value), dtype=torch.int32,
                                 device=self.row_ptr.device)
        L_.call("lnv_pattern_items", byref(self.struct), _ptr(self.items),
                self.items.numel() // 2, byref(cnt), _stream())
        self.items = self.items[:2 * cnt.value]
        self._sync()
        self.struct.n_items = cnt.value
        return self

    def build_cluster(self, m, g):
        """Cluster plan for clusters of m consecutive rows, g lanes per column
        (builds the pattern's index first)."""
        self.build_index()
        dev = self.row_ptr.device
        nc = (self.n + m - 1) // m
        cptr = torch.empty(nc + 1, dtype=torch.int32, device=dev)
        ln = c_int64(0)
        ni = c_int32(0)
        L_.call("lnv_pattern_cluster", byref(self.struct), m, g, _ptr(cptr), None, None, None, 0,
                None, 0, byref(ln), byref(ni), _stream())
        ccol = torch.empty(max(1, ln.value), dtype=torch.int32, device=dev)
        cpos = torch.empty(max(1, ln.value * m), dtype=torch.int32, device=dev)
        ccell = torch.empty(max(2, 2 * ln.value), dtype=torch.int32, device=dev)
        citems = torch.empty(max(2, 2 * ni.value), dtype=torch.int32, device=dev)
        L_.call("lnv_pattern_cluster", byref(self.struct), m, g, _ptr(cptr), _ptr(ccol), _ptr(cpos),
                _ptr(ccell), ccol.numel(), _ptr(citems), citems.numel() // 2, byref(ln),
                byref(ni), _stream())
        self.cl = (m, g, cptr, ccol, cpos, citems[:2 * ni.value], ccell)
        self._sync()
        if m == 16:
            self.check_tile4()
        return self

    def host(self):
        return self.row_ptr.cpu().numpy(), self.col.cpu().numpy()


def split_rows(nfun, blk=BLK):
    """Stored-row layout of atoms with nfun support functions in blk x blk
    blocks: atom a spans ceil(nfun[a]/blk) consecutive rows; row i holds the
    atom's functions off_of[i] .. off_of[i]+blk-1 (those past nfun[a] are
    padding).  Returns (atom_of, off_of), int32 [n_rows]."""
    nfun = np.asarray(nfun, dtype=np.int64)
    nsub = (nfun + blk - 1) // blk
    atom_of = np.repeat(np.arange(len(nfun)), nsub)
    first = np.repeat(np.cumsum(nsub) - nsub, nsub)
    off_of = (np.arange(int(nsub.sum())) - first) * blk
    return atom_of.astype(np.int32), off_of.astype(np.int32)


def cell_order(pos, box, edge=10.26):
    """Atoms ordered cell by cell (cubic cells of about `edge` bohr, x slowest,
    z fastest), stable within a cell: neighbouring rows are then spatial
    neighbours, which the 4-row clusters and the per-XCD row ranges of the
    multiply rely on.  Diamond cells generated cube by cube are already
    nearly in this order (up to atoms displaced across a cube face)."""
    pos = np.asarray(pos)
    box = np.asarray(box, dtype=np.float64)
    m = np.maximum(1, np.round(box / edge)).astype(np.int64)
    c = np.minimum((pos / (box / m)).astype(np.int64), m - 1)
    key = (c[:, 0] * m[1] + c[:, 1]) * m[2] + c[:, 2]
    return np.argsort(key, kind="stable")


def row_order(w, reorder, split):
    """Order of the atoms along the rows (None: the workload's own order,
    rows = atoms).  reorder: None -- spatial cells for split systems, the
    atoms' own order otherwise (diamond cells are generated cube by cube);
    False -- the atoms' own order; "cell" -- cell_order; "bonds" -- the
    workload's groups of four bonded atoms (w.groups), so that each 4-row
    cluster of the multiply holds one compact group and the union of its
    rows' columns stays small (on the 4096-atom diamond cell the clusters'
    unions of L's columns drop from 204 to 186 atoms, below three 64-lane
    waves); or an explicit permutation of the atoms.  Values follow the
    atoms: S and H are generated per atom pair, so any order gives the same
    matrices up to the permutation."""
    n = int(w.pos.shape[0])
    if reorder is None:
        reorder = "cell" if split else False
    if reorder is False:
        return np.arange(n) if split else None
    if isinstance(reorder, str):
        if reorder == "cell":
            return cell_order(w.pos, w.box)
        if reorder == "bonds":
            if getattr(w, "groups", None) is None:
                raise ValueError(f"workload {w.name} carries no bonded groups")
            order = np.asarray(w.groups, dtype=np.int64)
        else:
            raise ValueError(f"unknown row order {reorder!r}")
    else:
        order = np.asarray(reorder, dtype=np.int64)
    if order.shape != (n,) or not np.array_equal(np.sort(order), np.arange(n)):
        raise ValueError("a row order must be a permutation of the atoms")
    return order


def neighbours(pos_dev, box, R):
    """a0: range pattern for cutoff R (lnv_neighbours, two-phase)."""
    n = pos_dev.shape[0]
    box_c = (c_double * 3)(*[float(b) for b in box])
    rp = torch.empty(n + 1, dtype=torch.int32, device=pos_dev.device)
    nnz = c_int64(0)
    L_.call("lnv_neighbours", _ptr(pos_dev), n, box_c, float(R), _ptr(rp), None, 0,
            byref(nnz), _stream())
    col = torch.empty(nnz.value, dtype=torch.int32, device=pos_dev.device)
    L_.call("lnv_neighbours", _ptr(pos_dev), n, box_c, float(R), _ptr(rp), _ptr(col),
            nnz.value, byref(nnz), _stream())
    return Pattern(n, rp, col)


def xz_range(R_S, R_L):
    """Cutoff of the stored X = H.L.S and Z = S.L.S: the farthest pair that a
    product onto L's range with S.L on the left reads, R_S + 2 R_L, with a
    margin of 1e-9 relative for the rounding of the distances."""
    return (float(R_S) + 2.0 * float(R_L)) * (1.0 + 1e-9)


def product_pattern(A, B, mask=None, triples=True):
    """a2: pattern of A.B (natural range) or of P_mask(A.B), with triple count."""
    n = A.n
    dev = A.row_ptr.device
    rp = torch.empty(n + 1, dtype=torch.int32, device=dev)
    rt = torch.empty(n + 1, dtype=torch.int64, device=dev) if triples else None
    nnz = c_int64(0)
    tr = c_int64(0)
    mp = byref(mask.struct) if mask is not None else None
    L_.call("lnv_pattern_product", byref(A.struct), byref(B.struct), mp, _ptr(rp), None, 0,
            byref(nnz), _ptr(rt), byref(tr) if triples else None, _stream())
    col = torch.empty(max(1, nnz.value), dtype=torch.int32, device=dev)
    L_.call("lnv_pattern_product", byref(A.struct), byref(B.struct), mp, _ptr(rp), _ptr(col),
            col.numel(), byref(nnz), None, None, _stream())
    P = Pattern(n, rp, col[:nnz.value], A.cells)
    P.triples = tr.value if triples else None
    return P


def half_pattern(P):
    """The half of the symmetric pattern P that holds each pair of blocks
    once, balanced over the rows (lnv_pattern_half), with its work list and
    index table (the mirror finds its blocks through it)."""
    dev = P.row_ptr.device
    rp = torch.empty(P.n + 1, dtype=torch.int32, device=dev)
    nnz = c_int64(0)
    L_.call("lnv_pattern_half", byref(P.struct), _ptr(rp), None, 0, byref(nnz), _stream())
    col = torch.empty(max(1, nnz.value), dtype=torch.int32, device=dev)
    L_.call("lnv_pattern_half", byref(P.struct), _ptr(rp), _ptr(col), col.numel(), byref(nnz),
            _stream())
    return Pattern(P.n, rp, col[:nnz.value], P.cells).build_items().build_index()


def is_symmetric(P):
    """Whether every block (i, j) of P has its transpose (j, i) in P (on the
    device, through the transpose map of P onto itself; builds P's index)."""
    P.build_index()
    try:
        transpose_map(P, P)
    except L_.LnvError as e:
        if e.status == L_.EPATTERN:
            return False
        raise
    return True


class Matrix:
    """Block values on a pattern: tensor [nnzb, 4, 4] (float64, or float32 for
    the mixed-precision products) plus lnv_bsm."""

    def __init__(self, pattern, values=None, dtype=torch.float64):
        self.pat = pattern
        if values is None:
            values = torch.zeros(max(1, pattern.nnzb), BLK, BLK, dtype=dtype,
                                 device=pattern.row_ptr.device)
        if values.dtype not in (torch.float64, torch.float32):
            raise ValueError("block values must be float64 or float32")
        self.val = values
        self.struct = L_.LnvBsm()
        self.struct.pat = ctypes.pointer(pattern.struct)
        self.struct.blk = BLK
        self.struct.dtype = L_.F32 if values.dtype == torch.float32 else L_.F64
        self.struct.val = values.data_ptr()

    def rebind(self, values):
        self.val = values
        self.struct.val = values.data_ptr()
        self.struct.dtype = L_.F32 if values.dtype == torch.float32 else L_.F64
        return self


def transpose_map(P, PT):
    """perm[p] = position in PT of the transpose of block p of P."""
    perm = torch.empty(max(1, P.nnzb), dtype=torch.int32, device=P.row_ptr.device)
    L_.call("lnv_pattern_transpose_map", byref(P.struct), byref(PT.struct), _ptr(perm), _stream())
    return perm


def transpose(A, perm, AT):
    L_.call("lnv_bsm_transpose", byref(A.struct), _ptr(perm), byref(AT.struct), _stream())
    return AT


def bsm(pattern, tensor):
    """lnv_bsm view of a raw value tensor on a pattern."""
    return Matrix(pattern, tensor)


def multiply(alpha, A, B, transB, beta, C):
    L_.call("lnv_bsm_multiply", float(alpha), byref(A.struct), byref(B.struct), int(transB),
            float(beta), byref(C.struct), _stream())
    return C


def multiply_dot(alpha, A, B, transB, beta, C, store, M1, M2=None):
    dev = C.val.device
    st = C.pat.struct       # one partial pair per work piece (row or cluster pieces)
    part = torch.empty(max(2, 2 * max(st.n_items, st.n_cl_items)), dtype=torch.float64,
                       device=dev)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    L_.call("lnv_bsm_multiply_dot", float(alpha), byref(A.struct), byref(B.struct), int(transB),
            float(beta), byref(C.struct), int(store), byref(M1.struct),
            byref(M2.struct) if M2 is not None else None, _ptr(part), _ptr(out), _stream())
    return out


def dot(A, B):
    dev = A.val.device
    part = torch.empty(L_.DOT_PARTIALS, dtype=torch.float64, device=dev)
    out = torch.zeros(1, dtype=torch.float64, device=dev)
    L_.call("lnv_bsm_dot", byref(A.struct), byref(B.struct), _ptr(part), _ptr(out), _stream())
    return out


@dataclasses.dataclass
class Opts:
    reset_period: int = 40
    n_tol: float = 1e-11
    step_cap: float = 0.1
    mixed: bool = False      # the step's evaluation with FP32 block products
    occ_every: int = 10      # occupation bounds of L S every occ_every-th iteration (0: never)
    occ_iter: int = 16       # Lanczos steps of each bound


class LNVSystem:
    """One geometry on one GPU: patterns, S, H, L and the CG workspace.

    metric: "hotelling" builds T ~ S^-1 on L's range (n_hotelling steps) and
    runs the CG in that metric; None uses the identity.  symmetric: form only
    the blocks of one half (half_pattern) of the symmetric products SLS,
    P_L(SLHLS), P_L(SLSLS) and P_L(TGT) and copy the rest transposed (needs
    symmetric patterns, which L, S, H have).  reorder: the order of the atoms
    along the rows (row_order); every result is the same up to that
    permutation, and atom_of maps rows back to atoms.  lean: evaluation only
    (no stored L.S, X^T, no CG buffers).  grid: cells of the spatial index
    per axis (default: Cells.choose_grid; (1, 1, 1) is the dense table).
    """

    def __init__(self, w, device="cuda", R_L=None, metric="hotelling", n_hotelling=16,
                 cluster=(4, 1), reorder=None, symmetric=True, lean=False, grid=None):
        if not torch.cuda.is_available():
            raise RuntimeError("LNVSystem needs a GPU (HIP device)")
        L_.load()
        dev = torch.device(device)
        self.dev = dev
        self.cells = list(w) if isinstance(w, (list, tuple)) else None
        if self.cells is not None:
            self._layout_cells(self.cells, R_L)
        else:
            self._layout_single(w, R_L, reorder, grid)
        # a2: product patterns (A = LS is stored as its transpose SL).  X =
        # H.L.S and Z = S.L.S are read only by products onto L's range with
        # S.L on the left, and by L's own blocks: entry (k, j) is read when
        # some i has (i, k) in S.L and (i, j) in L, so the distance of k and
        # j is at most R_S + 2 R_L (triangle inequality over the nearest
        # images).  Both are formed on that ball within their natural range
        # (a margin of 1e-9 relative covers the rounding of the distances).
        self.pSL = product_pattern(self.pS, self.pL)            # S.L
        self.pLS = product_pattern(self.pL, self.pS, triples=False)   # L.S (row form of A)
        self.R_XZ = xz_range(self.R_S, self.R_L)
        pM = self._range_pattern(self.R_XZ)
        self.pX = product_pattern(self.pH, self.pLS, mask=pM)   # H.L.S
        self.pZ = product_pattern(self.pS, self.pLS, mask=pM)   # S.L.S
        self.pXT = product_pattern(self.pSL, self.pH, mask=pM, triples=False)   # pat(X)^T
        del pM
        # lean: evaluation only, without the stored transposes L.S and X^T (the
        # atom-tile products read S.L and X transposed) and without the CG's
        # buffers -- for cells whose natural-range intermediates fill the GPU
        self.lean = bool(lean)
        self.triples = dict(
            SL=self.pSL.triples, X=self.pX.triples, Z=self.pZ.triples,
            YT=product_pattern(self.pSL, self.pXT, mask=self.pL).triples,
            W=product_pattern(self.pSL, self.pX, mask=self.pL).triples,
            V=product_pattern(self.pSL, self.pZ, mask=self.pL).triples,
        )
        self.metric = metric
        if metric is not None:
            self.pLL = product_pattern(self.pL, self.pL)          # T.G, T.F
            self.triples["TG"] = self.pLL.triples
            # P_L(T (G T)): T on the left of the restricted product
            self.triples["TGT"] = product_pattern(self.pL, self.pLL, mask=self.pL).triples
        # symmetric products Z, W, V (and P_L(TGT)): balanced halves
        self.symmetric = bool(symmetric) and is_symmetric(self.pL) and is_symmetric(self.pZ)
        self.pZu = self.pLu = None
        if self.symmetric:
            self.pZu, self.pLu = half_pattern(self.pZ), half_pattern(self.pL)
            # block triples of the halves (what the kernels multiply)
            self.triples_upper = dict(
                Z=product_pattern(self.pS, self.pLS, mask=self.pZu).triples,
                W=product_pattern(self.pSL, self.pX, mask=self.pLu).triples,
                V=product_pattern(self.pSL, self.pZ, mask=self.pLu).triples)
            if metric is not None:
                self.triples_upper["TGT"] = product_pattern(self.pL, self.pLL,
                                                            mask=self.pLu).triples
        # index tables and work lists
        self.pL.build_index().build_items()
        self.pS.build_index()
        self.pH.build_items()
        self.pSL.build_index().build_items()
        self.pX.build_index().build_items()
        self.pZ.build_index().build_items()
        if not self.lean:
            self.pLS.build_index()
            self.pXT.build_index()
        if metric is not None and not self.lean:
            self.pLL.build_index().build_items()
        assert self.pX.nnzb >= self.pZ.nnzb
        self.cluster = None
        if cluster is not None:
            self.set_cluster(cluster)
        if self.lean:
            # X^T's pattern only counted the triples of P_L(S.L X^T)
            if self.split:
                self._alg_flops(("YT",))
            self.pXT = None
            self.perm_SL = self.perm_X = None
        else:
            self.perm_SL = transpose_map(self.pSL, self.pLS)
            self.perm_X = transpose_map(self.pX, self.pXT)
        # buffers
        nL = self.pL.nnzb

        def lbuf():
            return torch.zeros(nL, BLK, BLK, dtype=torch.float64, device=dev)

        self.L = Matrix(self.pL)
        self.G = Matrix(self.pL)
        self.F = Matrix(self.pL)
        self.SL = Matrix(self.pSL)
        self.X = Matrix(self.pX)
        self.Z = Matrix(self.pZ)
        self.LS = self.XT = None
        if not self.lean:
            self.LS = Matrix(self.pLS)
            self.XT = Matrix(self.pXT)
        self.YT, self.W, self.V = lbuf(), lbuf(), lbuf()
        if self.symmetric:
            self.Zu, self.Lu = Matrix(self.pZu), Matrix(self.pLu)
            self.Vu = torch.zeros_like(self.Lu.val)
        self.Gc = Matrix(self.pL) if metric is not None else None
        self.T = Matrix(self.pL) if metric is not None else None
        if not self.lean:
            self.SL2 = torch.zeros_like(self.SL.val)
            self.Hp = torch.zeros_like(self.H.val)
            self.g, self.gc_prev, self.D, self.D_prev = lbuf(), lbuf(), lbuf(), lbuf()
            self.gc = lbuf() if metric is not None else None
            self.Fc = Matrix(self.pL) if metric is not None else None
        if metric is not None and not self.lean:
            # T G lives in XT's memory when it fits (XT is dead at that point)
            if self.pLL.nnzb <= self.pXT.nnzb:
                llv = self.XT.val.view(-1)[:self.pLL.nnzb * BLK * BLK].view(-1, BLK, BLK)
            else:
                llv = torch.zeros(self.pLL.nnzb, BLK, BLK, dtype=torch.float64, device=dev)
            self.LL = Matrix(self.pLL, llv)
        plen = L_.load().lnv_partials_len(max(self.pL.struct.n_items, self.pL.struct.n_cl_items))
        self.partials = torch.zeros(plen, dtype=torch.float64, device=dev)
        self.scalars = torch.zeros(L_.NSCALARS, dtype=torch.float64, device=dev)
        self.EN = torch.zeros(2, dtype=torch.float64, device=dev)
        self.ws = L_.LnvCgWs()
        ev = self.ws.ev
        ev.SL = self.SL.struct
        ev.X = self.X.struct
        ev.Z = self.Z.struct
        if not self.lean:
            ev.LS = self.LS.struct
            ev.XT = self.XT.struct
            ev.perm_SL = self.perm_SL.data_ptr()
            ev.perm_X = self.perm_X.data_ptr()
        ev.YT, ev.W, ev.V = self.YT.data_ptr(), self.W.data_ptr(), self.V.data_ptr()
        ev.partials = self.partials.data_ptr()
        ev.partials_len = plen
        ev.scalars = self.scalars.data_ptr()
        if self.symmetric:
            ev.Zu, ev.Lu, ev.Vu = self.Zu.struct, self.Lu.struct, self.Vu.data_ptr()
        self.ws.G = self.G.val.data_ptr()
        self.ws.F = self.F.val.data_ptr()
        self._bufs = {}
        if not self.lean:
            self.ws.SL2 = self.SL2.data_ptr()
            self.ws.Hp = self.Hp.data_ptr()
            self._bufs = {t.data_ptr(): t for t in (self.g, self.gc_prev, self.D, self.D_prev)}
            self.ws.g, self.ws.gc_prev = self.g.data_ptr(), self.gc_prev.data_ptr()
            self.ws.D, self.ws.D_prev = self.D.data_ptr(), self.D_prev.data_ptr()
            self.lanczos = torch.zeros(int(L_.load().lnv_lanczos_len(self.pL.n)),
                                       dtype=torch.float64, device=dev)
            self.ws.lanczos = self.lanczos.data_ptr()
        if metric is not None:
            self.ws.Gc = self.Gc.val.data_ptr()
            if not self.lean:
                self.ws.LL = self.LL.struct
                self.ws.Fc = self.Fc.val.data_ptr()
                self.ws.gc = self.gc.data_ptr()
                self._bufs[self.gc.data_ptr()] = self.gc
            if self.cells is not None:
                # each cell's own sigma, the products for all cells at once
                L_.call("lnv_hotelling_batch", byref(self.S.struct), byref(self.T.struct),
                        int(n_hotelling), byref(self.batch()), byref(self.ws), _stream())
            else:
                L_.call("lnv_hotelling", byref(self.S.struct), byref(self.T.struct),
                        int(n_hotelling), byref(self.ws), _stream())
        self.opts = Opts()
        self.k = 0
        self.adj_ws = None
        self.ws32 = None
        torch.cuda.synchronize()

    def synth_values(self, kind, pat, R, decay, seed=None, scale=None, seed_offset=0):
        """Synthetic blocks (kind 0: overlap-like w M + 2I, 1: -w M) on one of
        this system's patterns, in its row layout (lnv_synth_blocks, or
        lnv_synth_blocks_cells); seed None: the master seed (each cell's own
        in a batch), plus seed_offset."""
        M = Matrix(pat)
        scale = float(self.scale if scale is None else scale)
        if self.cells is not None:
            seeds = (self.seeds if seed is None else torch.full_like(self.seeds, int(seed)))
            seeds = seeds + int(seed_offset)
            L_.call("lnv_synth_blocks_cells", _ptr(self.pos), _ptr(self.cell_of), _ptr(self.boxes),
                    _ptr(seeds), _ptr(self.atom_of), _ptr(self.fun_of), _ptr(self.off_of),
                    byref(M.struct), int(kind), float(R), float(decay), scale, _stream())
            return M
        box_c = (c_double * 3)(*self.box)
        seed = (self.seed if seed is None else int(seed)) + int(seed_offset)
        L_.call("lnv_synth_blocks", _ptr(self.pos), box_c, _ptr(self.nfun), _ptr(self.atom_of),
                _ptr(self.off_of), byref(M.struct), int(kind), float(R), float(decay), seed,
                scale, _stream())
        return M

    # ----------------------------------------------------------- mixed precision
    def mixed_setup(self):
        """FP32 copies of L, S, H and FP32 intermediates for lnv_eval_mixed
        (same patterns, tables and transpose maps as the FP64 evaluation).
        A lean system keeps its FP32 intermediates in the memory of the FP64
        ones (each evaluation forms all of its intermediates before reading
        them, so FP64 and FP32 evaluations may alternate; a lean system runs
        no CG, which would need both at once)."""
        if self.ws32 is not None:
            return

        def f32(pat, share=None):
            if share is not None and self.lean:
                v = share.view(-1).view(torch.float32)[:max(1, pat.nnzb) * BLK * BLK]
                return Matrix(pat, v.view(-1, BLK, BLK))
            return Matrix(pat, dtype=torch.float32)

        self.L32, self.S32, self.H32 = f32(self.pL), f32(self.pS), f32(self.pH)
        self.SL32 = f32(self.pSL, self.SL.val)
        self.X32, self.Z32 = f32(self.pX, self.X.val), f32(self.pZ, self.Z.val)
        self.LS32 = self.XT32 = None
        if not self.lean:
            self.LS32, self.XT32 = f32(self.pLS), f32(self.pXT)
        nL = self.pL.nnzb
        if self.lean:
            self.YT32, self.W32, self.V32 = (f32(self.pL, t).val for t in (self.YT, self.W, self.V))
        else:
            self.YT32, self.W32, self.V32 = (torch.zeros(nL, BLK, BLK, dtype=torch.float32,
                                                         device=self.dev) for _ in range(3))
        ws = L_.LnvEval32Ws()
        ws.L, ws.S, ws.H = self.L32.struct, self.S32.struct, self.H32.struct
        ws.SL = self.SL32.struct
        ws.X, ws.Z = self.X32.struct, self.Z32.struct
        if not self.lean:
            ws.LS, ws.XT = self.LS32.struct, self.XT32.struct
            ws.perm_SL, ws.perm_X = self.perm_SL.data_ptr(), self.perm_X.data_ptr()
        ws.YT, ws.W, ws.V = self.YT32.data_ptr(), self.W32.data_ptr(), self.V32.data_ptr()
        ws.partials = self.partials.data_ptr()
        ws.partials_len = self.ws.ev.partials_len
        ws.scalars = self.scalars.data_ptr()
        if self.symmetric:
            self.Zu32, self.Lu32 = f32(self.pZu, self.Zu.val), f32(self.pLu, self.Lu.val)
            self.Vu32 = (f32(self.pLu, self.Vu).val if self.lean
                         else torch.zeros_like(self.Lu32.val))
            ws.Zu, ws.Lu, ws.Vu = self.Zu32.struct, self.Lu32.struct, self.Vu32.data_ptr()
        self.ws32 = ws
        torch.cuda.synchronize()

    def eval_mixed(self):
        """lnv_eval_mixed at the current L: FP32 products, FP64 assembly and
        traces; writes G, F, EN like eval()."""
        self.mixed_setup()
        L_.call("lnv_eval_mixed", byref(self.L.struct), byref(self.S.struct),
                byref(self.H.struct), byref(self.G.struct), byref(self.F.struct), _ptr(self.EN),
                byref(self.ws32), _stream())
        return self.EN

    # ----------------------------------------------------------- work decomposition
    def _cluster_patterns(self):
        """Patterns that are a left operand or an output of some multiply."""
        pats = [self.pS, self.pH, self.pL, self.pSL, self.pX, self.pZ]
        if getattr(self, "symmetric", False):
            pats += [self.pZu, self.pLu]
        if self.metric is not None and not getattr(self, "lean", False):
            pats.append(self.pLL)
        if getattr(self, "adj_ws", None) is not None:
            pats += [self.pLSL, self.pHL, self.pLS, self.pLH]
            if self.symmetric:
                pats += [self.pLSLu, self.pHu, self.pSu]
        return pats

    def tile_shapes(self):
        """Atom-tile shapes ((16, 4): 4 x 4 atom tiles per wave, (16, 8):
        4 x 2) when every atom is stored as 4 rows (13 support functions),
        else ()."""
        if self.cells is None and self.n_rows == 4 * self.n and self.pL.check_tile4() == 1:
            return ((16, 4), (16, 8))
        return ()

    def _all_patterns(self):
        return [v for v in vars(self).values() if isinstance(v, Pattern)]

    def set_cluster(self, shape):
        """Row-cluster shape of the multiply: (4, 1) (4 rows per wave, one lane
        per output column), None (one row per wave), or the atom tiles
        (16, 4) / (16, 8) (16-row
        plans: 4 atoms of 4 rows, products of whole 16x16 atom tiles on the
        matrix cores; right operands need tile4).  Rebuilds the plans in
        place."""
        if shape is not None and shape[0] == 16:
            for P in self._all_patterns():
                P.check_tile4()
        for P in self._cluster_patterns():
            if shape is None:
                P.cl = None
                P._sync()
                continue
            P.build_cluster(*shape)
        self.cluster = shape
        self._size_partials()
        torch.cuda.synchronize()

    def _size_partials(self):
        """Trace partials: one pair per work piece of L's pattern (row items or
        cluster pieces, whichever are more); grown when a plan needs more."""
        st = self.pL.struct
        need = L_.load().lnv_partials_len(max(st.n_items, st.n_cl_items))
        if getattr(self, "partials", None) is not None and self.partials.numel() >= need:
            return
        self.partials = torch.zeros(need, dtype=torch.float64, device=self.dev)
        if getattr(self, "ws", None) is not None:
            self.ws.ev.partials = self.partials.data_ptr()
            self.ws.ev.partials_len = need
        if getattr(self, "ws32", None) is not None:
            self.ws32.partials = self.partials.data_ptr()
            self.ws32.partials_len = need

    # ----------------------------------------------------------- row layout
    def _layout_single(self, w, R_L, reorder, grid=None):
        """a0/a1 of one periodic cell: range patterns and synthetic S, H."""
        dev = self.dev
        self.w = w
        self.n = w.n
        self.n_elec = float(w.n_elec)
        self.R_S, self.R_H = float(w.R_S), float(w.R_H)
        self.R_L = float(w.R_L if R_L is None else R_L)
        self.seed, self.scale = int(w.seed), float(w.scale)
        self.box = [float(b) for b in w.box]
        nfun = np.asarray(w.nfun, dtype=np.int32)
        # atoms with other than 4 support functions span several 4x4-blocked
        # rows; rows follow the atoms in the order row_order picks
        self.split = bool(np.any(nfun != BLK))
        order = row_order(w, reorder, self.split)
        if order is not None:
            sub, off_of = split_rows(nfun[order])
            atom_of = order[sub].astype(np.int32)
            self.atom_of = torch.as_tensor(atom_of, device=dev)
            self.off_of = torch.as_tensor(off_of, device=dev)
            self.nfun = torch.as_tensor(nfun, device=dev)
            self.fun_rows = torch.as_tensor(np.minimum(BLK, nfun[atom_of] - off_of)
                                            .astype(np.int32), device=dev)
            pos_rows = np.ascontiguousarray(w.pos[atom_of])
        else:
            self.atom_of = self.off_of = self.nfun = self.fun_rows = None
            pos_rows = np.ascontiguousarray(w.pos)
        self.n_rows = int(pos_rows.shape[0])
        self.pos = torch.as_tensor(pos_rows, dtype=torch.float64, device=dev)
        # a0: range patterns
        self.pS = neighbours(self.pos, self.box, self.R_S)
        self.pH = neighbours(self.pos, self.box, self.R_H)
        self.pL = neighbours(self.pos, self.box, self.R_L)
        # cells of the spatial index: atoms of 4 rows each (13 support
        # functions) are the index's units, else the rows
        qs = 2 if self.split and self.n_rows == 4 * self.n else 0
        units = pos_rows[::4] if qs else pos_rows
        g = Cells.choose_grid(units, self.box, self._index_ranges()) if grid is None else grid
        self.ix_cells = Cells(units, self.box, g, qs, dev)
        for P in (self.pS, self.pH, self.pL):
            P.cells = self.ix_cells
        # a1: synthetic S, H
        self.S = self.synth_values(0, self.pS, self.R_S, 3.0, self.seed)
        self.H = self.synth_values(1, self.pH, self.R_H, 2.5, self.seed)

    def _layout_cells(self, cells, R_L):
        """a0/a1 of a batch of independent cells: one block-diagonal system
        whose rows are the cells' rows one cell after another (each cell's
        atoms in spatial-cell order, split into 4x4-blocked rows)."""
        dev = self.dev
        w0 = cells[0]
        for c in cells:
            if (c.R_S, c.R_H, c.R_L, c.scale) != (w0.R_S, w0.R_H, w0.R_L, w0.scale):
                raise ValueError("cells of a batch share ranges and entry scale")
        self.w = None
        self.n = int(sum(c.n for c in cells))
        self.n_elec = float(sum(c.n_elec for c in cells))
        self.R_S, self.R_H = float(w0.R_S), float(w0.R_H)
        self.R_L = float(w0.R_L if R_L is None else R_L)
        self.seed, self.scale = None, float(w0.scale)
        self.box = None
        self.split = True
        atom, off, fun, cell, pos = [], [], [], [], []
        start = [0]
        for ci, c in enumerate(cells):
            nfun = np.asarray(c.nfun, dtype=np.int32)
            order = cell_order(c.pos, c.box)
            sub, off_c = split_rows(nfun[order])
            a = order[sub]
            atom.append(a)
            off.append(off_c)
            fun.append(nfun[a])
            cell.append(np.full(len(a), ci))
            pos.append(c.pos[a])
            start.append(start[-1] + len(a))
        i32 = lambda x: torch.as_tensor(np.concatenate(x).astype(np.int32), device=dev)  # noqa
        self.atom_of, self.off_of, self.fun_of, self.cell_of = i32(atom), i32(off), i32(fun), i32(cell)
        self.nfun = None
        self.fun_rows = torch.minimum(torch.full_like(self.off_of, BLK), self.fun_of - self.off_of)
        self.cell_start = torch.as_tensor(np.array(start, dtype=np.int32), device=dev)
        self.cell_rows = np.array(start)
        self.boxes = torch.as_tensor(np.array([c.box for c in cells], dtype=np.float64), device=dev)
        self.seeds = torch.as_tensor(np.array([c.seed for c in cells], dtype=np.uint64)
                                     .view(np.int64), device=dev)
        self.pos = torch.as_tensor(np.ascontiguousarray(np.concatenate(pos)), dtype=torch.float64,
                                   device=dev)
        self.n_rows = int(self.pos.shape[0])
        self.pS = self._neighbours_cells(self.R_S)
        self.pH = self._neighbours_cells(self.R_H)
        self.pL = self._neighbours_cells(self.R_L)
        # spatial index: one index cell per batch cell (their patterns are
        # block diagonal, so each row's window is its own cell)
        nc = len(cells)
        units = np.zeros((self.n_rows, 3))
        units[:, 0] = np.repeat(np.arange(nc), np.diff(self.cell_rows)) + 0.5
        units[:, 1:] = 0.5
        self.ix_cells = Cells(units, (float(nc), 1.0, 1.0), (nc, 1, 1), 0, dev,
                              origin=(0.0, 0.0, 0.0))
        for P in (self.pS, self.pH, self.pL):
            P.cells = self.ix_cells
        self.S = self.synth_values(0, self.pS, self.R_S, 3.0, None)
        self.H = self.synth_values(1, self.pH, self.R_H, 2.5, None)

    def _index_ranges(self):
        """Ranges of the patterns that get a spatial index (S, H, L and the
        products), for the choice of its grid."""
        rs, rh, rl = self.R_S, self.R_H, self.R_L
        rxz = rs + 2 * rl
        return (rs, rh, rl, rs + rl, min(rh + rl + rs, rxz), min(2 * rs + rl, rxz), 2 * rl,
                2 * rl + rs, rh + rl)

    def _range_pattern(self, R):
        """Range pattern of cutoff R over the system's rows (one cell, or
        every cell of a batch on its own)."""
        if self.cells is not None:
            return self._neighbours_cells(R)
        return neighbours(self.pos, self.box, R)

    def _neighbours_cells(self, R):
        n, nc = self.n_rows, len(self.cells)
        rp = torch.empty(n + 1, dtype=torch.int32, device=self.dev)
        nnz = c_int64(0)
        args = (_ptr(self.pos), n, nc, _ptr(self.cell_start), _ptr(self.cell_of), _ptr(self.boxes),
                float(R))
        L_.call("lnv_neighbours_cells", *args, _ptr(rp), None, 0, byref(nnz), _stream())
        col = torch.empty(max(1, nnz.value), dtype=torch.int32, device=self.dev)
        L_.call("lnv_neighbours_cells", *args, _ptr(rp), _ptr(col), nnz.value, byref(nnz),
                _stream())
        return Pattern(n, rp, col[:nnz.value])

    def cell_item_ptr(self):
        """Work items of L's pattern per cell (device [n_cells+1])."""
        if getattr(self, "_cell_items", None) is None:
            rows = self.pL.items.view(-1, 2)[:, 0].cpu().numpy()
            ptr = np.searchsorted(rows, self.cell_rows, side="left").astype(np.int32)
            self._cell_items = torch.as_tensor(ptr, device=self.dev)
        return self._cell_items

    def cell_energies(self, mixed=False):
        """Per-cell (E, N) of a batch at the current L: one evaluation of the
        whole batch (lnv_eval or lnv_eval_mixed), then lnv_cell_traces."""
        if self.cells is None:
            raise ValueError("not a batch of cells")
        self.eval_mixed() if mixed else self.eval()
        out = torch.empty(len(self.cells), 2, dtype=torch.float64, device=self.dev)
        L_.call("lnv_cell_traces", byref(self.pL.struct), byref(self.ws.ev), len(self.cells),
                _ptr(self.cell_item_ptr()), _ptr(out), _stream())
        return out

    # ----------------------------------------------------------- adjoint set-up
    def adjoint_setup(self):
        """Patterns and buffers of lnv_adjoint: natural pat(L.S.L) and pat(H.L),
        work lists of S's pattern, and the scratch on S's pattern.  The S.L
        values share the evaluation's buffer (both are recomputed per call)."""
        if self.adj_ws is not None:
            return
        dev = self.dev
        self.pLSL = product_pattern(self.pL, self.pSL)           # L.S.L
        self.pHL = product_pattern(self.pH, self.pL)             # H.L
        self.pLH = product_pattern(self.pL, self.pH, triples=False)   # L.H = pat(H.L)^T
        self.pLH.build_index()
        self.perm_HL = transpose_map(self.pHL, self.pLH)
        # the restricted products with L.S.L take it on the right: P_H(LS.LSL),
        # P_S(LH.LSL) (the transposes LS, LH are formed per call)
        self.triples.update(
            LSL=self.pLSL.triples, HL=self.pHL.triples,
            dH4=product_pattern(self.pLS, self.pLSL, mask=self.pH).triples,
            dH6=product_pattern(self.pL, self.pSL, mask=self.pH).triples,
            dS4=product_pattern(self.pLH, self.pLSL, mask=self.pS).triples,
            dS6=product_pattern(self.pL, self.pHL, mask=self.pS).triples,
        )
        self.pSL.build_index()
        self.pLSL.build_index().build_items()
        self.pLS.build_items()
        self.pLH.build_items()
        self.pHL.build_index().build_items()
        self.pS.build_index().build_items()
        adj_upper = []
        if self.symmetric:
            # halves of the symmetric adjoint products (L.S.L and H get index
            # tables)
            self.pLSL.build_index()
            self.pH.build_index()
            self.pLSLu, self.pHu, self.pSu = (half_pattern(P) for P in
                                              (self.pLSL, self.pH, self.pS))
            adj_upper = [self.pLSLu, self.pHu, self.pSu]
            self.triples_upper.update(
                LSL=product_pattern(self.pL, self.pSL, mask=self.pLSLu).triples,
                dH4=product_pattern(self.pLS, self.pLSL, mask=self.pHu).triples,
                dH6=product_pattern(self.pL, self.pSL, mask=self.pHu).triples,
                dS6=product_pattern(self.pL, self.pHL, mask=self.pSu).triples)
        if self.cluster is not None:
            # left operands L.S.L, L.S, L.H and outputs H.L (and the halves)
            # take part in clustered products
            self.pLSL.build_cluster(*self.cluster)
            self.pHL.build_cluster(*self.cluster)
            self.pLS.build_cluster(*self.cluster)
            self.pLH.build_cluster(*self.cluster)
            if self.cluster[0] == 16:
                self.pSL.check_tile4()
            for P in adj_upper:
                P.build_cluster(*self.cluster)
        self.LSL = Matrix(self.pLSL)
        self.HL = Matrix(self.pHL)
        self.YS = torch.zeros(self.pS.nnzb, BLK, BLK, dtype=torch.float64, device=dev)
        self.adj_ws = L_.LnvAdjWs()
        self.adj_ws.SL = self.SL.struct
        self.adj_ws.LSL = self.LSL.struct
        self.adj_ws.HL = self.HL.struct
        self.adj_ws.YS = self.YS.data_ptr()
        # transposes of S.L (the evaluation's L.S buffer, recomputed per call)
        # and of H.L
        self.LH = Matrix(self.pLH)
        self.adj_ws.LS = self.LS.struct
        self.adj_ws.perm_SL = self.perm_SL.data_ptr()
        self.adj_ws.LH = self.LH.struct
        self.adj_ws.perm_HL = self.perm_HL.data_ptr()
        if self.symmetric:
            self.LSLu, self.Hu, self.Su = (Matrix(P) for P in adj_upper)
            self.adj_ws.LSLu = self.LSLu.struct
            self.adj_ws.Hu = self.Hu.struct
            self.adj_ws.Su = self.Su.struct
        torch.cuda.synchronize()

    def adjoint_flops(self, dS=True, dH=True, padded=False):
        """Algorithmic flops of one lnv_adjoint call."""
        t = self._weights(padded)
        tot = t["SL"] + t["LSL"]
        if dH:
            tot += t["dH4"] + t["dH6"]
        if dS:
            tot += t["HL"] + t["dS4"] + t["dS6"]
        return tot

    def adjoint(self, L, S, H, dS=None, dH=None, dNS=None):
        """dE/dS (into dS, on S's pattern), dE/dH (into dH, on H's pattern) and
        dN/dS (into dNS) at the values L, S, H (tensors [nnzb, 4, 4] on this
        system's patterns)."""
        self.adjoint_setup()
        Lm, Sm, Hm = bsm(self.pL, L), bsm(self.pS, S), bsm(self.pH, H)
        ref = [byref(bsm(P, t).struct) if t is not None else None
               for P, t in ((self.pS, dS), (self.pH, dH), (self.pS, dNS))]
        L_.call("lnv_adjoint", byref(Lm.struct), byref(Sm.struct), byref(Hm.struct), *ref,
                byref(self.adj_ws), _stream())
        return dS, dH

    # ----------------------------------------------------------- forces
    def _segments(self):
        """Stored rows of each atom (consecutive): (seg_ptr, seg_atom) on device."""
        if getattr(self, "_seg", None) is None:
            if self.atom_of is None:
                atom = np.arange(self.n_rows)
            else:
                atom = self.atom_of.cpu().numpy()
            first = np.concatenate([[True], atom[1:] != atom[:-1]])
            starts = np.nonzero(first)[0]
            seg_ptr = np.append(starts, len(atom)).astype(np.int32)
            seg_atom = atom[starts].astype(np.int32)
            assert len(np.unique(seg_atom)) == len(seg_atom) == self.n
            self._seg = (torch.as_tensor(seg_ptr, device=self.dev),
                         torch.as_tensor(seg_atom, device=self.dev))
        return self._seg

    def forces(self, L=None, mu=None):
        """Forces on the atoms [n_atoms, 3] (Hartree/bohr, original atom order)
        from the synthetic S(x), H(x) at fixed L (default: the current L):
        -dE/dx, or with mu the force of a minimum under N = N_e, -(dE/dx -
        mu dN/dx).  Adjoint (lnv_adjoint) plus lnv_forces."""
        if self.cells is not None:
            raise NotImplementedError("forces of a batch of cells")
        self.adjoint_setup()
        self.pH.build_index()
        Lv = self.L.val if L is None else L
        dS = torch.empty_like(self.S.val)
        dH = torch.empty_like(self.H.val)
        dNS = torch.empty_like(self.S.val) if mu is not None else None
        self.adjoint(Lv, self.S.val, self.H.val, dS=dS, dH=dH, dNS=dNS)
        seg_ptr, seg_atom = self._segments()
        acc = torch.empty(self.n_rows * 3, dtype=torch.float64, device=self.dev)
        F = torch.empty(self.n, 3, dtype=torch.float64, device=self.dev)
        box_c = (c_double * 3)(*self.box)
        gS, gH = bsm(self.pS, dS), bsm(self.pH, dH)
        gN = bsm(self.pS, dNS) if dNS is not None else None
        L_.call("lnv_forces", _ptr(self.pos), box_c, _ptr(self.nfun), _ptr(self.atom_of),
                _ptr(self.off_of), int(self.seed), float(self.scale), byref(gS.struct),
                byref(gN.struct) if gN is not None else None, float(mu or 0.0),
                float(self.R_S), 3.0, byref(gH.struct), float(self.R_H), 2.5,
                int(seg_ptr.numel() - 1), _ptr(seg_ptr), _ptr(seg_atom), _ptr(acc), _ptr(F),
                _stream())
        return F

    def move_atoms(self, pos):
        """New atomic positions [n_atoms, 3] (original order): S and H are
        generated again at the new positions on the existing range patterns
        (the caller keeps the displacement below the distance of every pair
        from its cutoff, or builds a new system)."""
        if self.cells is not None:
            raise NotImplementedError("moving the atoms of a batch of cells")
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        rows = pos if self.atom_of is None else pos[self.atom_of.cpu().numpy()]
        self.pos.copy_(torch.as_tensor(np.ascontiguousarray(rows)))
        self.S.rebind(self.synth_values(0, self.pS, self.R_S, 3.0).val)
        self.H.rebind(self.synth_values(1, self.pH, self.R_H, 2.5).val)
        self.ws.ev.carry = 0     # S.L and S.L.S of the old S are stale

    def eval_values(self, L, S, H, G, F, EN):
        """lnv_eval at the given value tensors (on this system's patterns)."""
        Lm, Sm, Hm = bsm(self.pL, L), bsm(self.pS, S), bsm(self.pH, H)
        Gm, Fm = bsm(self.pL, G), bsm(self.pL, F)
        L_.call("lnv_eval", byref(Lm.struct), byref(Sm.struct), byref(Hm.struct),
                byref(Gm.struct), byref(Fm.struct), _ptr(EN), byref(self.ws.ev), _stream())
        return EN

    # ----------------------------------------------------------- flop accounting
    def _weights(self, padded):
        """Flops per product: 2 * 4^3 per stored block triple (padded), or the
        algorithmic count with the functions each stored row holds."""
        if padded or not self.split:
            t = dict(self.triples)
            t["Vf"] = t["V"]               # P_L(SL.Z) in full (trace products)
            t["Wf"] = t["W"]               # P_L(SL.X) in full (trace product)
            if self.symmetric:
                t.update(self.triples_upper)
            return {k: 2 * BLK ** 3 * v for k, v in t.items()}
        return self._alg_flops()

    def _alg_flops(self, only=None):
        """Algorithmic flops per product (cached); only: the keys to compute
        now (all by default)."""
        if getattr(self, "_alg", None) is None:
            self._alg = {}
        up = self.pLu if self.symmetric else self.pL     # symmetric products: halves
        specs = {"SL": (self.pS, self.pL, None), "X": (self.pH, self.pLS, self.pX),
                 "Z": (self.pS, self.pLS, self.pZu), "YT": (self.pSL, self.pXT, self.pL),
                 "W": (self.pSL, self.pX, up), "V": (self.pSL, self.pZ, up),
                 "Vf": (self.pSL, self.pZ, self.pL), "Wf": (self.pSL, self.pX, self.pL)}
        if self.metric is not None:
            specs.update(TG=(self.pL, self.pL, None), TGT=(self.pL, self.pLL, up))
        if getattr(self, "adj_ws", None) is not None:
            sym = self.symmetric
            mL, mH, mS = ((self.pLSLu, self.pHu, self.pSu) if sym else (None, self.pH, self.pS))
            specs.update(LSL=(self.pL, self.pSL, mL), HL=(self.pH, self.pL, None),
                         dH4=(self.pLS, self.pLSL, mH), dH6=(self.pL, self.pSL, mH),
                         dS4=(self.pLH, self.pLSL, self.pS), dS6=(self.pL, self.pHL, mS))
        fun = self.fun_rows
        for k, (A, B, M) in specs.items():
            if only is not None and k not in only:
                continue
            if k not in self._alg:
                f = c_int64(0)
                L_.call("lnv_pattern_flops", byref(A.struct), byref(B.struct),
                        byref(M.struct) if M is not None else None, _ptr(fun), byref(f),
                        _stream())
                self._alg[k] = f.value
        return self._alg

    def flops(self, what="eval", padded=False):
        """Algorithmic flops (2 n_i n_k n_j per block triple, the functions
        present) of one piece of work: "eval", "init" (L0), "step_base" (an
        FP64 CG step after the first of a minimisation, without the
        electron-number correction: its S.L and S.L.S come from the previous
        step and the check's S.L_new from the line search's S.D, by
        linearity), "first_extra" (the S.L and S.L.S products the first step
        and each reset step form), "ncorr" (the
        correction), "step" (step_base + ncorr).  padded=True: 2 * 4^3 per
        stored triple, the arithmetic the kernels do (the same unless atoms
        are split)."""
        t = self._weights(padded)
        ev = t["SL"] + t["X"] + t["Z"] + t["YT"] + t["W"] + t["V"]
        nchk = t["SL"] + t["Z"] + t["V"]
        if self.symmetric:
            # traces of the cubics: the symmetric A_P^T X_P on the half of L's
            # pattern, plus (energy line) S L X_P in full
            line = t["SL"] + t["X"] + t["W"] + t["Wf"]
            ncor = t["SL"] + t["Z"] + t["V"]
            init = t["SL"] + t["Z"] + t["V"]
        else:
            line = t["SL"] + t["X"] + 2 * t["YT"]
            ncor = t["SL"] + t["Z"] + 2 * t["Vf"]
            init = t["SL"] + t["Z"] + t["Vf"]
        met = 2 * (t["TG"] + t["TGT"]) if self.metric is not None else 0
        tot = {"eval": ev, "init": init,
               "step_base": ev + met + line + nchk - 2 * t["SL"] - t["Z"], "ncorr": ncor,
               "first_extra": t["SL"] + t["Z"],
               "step": ev + met + line + nchk - 2 * t["SL"] - t["Z"] + ncor}[what]
        return tot

    # ----------------------------------------------------------- hot path
    def eval(self):
        L_.call("lnv_eval", byref(self.L.struct), byref(self.S.struct), byref(self.H.struct),
                byref(self.G.struct), byref(self.F.struct), _ptr(self.EN), byref(self.ws.ev),
                _stream())
        return self.EN

    def _T(self):
        return byref(self.T.struct) if self.metric is not None else None

    def _need_cg(self):
        if self.lean:
            raise RuntimeError("a lean system is evaluated, not minimised (no CG buffers)")

    def batch(self):
        """The lnv_batch descriptor of a batch of cells (built once): L's work
        items and values per cell, the cell of each row, each cell's electron
        count and its scalar block (cell_scalars)."""
        if self.cells is None:
            raise ValueError("not a batch of cells")
        if getattr(self, "_batch", None) is None:
            rp = self.pL.row_ptr.cpu().numpy().astype(np.int64)
            self._val_ptr = torch.as_tensor(16 * rp[self.cell_rows], device=self.dev)
            self._n_elec_cells = torch.as_tensor(
                np.array([c.n_elec for c in self.cells], dtype=np.float64), device=self.dev)
            self._n_orb_cells = torch.as_tensor(
                np.array([float(np.sum(c.nfun)) for c in self.cells], dtype=np.float64),
                device=self.dev)
            self.cell_scalars = torch.zeros(len(self.cells), L_.NSCALARS, dtype=torch.float64,
                                            device=self.dev)
            b = L_.LnvBatch()
            b.n_cells = len(self.cells)
            b.item_ptr = self.cell_item_ptr().data_ptr()
            b.val_ptr = self._val_ptr.data_ptr()
            b.row_cell = self.cell_of.data_ptr()
            b.n_elec = self._n_elec_cells.data_ptr()
            b.scalars = self.cell_scalars.data_ptr()
            b.row_off = self.cell_start.data_ptr()
            b.n_orb = self._n_orb_cells.data_ptr()
            self._batch = b
        return self._batch

    def cg_init(self):
        """L0 = lambda T (lnv_cg_init; T = I without a metric); for a batch of
        cells lambda_c T per cell (lnv_cg_init_batch)."""
        self._need_cg()
        if self.cells is not None:
            L_.call("lnv_cg_init_batch", byref(self.L.struct), byref(self.S.struct), self._T(),
                    byref(self.batch()), byref(self.ws), _stream())
        else:
            L_.call("lnv_cg_init", byref(self.L.struct), byref(self.S.struct), self._T(),
                    self.n_elec, byref(self.ws), _stream())
        self.k = 0

    def cg_restart(self):
        """Start a new minimisation from the current L (e.g. a purified start):
        the next step is iteration 0 (steepest descent, no history) with the
        status bits cleared."""
        blocks = [self.scalars]
        if self.cells is not None:
            self.batch()
            blocks = [self.cell_scalars[c] for c in range(len(self.cells))]
        for sc in blocks:
            sc[L_.SC["STATUS"]] = 0.0
            sc[L_.SC["FORCE_RESET"]] = 0.0
            sc[L_.SC["E_PREV"]] = float("nan")
            sc[L_.SC["RISES"]] = 0.0
            sc[L_.SC["GUARD_K"]] = -1e9
        self.ws.ev.carry = 0
        self.k = 0

    def cg_check(self):
        """Synchronise and raise LnvError (LNV_ENUMERIC) when the minimisation
        produced a non-finite value or its runaway guard tripped twice within a
        reset period; returns the status bits otherwise."""
        bits = c_int32(0)
        L_.call("lnv_cg_check", _ptr(self.scalars), byref(bits), _stream())
        return bits.value

    def occupation_bounds(self, steps=32, L=None):
        """(smallest, largest) occupation number of L S from `steps` Lanczos
        steps (lnv_occupation_bounds); L: the current L by default."""
        out = torch.zeros(2, dtype=torch.float64, device=self.dev)
        M = self.L if L is None else Matrix(self.pL, L)
        L_.call("lnv_occupation_bounds", byref(M.struct), byref(self.S.struct), int(steps),
                _ptr(self.lanczos), _ptr(out), _stream())
        return tuple(float(x) for x in out.cpu())

    def cg_step(self):
        self._need_cg()
        o = L_.LnvOpts(self.opts.reset_period, self.opts.n_tol, self.opts.step_cap, None,
                       int(self.opts.occ_every), int(self.opts.occ_iter))
        if self.cells is not None:
            # every cell minimised at once with its own scalars (FP64)
            if self.opts.mixed:
                raise NotImplementedError("a batch of cells is minimised in FP64")
            L_.call("lnv_cg_step_batch", byref(self.L.struct), byref(self.S.struct),
                    byref(self.H.struct), self._T(), byref(self.batch()), self.k, byref(o),
                    byref(self.ws), _stream())
            self.k += 1
            return
        if self.opts.mixed:
            self.mixed_setup()
            o.eval32 = ctypes.addressof(self.ws32)
        L_.call("lnv_cg_step", byref(self.L.struct), byref(self.S.struct), byref(self.H.struct),
                self._T(), self.n_elec, self.k, byref(o), byref(self.ws), _stream())
        self.k += 1

    def scalar(self, name):
        return float(self.scalars[L_.SC[name]].item())

    def scalars_host(self):
        v = self.scalars.cpu().numpy()
        return {k: float(v[i]) for k, i in L_.SC.items()}

    def cell_scalars_host(self):
        """Per-cell scalar blocks of a batch minimisation (list of dicts)."""
        v = self.cell_scalars.cpu().numpy()
        return [{k: float(r[i]) for k, i in L_.SC.items()} for r in v]

    def buffer(self, ptr):
        return self._bufs[ptr]
