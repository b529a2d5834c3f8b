"""A 13/9/4-function Si/O/H cell built and evaluated through the C ABI alone
(atoms with their own support-function counts, Sec. II.B; the evaluation of
Sec. II.C.2, Eq. 4), against the oracle.

Between the library calls there is only marshalling: device memory from
torch, the two-phase size queries, the ctypes structs (the pattern and
matrix wrappers of the binding).  The atoms-to-rows layout comes from
lnv_atoms_layout (atoms stored in a permuted order), the row positions from
lnv_atoms_rows, the range patterns from lnv_neighbours, S, H and the test L
from lnv_synth_blocks on those rows (the test L: the overlap generator with
master seed + 1000, range R_L and decay 3, times 0.1 through lnv_bsm_lincomb;
the oracle draws the same counters itself), and G and F come back as atom
blocks of n_i x n_j values through lnv_vbsm_unpack on the atom pattern that
lnv_neighbours gives for the atoms.  The oracle's own S goes in through
lnv_vbsm_pack and must equal the library's S.
"""
import ctypes
import dataclasses
from ctypes import byref, c_int32, c_int64

import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost

pytestmark = pytest.mark.gpu

L_SEED_OFFSET = 1000
L_SCALE = 0.1


def _lib():
    from paper_2002_07704_amd import lib as L_
    return L_


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Built:
    """The cell on the device, every step a library call."""

    def __init__(self, w, order):
        from paper_2002_07704_amd import system as sy
        L_ = _lib()
        dev = "cuda"
        self.w = w
        n = w.n
        self.nfun = torch.as_tensor(np.asarray(w.nfun, dtype=np.int32), device=dev)
        self.order = torch.as_tensor(np.asarray(order, dtype=np.int32), device=dev)
        self.row_start = torch.empty(n + 1, dtype=torch.int32, device=dev)
        nr = c_int32(0)
        L_.call("lnv_atoms_layout", _ptr(self.nfun), n, _ptr(self.order), _ptr(self.row_start),
                None, None, 0, byref(nr), _stream())
        self.n_rows = nr.value
        self.atom_of = torch.empty(self.n_rows, dtype=torch.int32, device=dev)
        self.off_of = torch.empty(self.n_rows, dtype=torch.int32, device=dev)
        L_.call("lnv_atoms_layout", _ptr(self.nfun), n, _ptr(self.order), _ptr(self.row_start),
                _ptr(self.atom_of), _ptr(self.off_of), self.n_rows, byref(nr), _stream())
        self.atoms = L_.LnvAtoms(n, self.n_rows, self.nfun.data_ptr(), self.row_start.data_ptr(),
                                 self.atom_of.data_ptr(), self.off_of.data_ptr())
        self.atom_pos = torch.as_tensor(np.ascontiguousarray(w.pos), device=dev)
        self.row_pos = torch.empty(self.n_rows, 3, dtype=torch.float64, device=dev)
        L_.call("lnv_atoms_rows", byref(self.atoms), _ptr(self.atom_pos), _ptr(self.row_pos),
                _stream())
        # range patterns over the stored rows, their indices and work lists
        P = {k: sy.neighbours(self.row_pos, w.box, R)
             for k, R in (("S", w.R_S), ("H", w.R_H), ("L", w.R_L))}
        P["SL"] = sy.product_pattern(P["S"], P["L"])
        P["LS"] = sy.product_pattern(P["L"], P["S"], triples=False)
        P["X"] = sy.product_pattern(P["H"], P["LS"])
        P["Z"] = sy.product_pattern(P["S"], P["LS"])
        P["XT"] = sy.product_pattern(P["SL"], P["H"], triples=False)
        for k in ("S", "H", "L", "SL", "LS", "X", "Z", "XT"):
            P[k].build_index()
        for k in ("L", "SL", "X", "Z", "S", "H"):
            P[k].build_items()
        self.P = P
        self.M = {}
        for k in ("S", "H", "L"):
            self.M[k] = sy.Matrix(P[k])
        self.M["G"], self.M["F"] = sy.Matrix(P["L"]), sy.Matrix(P["L"])
        box = (ctypes.c_double * 3)(*[float(b) for b in w.box])
        for k, kind, R, decay, seed in (("S", 0, w.R_S, 3.0, w.seed), ("H", 1, w.R_H, 2.5, w.seed),
                                        ("L", 0, w.R_L, 3.0, w.seed + L_SEED_OFFSET)):
            L_.call("lnv_synth_blocks", _ptr(self.row_pos), box, _ptr(self.nfun),
                    _ptr(self.atom_of), _ptr(self.off_of), byref(self.M[k].struct), kind,
                    float(R), decay, seed, float(w.scale), _stream())
        Lm = self.M["L"]
        L_.call("lnv_bsm_lincomb", L_SCALE, byref(Lm.struct), 0.0, None, 0.0, None,
                byref(Lm.struct), _stream())

    def evaluate(self):
        from paper_2002_07704_amd import system as sy
        L_ = _lib()
        P, dev = self.P, "cuda"
        inter = {k: sy.Matrix(P[k]) for k in ("SL", "LS", "X", "XT", "Z")}
        nL = P["L"].nnzb
        bufs = [torch.zeros(nL, 4, 4, dtype=torch.float64, device=dev) for _ in range(3)]
        plen = L_.load().lnv_partials_len(P["L"].struct.n_items)
        part = torch.zeros(plen, dtype=torch.float64, device=dev)
        scal = torch.zeros(L_.NSCALARS, dtype=torch.float64, device=dev)
        EN = torch.zeros(2, dtype=torch.float64, device=dev)
        perm_SL = sy.transpose_map(P["SL"], P["LS"])
        perm_X = sy.transpose_map(P["X"], P["XT"])
        ev = L_.LnvEvalWs()
        for k in ("SL", "LS", "X", "XT", "Z"):
            setattr(ev, k, inter[k].struct)
        ev.perm_SL, ev.perm_X = perm_SL.data_ptr(), perm_X.data_ptr()
        ev.YT, ev.W, ev.V = (b.data_ptr() for b in bufs)
        ev.partials, ev.partials_len, ev.scalars = part.data_ptr(), plen, scal.data_ptr()
        M = self.M
        L_.call("lnv_eval", byref(M["L"].struct), byref(M["S"].struct), byref(M["H"].struct),
                byref(M["G"].struct), byref(M["F"].struct), _ptr(EN), byref(ev), _stream())
        torch.cuda.synchronize()
        self._keep = (inter, bufs, part, scal, perm_SL, perm_X)
        return EN.cpu().numpy()

    def atom_pattern(self, R):
        """The atoms' own range pattern (lnv_neighbours on atom positions)."""
        from paper_2002_07704_amd import system as sy
        return sy.neighbours(self.atom_pos, self.w.box, R)

    def vbsm(self, rp, col, dtype=torch.float64):
        """Zeroed atom-blocked matrix on an atom pattern (lnv_vbsm_offsets)."""
        L_ = _lib()
        nnz = int(col.numel())
        off = torch.empty(nnz + 1, dtype=torch.int64, device="cuda")
        ln = c_int64(0)
        L_.call("lnv_vbsm_offsets", byref(self.atoms), _ptr(rp), _ptr(col), nnz, _ptr(off),
                byref(ln), _stream())
        val = torch.zeros(max(1, ln.value), dtype=dtype, device="cuda")
        st = L_.LnvVbsm(ctypes.pointer(self.atoms), rp.data_ptr(), col.data_ptr(),
                        off.data_ptr(), nnz, L_.F64 if dtype == torch.float64 else L_.F32,
                        val.data_ptr())
        return st, off, val

    def unpack(self, M, rp, col):
        L_ = _lib()
        st, off, val = self.vbsm(rp, col)
        L_.call("lnv_vbsm_unpack", byref(M.struct), byref(st), _stream())
        torch.cuda.synchronize()
        return off.cpu().numpy(), val.cpu().numpy()


def _blocks_vs_dense(off, val, rp, col, nfun, D):
    """Largest |difference| between atom blocks (offsets off into val) and
    the dense matrix D over the pattern."""
    o = ost.offsets(nfun)
    worst = 0.0
    for i in range(len(nfun)):
        for p in range(rp[i], rp[i + 1]):
            j = col[p]
            b = val[off[p]:off[p + 1]].reshape(nfun[i], nfun[j])
            worst = max(worst, float(np.abs(b - D[o[i]:o[i + 1], o[j]:o[j + 1]]).max()))
    return worst


@pytest.fixture(scope="module")
def cell():
    w = W.amorphous_workload("siOH48", 48, seed=21)
    # atoms stored sorted along x (a permutation of the atom order)
    order = np.argsort(w.pos[:, 0], kind="stable")
    b = Built(w, order)
    osys = ost.System(w)
    w2 = dataclasses.replace(w, seed=w.seed + L_SEED_OFFSET, R_S=w.R_L)
    Lb = L_SCALE * ost.synth_blocks(w2, "S", *osys.pat["L"])
    Ld = ost.blocks_to_dense(Lb, *osys.pat["L"], w.nfun)
    return b, osys, Ld


def test_layout_rows_follow_the_order(cell):
    b, _, _ = cell
    w = b.w
    nf = np.asarray(w.nfun)
    assert set(nf.tolist()) == {4, 9, 13}
    order = b.order.cpu().numpy()
    rs = b.row_start.cpu().numpy()
    ao, oo = b.atom_of.cpu().numpy(), b.off_of.cpu().numpy()
    assert b.n_rows == int(((nf + 3) // 4).sum()) == rs[-1]
    r = 0
    for a in order:                       # atoms in storage order, rows consecutive
        k = (nf[a] + 3) // 4
        assert rs[a] == r
        assert (ao[r:r + k] == a).all() and (oo[r:r + k] == 4 * np.arange(k)).all()
        r += k
    rp = b.row_pos.cpu().numpy()
    assert np.array_equal(rp, w.pos[ao])


def test_atom_pattern_is_the_oracle_pattern(cell):
    b, osys, _ = cell
    for R, name in ((b.w.R_S, "S"), (b.w.R_L, "L")):
        P = b.atom_pattern(R)
        rp, col = P.host()
        assert np.array_equal(rp, osys.pat[name][0]) and np.array_equal(col, osys.pat[name][1])


def test_pack_of_oracle_S_is_the_library_S(cell):
    b, osys, _ = cell
    L_ = _lib()
    rp, col = osys.pat["S"]
    rp_d = torch.as_tensor(np.asarray(rp, dtype=np.int32), device="cuda")
    col_d = torch.as_tensor(np.asarray(col, dtype=np.int32), device="cuda")
    st, off, val = b.vbsm(rp_d, col_d)
    offh = off.cpu().numpy()
    nf = np.asarray(b.w.nfun)
    flat = np.zeros(int(offh[-1]))
    for i in range(b.w.n):
        for p in range(rp[i], rp[i + 1]):
            j = col[p]
            flat[offh[p]:offh[p + 1]] = osys.Sb[p, :nf[i], :nf[j]].ravel()
    val.copy_(torch.as_tensor(flat))
    from paper_2002_07704_amd import system as sy
    packed = sy.Matrix(b.P["S"])
    packed.val.fill_(np.nan)
    L_.call("lnv_vbsm_pack", byref(st), byref(packed.struct), _stream())
    torch.cuda.synchronize()
    lib_S = b.M["S"].val.cpu().numpy()
    got = packed.val.cpu().numpy()
    assert np.isfinite(got).all()
    assert np.abs(got - lib_S).max() <= 1e-14 * np.abs(lib_S).max()
    # and back: unpack(pack(A)) is A exactly
    o2, v2 = b.unpack(packed, rp_d, col_d)
    assert np.array_equal(o2, offh) and np.array_equal(v2[:len(flat)], flat)


def test_eval_through_the_abi_matches_the_oracle(cell):
    b, osys, Ld = cell
    w = b.w
    EN = b.evaluate()
    E, N, G, F = olnv.evaluate(Ld, osys.S, osys.H, osys.maskL)
    assert abs(EN[0] - E) / w.n <= 1e-10
    assert abs(EN[1] - N) / w.n <= 1e-10
    PLa = b.atom_pattern(w.R_L)
    rp, col = PLa.host()
    nf = np.asarray(w.nfun)
    for name, ref in (("G", G), ("F", F)):
        off, val = b.unpack(b.M[name], PLa.row_ptr, PLa.col)
        assert _blocks_vs_dense(off, val, rp, col, nf, ref) <= 1e-10 * np.abs(ref).max(), name


def _pack_host(b, blocks, rp, col, P, dtype):
    """Oracle blocks ([nnz, p, p] on the atom pattern rp/col, host) packed
    through lnv_vbsm_pack into a stored-row matrix on the row pattern P."""
    from paper_2002_07704_amd import system as sy
    L_ = _lib()
    rp_d = torch.as_tensor(np.asarray(rp, dtype=np.int32), device="cuda")
    col_d = torch.as_tensor(np.asarray(col, dtype=np.int32), device="cuda")
    st, off, val = b.vbsm(rp_d, col_d, dtype)
    offh = off.cpu().numpy()
    nf = np.asarray(b.w.nfun)
    flat = np.zeros(int(offh[-1]))
    for i in range(b.w.n):
        for p in range(rp[i], rp[i + 1]):
            flat[offh[p]:offh[p + 1]] = blocks[p, :nf[i], :nf[col[p]]].ravel()
    val.copy_(torch.as_tensor(flat).to(dtype))
    M = sy.Matrix(P, torch.full((P.nnzb, 4, 4), float("nan"), dtype=dtype, device="cuda"))
    L_.call("lnv_vbsm_pack", byref(st), byref(M.struct), _stream())
    torch.cuda.synchronize()
    return M


def test_fp32_operands_into_fp64_product(cell):
    """C = S32 L32 in FP64 (FP32 A and B, FP64 C) on the oracle's S and L
    rounded to FP32 on the host: every product of FP32 values is exact in
    FP64, so C is the FP64 product of the rounded matrices up to the order
    of the FP64 sums."""
    b, osys, Ld = cell
    from paper_2002_07704_amd import system as sy
    L_ = _lib()
    P = b.P
    Lb = ost.dense_to_blocks(Ld, *osys.pat["L"], b.w.nfun)
    S32 = _pack_host(b, osys.Sb.astype(np.float32), *osys.pat["S"], P["S"], torch.float32)
    L32 = _pack_host(b, Lb.astype(np.float32), *osys.pat["L"], P["L"], torch.float32)
    C = sy.Matrix(P["SL"])
    nb = c_int64(-1)
    L_.call("lnv_multiply_ws_bytes", byref(S32.struct), byref(L32.struct), 0, byref(C.struct), 0,
            byref(nb))
    assert nb.value == 0
    L_.call("lnv_multiply_ws_bytes", byref(S32.struct), byref(L32.struct), 0, byref(C.struct), 1,
            byref(nb))
    assert nb.value == 16 * P["SL"].struct.n_items
    L_.call("lnv_bsm_multiply", 1.0, byref(S32.struct), byref(L32.struct), 0, 0.0,
            byref(C.struct), _stream())
    # the oracle: dense FP64 product of the FP32-rounded matrices on the
    # atoms' pattern of S.L
    S_r = osys.S.astype(np.float32).astype(np.float64)
    L_r = Ld.astype(np.float32).astype(np.float64)
    ref = S_r @ L_r
    PS, PL = b.atom_pattern(b.w.R_S), b.atom_pattern(b.w.R_L)
    PSL = sy.product_pattern(PS, PL, triples=False)
    rp, col = PSL.host()
    off, val = b.unpack(C, PSL.row_ptr, PSL.col)
    err = _blocks_vs_dense(off, val, rp, col, np.asarray(b.w.nfun), ref)
    assert err <= 1e-13 * np.abs(ref).max()
    # a mix other than FP32 x FP32 -> FP64 is refused before any launch
    with pytest.raises(L_.LnvError) as e:
        L_.call("lnv_bsm_multiply", 1.0, byref(S32.struct), byref(b.M["L"].struct), 0, 0.0,
                byref(C.struct), _stream())
    assert e.value.status == L_.EUNSUPPORTED
