"""Atom-tile multiply: atoms with 13 support functions (stored as 4 rows of 4,
padded to 16) multiplied as whole 16x16 atom tiles on the matrix cores.

Cells, each with every atom at 13 functions and the 13-function workload's
ranges (S 12, H 14, L 10 bohr):
* 64-atom diamond Si (16 clusters of 4 atoms);
* 22 atoms of an amorphous cell (the last 4-atom cluster holds 2 atoms);
* one atom in a small periodic cell (one cluster holding one atom, every
  block a sum over many images).

Checks: with each tile shape, E, N, G, F against the oracle at a seeded L
(|dE|, |dN| <= 1e-10 per atom, G and F 1e-12 relative, padding exactly zero)
and against the 4x4 path on the same L; Hotelling-metric CG iterations and the
adjoint against the oracle; the three mixed-precision modes of the tiles
(FP32 MFMA, FP32 storage with FP64 MFMA, FP16 hi/lo split) within 1e-6 Ha/atom
of the oracle's energy, N, G and F within the FP32 rounding bound 3 sqrt(k) u
(u = 2^-22 for the hi/lo split).  At 8192 atoms (the 13-function workload at a quarter
of its size) the tile evaluation is compared with the 4x4 path's.
"""
import math

import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost
from paper_2002_07704_amd import lib as L_
from test_gpu_split import Layout, _rand_sym

pytestmark = pytest.mark.gpu

SHAPES = [(16, 4), (16, 8)]
ACC_F32, ACC_F64, ACC_F16X3 = 0, 1, 2


def _w13(name, pos, box, seed):
    n = pos.shape[0]
    return W.Workload(name=name, pos=np.mod(pos, box), box=np.asarray(box, dtype=np.float64),
                      nfun=np.full(n, 13, dtype=np.int32), species=np.zeros(n, dtype=np.int8),
                      R_S=12.0, R_H=14.0, R_L=10.0, n_elec=4 * n, seed=seed,
                      scale=math.sqrt(4.0 / 13.0), blk_pad=16)


def _cells():
    pos22, box22 = W.amorphous_positions(22, 0.0074, 3.0, seed=31)
    return {
        "si64_13": W.diamond_workload("si64_13f", (2, 2, 2), seed=3, nfun=13,
                                      R=(12.0, 14.0, 10.0)),
        "am22_13": _w13("am22_13f", pos22, box22, 31),
        "one13": _w13("one13f", np.array([[1.0, 2.0, 3.0]]), np.array([7.0, 7.5, 8.0]), 41),
    }


NAMES = ["si64_13", "si64_13b", "am22_13", "one13"]


@pytest.fixture(scope="module")
def cells(gpu):
    """The cells in spatial-cell row order; si64_13b: the diamond cell with
    its rows in groups of four bonded atoms (the benchmark's layout)."""
    from paper_2002_07704_amd.system import LNVSystem
    out = {}
    ws = _cells()
    ws["si64_13b"] = ws["si64_13"]
    for name, w in ws.items():
        order = "bonds" if name.endswith("b") else None
        s = LNVSystem(w, metric="hotelling", n_hotelling=16, reorder=order)
        out[name] = (s, ost.System(w), Layout(s))
    yield out
    L_.call("lnv_set_f32_accumulation", ACC_F32)


def _tol(s, acc):
    """3 sqrt(k) u relative: the rounding bound of one FP32-accumulated entry
    over a contraction of k = 4 x the longest row of pat(S.L) terms, with u
    the operands' unit roundoff (2^-24 in FP32; 2^-22 for the FP16 hi/lo
    split's 11 + 11 significant bits)."""
    rp = s.pSL.row_ptr.cpu().numpy()
    k = 4 * int(np.diff(rp).max())
    u = 2.0 ** -22 if acc == ACC_F16X3 else 2.0 ** -24
    return 3.0 * math.sqrt(k) * u


def _seeded_L(s, ref, lay, seed):
    n = lay.n_orb
    Ld = _rand_sym(n, ref.maskL, seed) + 0.2 * np.eye(n) * ref.maskL
    s.L.val.copy_(lay.to_blocks(Ld, s.pL))
    return Ld


@pytest.mark.parametrize("name", NAMES)
def test_tile_shapes_offered(cells, name):
    s, _, _ = cells[name]
    assert s.tile_shapes() == tuple(SHAPES)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("name", NAMES)
def test_tile_eval_matches_oracle(cells, name, shape):
    s, ref, lay = cells[name]
    w = s.w
    Ld = _seeded_L(s, ref, lay, 5)
    s.set_cluster((4, 1))
    s.eval()
    torch.cuda.synchronize()
    EN4, G4 = s.EN.clone(), s.G.val.clone()
    s.set_cluster(shape)
    assert s.pS.cl[0] == 16 and s.pS.tile4 == 1 and s.pLS.tile4 == 1 and s.pX.tile4 == 1
    assert s.pLu.tile4 == 1 and s.pZu.tile4 == 1     # halves keep whole atom tiles
    print(f"{name} {shape}: {s.n} atoms, {s.n_rows} rows, pieces of L {s.pL.struct.n_cl_items}",
          flush=True)
    s.eval()
    torch.cuda.synchronize()
    E, N = (float(x) for x in s.EN.cpu())
    Er, Nr, Gr, Fr = olnv.evaluate(Ld, ref.S, ref.H, ref.maskL)
    print(f"{name} {shape}: |dE|/atom {abs(E - Er) / w.n:.2e} |dN|/atom {abs(N - Nr) / w.n:.2e}",
          flush=True)
    assert abs(E - Er) / w.n <= 1e-10, (E, Er)
    assert abs(N - Nr) / w.n <= 1e-10, (N, Nr)
    G = lay.to_dense(s.G.val, s.pL)          # padding exactly zero
    F = lay.to_dense(s.F.val, s.pL)
    assert np.abs(G - Gr).max() <= 1e-12 * np.abs(Gr).max()
    assert np.abs(F - Fr).max() <= 1e-12 * np.abs(Fr).max()
    # the same evaluation on the 4x4 kernels (other summation order)
    assert torch.allclose(s.EN, EN4, rtol=1e-13, atol=0.0)
    assert (s.G.val - G4).abs().max() <= 1e-13 * G4.abs().max()
    s.set_cluster((4, 1))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("name", ["si64_13b", "am22_13", "one13"])
def test_tile_half_symmetric_operand(cells, name, shape):
    """transB = 2: the symmetric S.L.S given by the blocks of its half only
    (Z's half pattern), read as stored inside the half and transposed outside
    it.  S.L times it on L's pattern against the oracle's P_L(S L S L S) and
    against the product with the full S.L.S; outside the atom tiles the
    half operand is refused."""
    from paper_2002_07704_amd.system import Matrix, multiply
    s, ref, lay = cells[name]
    Ld = _seeded_L(s, ref, lay, 7)
    s.set_cluster(shape)
    s.eval()                                  # S.L, and S.L.S in full and on its half
    torch.cuda.synchronize()
    Vh, Vf = Matrix(s.pL), Matrix(s.pL)
    multiply(1.0, s.SL, s.Zu, 2, 0.0, Vh)
    multiply(1.0, s.SL, s.Z, 0, 0.0, Vf)
    torch.cuda.synchronize()
    Sd = ref.S
    Vr = (Sd @ Ld @ Sd @ Ld @ Sd) * ref.maskL
    V = lay.to_dense(Vh.val, s.pL)
    err = np.abs(V - Vr).max() / np.abs(Vr).max()
    print(f"{name} {shape}: half operand vs oracle {err:.2e}", flush=True)
    assert err <= 1e-12
    assert (Vh.val - Vf.val).abs().max() <= 1e-13 * Vf.val.abs().max()
    s.set_cluster((4, 1))
    with pytest.raises(L_.LnvError) as e:
        multiply(1.0, s.SL, s.Zu, 2, 0.0, Vh)
    assert e.value.status == L_.EUNSUPPORTED


@pytest.mark.parametrize("name", ["si64_13", "si64_13b"])
def test_tile_cg_trajectory(cells, name):
    s, ref, lay = cells[name]
    w = s.w
    steps = 6
    T = olnv.hotelling(ref.S, ref.maskL, 16)
    _, hist = olnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, steps, T=T)
    s.set_cluster((16, 4))
    s.cg_init()
    for k in range(steps):
        s.cg_step()
        sc = s.scalars_host()
        h = hist[k]
        print(f"tiles k={k} E/atom gpu {sc['E'] / w.n:.13f} oracle {h['E'] / w.n:.13f}",
              flush=True)
        assert abs(sc["E"] - h["E"]) / w.n <= 1e-10, k
        assert abs(sc["N"] - h["N"]) <= 1e-9 * max(1.0, w.n_elec / 64), k
        assert abs(sc["ALPHA"] - h["alpha"]) <= 1e-8 * abs(h["alpha"]), k
        assert abs(sc["DELTA"] - h["delta"]) <= 1e-8 * max(abs(h["delta"]), 1e-6), k
        assert int(sc["STATUS"]) & 3 == 0
    torch.cuda.synchronize()
    lay.to_dense(s.L.val, s.pL)
    s.set_cluster((4, 1))


@pytest.mark.parametrize("acc", [ACC_F32, ACC_F16X3], ids=["fp32", "fp16x3"])
def test_tile_mixed_cg_tracks_fp64(cells, acc):
    """CG iterations whose evaluation runs on the FP32 (or FP16 hi/lo) atom
    tiles, bonded rows, against the same iterations in FP64 from the same
    start: every iteration's energy within 1e-6 Ha/atom of the FP64
    trajectory, no failed line search."""
    s, ref, lay = cells["si64_13b"]
    w = s.w
    steps = 6
    s.set_cluster((16, 4))
    hist = []
    try:
        for mixed in (False, True):
            L_.call("lnv_set_f32_accumulation", acc)
            s.opts.mixed = mixed
            s.cg_init()
            run = []
            for _ in range(steps):
                s.cg_step()
                run.append(s.scalars_host())
            hist.append(run)
    finally:
        s.opts.mixed = False
        L_.call("lnv_set_f32_accumulation", ACC_F32)
        s.set_cluster((4, 1))
    for k, (a, b) in enumerate(zip(*hist)):
        print(f"acc {acc} k={k} E/atom fp64 {a['E'] / w.n:.12f} mixed {b['E'] / w.n:.12f}",
              flush=True)
        assert abs(a["E"] - b["E"]) / w.n <= 1e-6, k
        assert int(b["STATUS"]) & 3 == 0, k


def test_tile_adjoint(cells):
    s, ref, lay = cells["si64_13"]
    s.set_cluster((16, 4))
    Ld = _seeded_L(s, ref, lay, 9)
    dS = torch.empty_like(s.S.val)
    dH = torch.empty_like(s.H.val)
    s.adjoint(s.L.val, s.S.val, s.H.val, dS=dS, dH=dH)
    torch.cuda.synchronize()
    gS = olnv.grad_S(Ld, ref.S, ref.H, ref.maskS)
    gH = olnv.grad_H(Ld, ref.S, ref.maskH)
    assert np.abs(lay.to_dense(dS, s.pS) - gS).max() <= 1e-12 * np.abs(gS).max()
    assert np.abs(lay.to_dense(dH, s.pH) - gH).max() <= 1e-12 * np.abs(gH).max()
    s.set_cluster((4, 1))


@pytest.mark.parametrize("acc", [ACC_F32, ACC_F64, ACC_F16X3])
@pytest.mark.parametrize("name", ["si64_13", "am22_13"])
def test_tile_mixed_modes(cells, gpu, name, acc):
    s, ref, lay = cells[name]
    w = s.w
    Ld = _seeded_L(s, ref, lay, 7)
    Er, Nr, Gr, Fr = olnv.evaluate(Ld, ref.S, ref.H, ref.maskL)
    s.set_cluster((16, 4))
    L_.call("lnv_set_f32_accumulation", acc)
    try:
        s.eval_mixed()
        torch.cuda.synchronize()
    finally:
        L_.call("lnv_set_f32_accumulation", ACC_F32)
    E, N = (float(x) for x in s.EN.cpu())
    G = lay.to_dense(s.G.val, s.pL)
    F = lay.to_dense(s.F.val, s.pL)
    eG = np.abs(G - Gr).max() / np.abs(Gr).max()
    eF = np.abs(F - Fr).max() / np.abs(Fr).max()
    print(f"{name} acc={acc}: |dE|/atom {abs(E - Er) / w.n:.2e} |dN|/atom "
          f"{abs(N - Nr) / w.n:.2e} dG {eG:.2e} dF {eF:.2e}", flush=True)
    tol = _tol(s, acc)
    assert abs(E - Er) / w.n <= 1e-6
    assert abs(N - Nr) <= tol * abs(Nr)
    assert eG <= tol and eF <= tol
    s.set_cluster((4, 1))


@pytest.mark.parametrize("order", ["cell", "bonds"])
def test_tile_eval_at_scale(gpu, order):
    """8192 atoms with 13 functions (32768 rows): tile evaluations against the
    4x4 path's FP64 evaluation at the CG start, with the rows in spatial cells
    and in groups of four bonded atoms (the benchmark's layout)."""
    from paper_2002_07704_amd.system import LNVSystem
    w = W.diamond_workload("si8192_13f", (16, 16, 4), seed=3, nfun=13, R=(12.0, 14.0, 10.0))
    s = LNVSystem(w, metric="hotelling", reorder=order)
    s.cg_init()
    s.eval()
    torch.cuda.synchronize()
    E4, N4 = (float(x) for x in s.EN.cpu())
    G4 = s.G.val.clone()
    for shape in SHAPES:
        s.set_cluster(shape)
        s.eval()
        torch.cuda.synchronize()
        E, N = (float(x) for x in s.EN.cpu())
        dG = float((s.G.val - G4).abs().max() / G4.abs().max())
        print(f"si8192_13f {shape}: E/atom {E / w.n:.14f} (4x4 {E4 / w.n:.14f}) dG {dG:.1e}",
              flush=True)
        assert abs(E - E4) / w.n <= 1e-12 and abs(N - N4) / w.n <= 1e-12
        assert dG <= 1e-12
    s.mixed_setup()
    for acc in (ACC_F32, ACC_F16X3):
        L_.call("lnv_set_f32_accumulation", acc)
        try:
            s.eval_mixed()
            torch.cuda.synchronize()
        finally:
            L_.call("lnv_set_f32_accumulation", ACC_F32)
        E, N = (float(x) for x in s.EN.cpu())
        dG = float((s.G.val - G4).abs().max() / G4.abs().max())
        print(f"si8192_13f mixed acc={acc}: |dE|/atom {abs(E - E4) / w.n:.2e} "
              f"|dN|/atom {abs(N - N4) / w.n:.2e} dG {dG:.1e}", flush=True)
        tol = _tol(s, acc)
        assert abs(E - E4) / w.n <= 1e-6 and abs(N - N4) <= tol * abs(N4)
        assert dG <= tol


# ------------------------------------------------------------------ lean systems
@pytest.mark.parametrize("name", ["si64_13b", "si64_4x4"])
def test_lean_evaluation_reads_transposes(cells, name):
    """A lean system (no stored L.S and X^T: the products read S.L and X
    transposed; FP32 intermediates in the FP64 ones' memory) against the full
    system at the same L: FP64 evaluation to rounding, and the mixed-precision
    evaluations (FP32 MFMA, FP16 hi/lo on the atom tiles) identical to the
    full system's own.  The 4-function cell runs the transposed reads on the
    row kernel, the 13-function cell on the atom tiles."""
    from paper_2002_07704_amd.system import LNVSystem
    if name in cells:
        full, _, _ = cells[name]
        w = full.w
        kw = dict(reorder="bonds")
    else:
        w = W.get(name)
        full = LNVSystem(w, metric="hotelling", n_hotelling=16)
        kw = {}
    lean = LNVSystem(w, metric="hotelling", n_hotelling=16, lean=True, cluster=None, **kw)
    assert lean.LS is None and lean.XT is None and lean.pXT is None
    shape = (16, 4) if full.tile_shapes() else (4, 1)
    for s in (full, lean):
        s.set_cluster(shape)
    full.cg_init()
    lean.L.val.copy_(full.L.val)
    with pytest.raises(RuntimeError):
        lean.cg_init()
    res = {}
    for s in (full, lean):
        s.eval()
        torch.cuda.synchronize()
        res[id(s)] = [(s.EN.clone(), s.G.val.clone(), s.F.val.clone())]
        s.mixed_setup()
        for acc in ((ACC_F32, ACC_F16X3) if shape[0] == 16 else (ACC_F32,)):
            L_.call("lnv_set_f32_accumulation", acc)
            s.eval_mixed()
            torch.cuda.synchronize()
            res[id(s)].append((s.EN.clone(), s.G.val.clone(), s.F.val.clone()))
        L_.call("lnv_set_f32_accumulation", ACC_F32)
        s.eval()          # FP64 again after the FP32 ones (shared memory in the lean system)
        torch.cuda.synchronize()
        res[id(s)].append((s.EN.clone(), s.G.val.clone(), s.F.val.clone()))
    a, b = res[id(full)], res[id(lean)]
    for k, ((E1, G1, F1), (E2, G2, F2)) in enumerate(zip(a, b)):
        tol = 1e-12 if k in (0, len(a) - 1) else 1e-5
        print(f"{name} {k}: dE/atom {abs(float(E1[0] - E2[0])) / w.n:.2e} "
              f"dG {float((G1 - G2).abs().max() / G1.abs().max()):.2e}", flush=True)
        assert abs(float(E1[0] - E2[0])) / w.n <= tol * 1e2, k
        assert abs(float(E1[1] - E2[1])) <= tol * float(E1[1]), k
        assert (G1 - G2).abs().max() <= tol * G1.abs().max(), k
        assert (F1 - F2).abs().max() <= tol * F1.abs().max(), k
    assert torch.equal(b[0][0], b[-1][0])
    for s in (full, lean):
        s.set_cluster((4, 1))
