"""Degenerate and ragged systems on the GPU path against the oracle.

* one atom in a small periodic cell (every pattern is the single diagonal
  block, summed over many periodic images; clusters of 4 rows hold one row);
* five atoms (the last 4-row cluster holds one row);
* an L range shorter than every interatomic distance (L, and with it every
  product restricted to L, block-diagonal; the natural products are not);
* two 13-function atoms and one 4-function atom (split rows of 4, 4, 4, 1
  functions: padded rows with one present function).

Each: E, N, G, F at the CG start and every scalar of 4 Hotelling-metric CG
iterations against the oracle, to the bars of the parity tests (|dE|, |dN|
<= 1e-10 per atom, matrices 1e-12 relative).
"""
import math

import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost

pytestmark = pytest.mark.gpu


def _workload(name, pos, box, nfun, n_elec, R=(12.0, 14.0, 16.0), seed=21):
    pos = np.mod(np.asarray(pos, dtype=np.float64), box)
    nf = np.asarray(nfun, dtype=np.int32)
    return W.Workload(name=name, pos=pos, box=np.asarray(box, dtype=np.float64), nfun=nf,
                      species=np.zeros(len(nf), dtype=np.int8), R_S=R[0], R_H=R[1], R_L=R[2],
                      n_elec=int(n_elec), seed=seed, scale=math.sqrt(4.0 / int(nf.max())),
                      blk_pad=4 if int(nf.max()) == 4 else 16)


def _cases():
    rng = np.random.default_rng(5)
    box5 = np.array([9.0, 9.5, 10.0])
    return {
        "one_atom": _workload("one_atom", [[1.0, 2.0, 3.0]], np.array([7.0, 7.5, 8.0]), [4], 2),
        "five_atoms": _workload("five_atoms", rng.uniform(0, 1, (5, 3)) * box5, box5,
                                [4] * 5, 10, R=(6.0, 7.0, 8.0)),
        "diagonal_L": _workload("diagonal_L", [[0.0, 0.0, 0.0], [4.0, 0.5, 0.0],
                                                [0.5, 4.5, 0.5], [4.5, 4.0, 4.0]],
                                np.array([9.0, 9.0, 9.0]), [4] * 4, 8, R=(6.0, 7.0, 2.0)),
        "split_13_13_4": _workload("split_13_13_4", [[0.0, 0.0, 0.0], [3.5, 0.0, 0.0],
                                                     [0.0, 3.5, 1.0]],
                                   np.array([8.0, 8.0, 8.0]), [13, 13, 4], 8,
                                   R=(6.0, 7.0, 8.0)),
    }


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_systems_match_oracle(gpu, name):
    from paper_2002_07704_amd.system import LNVSystem
    w = CASES[name]
    sysg = LNVSystem(w, metric="hotelling", n_hotelling=16)
    ref = ost.System(w)
    if name == "diagonal_L":
        assert sysg.pL.nnzb == w.n and sysg.pX.nnzb > w.n
    T = olnv.hotelling(ref.S, ref.maskL, 16)
    sysg.cg_init()
    sysg.eval()
    torch.cuda.synchronize()
    L0, _ = olnv.initial_L(ref.S, ref.maskL, w.n_elec, T)
    lay = _layout(sysg)
    assert np.abs(lay(sysg.L.val, sysg.pL) - L0).max() <= 1e-12 * max(1.0, np.abs(L0).max())
    Er, Nr, Gr, Fr = olnv.evaluate(L0, ref.S, ref.H, ref.maskL)
    E, N = (float(x) for x in sysg.EN.cpu())
    assert abs(E - Er) / w.n <= 1e-10 and abs(N - Nr) / w.n <= 1e-10, (E, Er, N, Nr)
    for M, R in ((sysg.G, Gr), (sysg.F, Fr)):
        assert np.abs(lay(M.val, sysg.pL) - R).max() <= 1e-12 * max(1.0, np.abs(R).max())
    _, hist = olnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, 4, T=T)
    sysg.cg_init()
    for k in range(4):
        sysg.cg_step()
        sc = sysg.scalars_host()
        h = hist[k]
        assert abs(sc["E"] - h["E"]) / w.n <= 1e-10, (k, sc["E"], h["E"])
        assert abs(sc["N"] - h["N"]) <= 1e-9 * max(1.0, w.n_elec), k
        assert abs(sc["ALPHA"] - h["alpha"]) <= 1e-8 * max(abs(h["alpha"]), 1e-12), k


def _layout(sysg):
    """Stored blocks -> dense orbital matrix (the split layout when present)."""
    w = sysg.w
    nf = np.asarray(w.nfun)
    off = ost.offsets(nf)
    if sysg.atom_of is None:
        def dense(V, pat):
            rp, col = pat.host()
            return ost.blocks_to_dense(V.cpu().numpy(), rp, col, nf)
        return dense
    atom_of = sysg.atom_of.cpu().numpy()
    off_of = sysg.off_of.cpu().numpy()
    base = off[atom_of] + off_of
    nv = np.minimum(4, nf[atom_of] - off_of)

    def dense(V, pat):
        rp, col = pat.host()
        V = V.detach().cpu().double().numpy()
        A = np.zeros((int(off[-1]), int(off[-1])))
        for i in range(len(rp) - 1):
            for p in range(rp[i], rp[i + 1]):
                j = col[p]
                A[base[i]:base[i] + nv[i], base[j]:base[j] + nv[j]] = V[p, :nv[i], :nv[j]]
        return A
    return dense
