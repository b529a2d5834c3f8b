"""The bonded row order (atoms in groups of four bonded neighbours, the
layout bench.py times) against the oracle and against the atoms' own order.

A row order is a relabelling: patterns, S and H are the atom-order ones up to
the permutation (S, H bit for bit: the generator keys every entry by its atom
pair), and every scalar of the evaluation and the CG is the same up to the
summation order of the traces.
"""
import json
import os

import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "si4096_4x4.json")


def _orb_perm(s):
    """Orbital index in s's rows of each orbital in atom order (4-function atoms)."""
    atom_of = s.atom_of.cpu().numpy()
    inv = np.empty_like(atom_of)
    inv[atom_of] = np.arange(len(atom_of))
    return (inv[:, None] * 4 + np.arange(4)[None, :]).reshape(-1)


def _dense_atoms(s, M, pat):
    """Dense matrix of M (on pattern pat, in s's rows) in the atoms' own order."""
    rp, col = pat.host()
    D = ost.blocks_to_dense(M.val.cpu().numpy(), rp, col, s.w.nfun)
    if s.atom_of is None:
        return D
    o = _orb_perm(s)
    return D[np.ix_(o, o)]


@pytest.fixture(scope="module")
def si64_pair(gpu):
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get("si64_4x4")
    return (LNVSystem(w, metric=None, reorder="bonds"), LNVSystem(w, metric=None),
            ost.System(w))


def test_bonded_layout_patterns_and_matrices(si64_pair):
    """Range patterns equal the oracle's under the permutation (bit-exact), and
    S, H equal the atom-order system's bit for bit."""
    sb, sa, ref = si64_pair
    w = sb.w
    assert sb.atom_of is not None and not sb.split
    assert np.array_equal(sb.atom_of.cpu().numpy(), w.groups)
    for pat, M in ((sb.pS, ref.maskS), (sb.pH, ref.maskH), (sb.pL, ref.maskL)):
        rp, col = pat.host()
        A = np.zeros((w.n, w.n), dtype=bool)
        for r in range(w.n):
            A[r, col[rp[r]:rp[r + 1]]] = True
        g = np.asarray(w.groups)
        atom_mask = np.zeros_like(A)
        atom_mask[np.ix_(g, g)] = A
        assert np.array_equal(atom_mask, M[::4, ::4].astype(bool))
    assert np.array_equal(_dense_atoms(sb, sb.S, sb.pS), _dense_atoms(sa, sa.S, sa.pS))
    assert np.array_equal(_dense_atoms(sb, sb.H, sb.pH), _dense_atoms(sa, sa.H, sa.pH))


def test_bonded_layout_eval_matches_oracle(si64_pair):
    sb, _, ref = si64_pair
    w = sb.w
    sb.cg_init()
    sb.eval()
    torch.cuda.synchronize()
    L = _dense_atoms(sb, sb.L, sb.pL)
    E, N, G, F = olnv.evaluate(L, ref.S, ref.H, ref.maskL)
    Eg, Ng = (float(x) for x in sb.EN.cpu())
    assert abs(Eg - E) / w.n <= 1e-10
    assert abs(Ng - N) <= 1e-9
    Gg = _dense_atoms(sb, sb.G, sb.pL)
    Fg = _dense_atoms(sb, sb.F, sb.pL)
    assert np.abs(Gg - G).max() <= 1e-12 * np.abs(G).max()
    assert np.abs(Fg - F).max() <= 1e-12 * np.abs(F).max()


def test_bonded_layout_cg_trajectory(si64_pair):
    """20 identity-metric CG iterations in the bonded layout: every iteration's
    scalars against the oracle's, and the final L against the oracle's L."""
    sb, _, ref = si64_pair
    w = sb.w
    Lo, hist = olnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, 20)
    sb.cg_init()
    for k in range(20):
        sb.cg_step()
        sc = sb.scalars_host()
        h = hist[k]
        assert abs(sc["E"] - h["E"]) / w.n <= 1e-10, k
        assert abs(sc["N"] - h["N"]) <= 1e-9, k
        assert abs(sc["MU"] - h["mu"]) <= 1e-9 * max(1.0, abs(h["mu"])), k
        assert abs(sc["BETA"] - h["beta"]) <= 1e-7, k
        assert abs(sc["ALPHA"] - h["alpha"]) <= 1e-8 * abs(h["alpha"]), k
        assert int(sc["STATUS"]) == 0
    assert np.abs(_dense_atoms(sb, sb.L, sb.pL) - Lo).max() <= 1e-9


def test_bonded_layout_at_scale_matches_stored_oracle(gpu):
    """4096 atoms in the benchmark's layout: E, N and the norms of G, F at
    L0 = lambda*I against the stored oracle values (all invariant under the
    row permutation), and fewer 64-lane work pieces than the atom order."""
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get("si4096_4x4")
    gold = json.load(open(GOLD))
    s = LNVSystem(w, metric=None, reorder="bonds")
    s.cg_init()
    s.eval()
    torch.cuda.synchronize()
    assert abs(s.scalar("LAMBDA") - gold["lambda"]) <= 1e-12 * gold["lambda"]
    E, N = (float(x) for x in s.EN.cpu())
    print(f"E/atom gpu {E / w.n:.15f} oracle {gold['E0'] / w.n:.15f}", flush=True)
    assert abs(E - gold["E0"]) / w.n <= 1e-10
    assert abs(N - gold["N0"]) <= 1e-9 * w.n_elec
    g = float(torch.linalg.vector_norm(s.G.val).item())
    f = float(torch.linalg.vector_norm(s.F.val).item())
    assert abs(g - gold["G0_fro"]) <= 1e-11 * gold["G0_fro"]
    assert abs(f - gold["F0_fro"]) <= 1e-11 * gold["F0_fro"]
    assert 0 < s.pL.struct.n_cl_items < 4 * (w.n // 4)


def test_bonded_layout_cg_from_purified_start_at_scale(gpu):
    """The benchmark's run in both layouts: canonical purification then 6 CG
    iterations; both descend with status 0, N exact after the first correction, and the energies agree
    to 1e-9 Ha/atom at every iteration."""
    from paper_2002_07704_amd.pm import pm_initial_L
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get("si4096_4x4")
    runs = {}
    for order in ("bonds", False):
        s = LNVSystem(w, reorder=order)
        pm_initial_L(s, 60)
        s.cg_restart()
        E = []
        for k in range(6):
            s.cg_step()
            sc = s.scalars_host()
            E.append(sc["E"])
            assert int(sc["STATUS"]) == 0, (order, k, sc["STATUS"])
            if k > 0:     # N of the L the step starts from: corrected from step 1 on
                assert abs(sc["N"] - w.n_elec) <= 1e-9 * w.n_elec, (order, k)
        runs[order] = E
        print(order, [round(e / w.n, 12) for e in E], flush=True)
        del s
        torch.cuda.empty_cache()
    Eb, Ea = runs["bonds"], runs[False]
    assert all(b < a for a, b in zip(Eb, Eb[1:]))
    assert max(abs(a - b) for a, b in zip(Ea, Eb)) / w.n <= 1e-9


def atom_order(rp, col, blocks, atom_of):
    """A block pattern and its 4x4 blocks with rows in the atoms' own order
    (one row per atom, row r holding atom atom_of[r])."""
    n = len(rp) - 1
    lens = np.diff(rp)
    inv = np.empty(n, dtype=np.int64)
    inv[atom_of] = np.arange(n)
    rp2 = np.zeros(n + 1, dtype=np.int64)
    rp2[1:] = np.cumsum(lens[inv])
    col2 = np.empty_like(col)
    out = np.empty_like(blocks)
    for a in range(n):
        r = inv[a]
        c = atom_of[col[rp[r]:rp[r + 1]]]
        o = np.argsort(c, kind="stable")
        col2[rp2[a]:rp2[a + 1]] = c[o]
        out[rp2[a]:rp2[a + 1]] = blocks[rp[r]:rp[r + 1]][o]
    return rp2.astype(rp.dtype), col2, out


def test_bonded_layout_sampled_rows_at_benchmark_point(gpu):
    """The benchmark's configuration at full size: 4096 atoms, bonded rows,
    Hotelling metric, L after the purified start and two CG iterations.  Rows
    of G and F at that L, mapped back to atom order, against the row-wise
    oracle fed the same L (rows of both ends and the middle of the cell)."""
    from oracle import rows as orows
    from paper_2002_07704_amd.pm import pm_initial_L
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get("si4096_4x4")
    s = LNVSystem(w, reorder="bonds")
    pm_initial_L(s, 60)
    s.cg_restart()
    s.cg_step()
    s.cg_step()
    s.eval()
    torch.cuda.synchronize()
    rp, col = s.pL.host()
    atom_of = s.atom_of.cpu().numpy()
    rpa, cola, La = atom_order(rp, col, s.L.val.cpu().numpy(), atom_of)
    _, _, Ga = atom_order(rp, col, s.G.val.cpu().numpy(), atom_of)
    _, _, Fa = atom_order(rp, col, s.F.val.cpu().numpy(), atom_of)
    pS = ost.neighbours(w.pos, w.box, w.R_S)
    pH = ost.neighbours(w.pos, w.box, w.R_H)
    Sb = ost.synth_blocks(w, "S", *pS)
    Hb = ost.synth_blocks(w, "H", *pH)
    ro = orows.RowOracle(w, Sb, Hb, La, pS, pH, (rpa, cola))
    gmax, fmax = np.abs(Ga).max(), np.abs(Fa).max()
    for a in (0, 1, 777, 2048, 3000, 4095):
        _, _, Gi, Fi, cols = ro.row(a)
        assert np.array_equal(cols, cola[rpa[a]:rpa[a + 1]])
        eg = np.abs(Ga[rpa[a]:rpa[a + 1]] - Gi).max()
        ef = np.abs(Fa[rpa[a]:rpa[a + 1]] - Fi).max()
        print(f"atom {a}: |dG| {eg:.1e} (max {gmax:.1e}) |dF| {ef:.1e} (max {fmax:.1e})", flush=True)
        assert eg <= 1e-12 * gmax, a
        assert ef <= 1e-12 * fmax, a
