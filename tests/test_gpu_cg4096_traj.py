"""The benchmark's minimisation on the 4096-atom cell against the oracle:
Hotelling metric T (16 steps), canonical-purification start (60 steps),
then consecutive CG iterations, as bench.py times them (rows in bonded
groups).  The dense oracle needs about 20 minutes per iteration at 16384
orbitals, so its trajectory -- every iteration's E, N, mu, beta, alpha and
delta, and G and F rows of four atoms at three iterations -- is stored in
tests/golden/si4096_4x4_cg.json and si4096_4x4_cg_rows.npz, written by
tests/golden/make_golden.py (cgtraj) from the oracle alone."""
import json
import os

import numpy as np
import pytest
import torch

import lnv_workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
GOLD = os.path.join(HERE, "si4096_4x4_cg.json")
ROWS = os.path.join(HERE, "si4096_4x4_cg_rows.npz")


def _row_blocks(s, V, atom, cols):
    """Blocks (atom, j) for the oracle's column atoms j from GPU values V on
    L's pattern, rows in the system's order."""
    atom_of = s.atom_of.cpu().numpy()
    row_of = np.empty_like(atom_of)
    row_of[atom_of] = np.arange(len(atom_of))
    rp, col = s.pL.host()
    r = row_of[atom]
    pos = {int(c): p for p, c in enumerate(col[rp[r]:rp[r + 1]], start=int(rp[r]))}
    assert sorted(int(atom_of[c]) for c in pos) == sorted(int(j) for j in cols)
    return np.stack([V[pos[int(row_of[j])]] for j in cols])


def test_cg_trajectory_si4096_matches_stored_oracle(gpu):
    from paper_2002_07704_amd.pm import pm_initial_L
    from paper_2002_07704_amd.system import LNVSystem
    gold = json.load(open(GOLD))
    rows = np.load(ROWS)
    w = W.get("si4096_4x4")
    s = LNVSystem(w, reorder="bonds", metric="hotelling", n_hotelling=16)
    hist, _ = pm_initial_L(s, 60)
    assert len(hist) == gold["pm_steps"]
    s.cg_restart()
    for h in gold["cg"]:
        k = h["k"]
        s.cg_step()
        sc = s.scalars_host()
        print(f"k={k} E/atom gpu {sc['E'] / w.n:.15f} oracle {h['E'] / w.n:.15f} "
              f"alpha {sc['ALPHA']:.9e} ({h['alpha']:.9e}) delta {sc['DELTA']:.3e} "
              f"({h['delta']:.3e})", flush=True)
        assert abs(sc["E"] - h["E"]) / w.n <= 1e-10, k
        assert abs(sc["N"] - h["N"]) <= 1e-9 * w.n_elec / 64, k
        assert abs(sc["MU"] - h["mu"]) <= 1e-9 * max(1.0, abs(h["mu"])), k
        assert abs(sc["BETA"] - h["beta"]) <= 1e-7, k
        assert abs(sc["ALPHA"] - h["alpha"]) <= 1e-8 * abs(h["alpha"]), k
        assert abs(sc["DELTA"] - h["delta"]) <= 1e-8 * max(abs(h["delta"]), 1e-6), k
        assert int(sc["STATUS"]) == 0, k
        if k in gold["row_iters"]:
            G = s.G.val.cpu().numpy()
            F = s.F.val.cpu().numpy()
            for a in gold["row_atoms"]:
                cols = rows[f"cols_{a}"]
                Go, Fo = rows[f"G_{k}_{a}"], rows[f"F_{k}_{a}"]
                Gg, Fg = _row_blocks(s, G, a, cols), _row_blocks(s, F, a, cols)
                eg = np.abs(Gg - Go).max() / np.abs(Go).max()
                ef = np.abs(Fg - Fo).max() / np.abs(Fo).max()
                print(f"  rows of atom {a}: G {eg:.2e}, F {ef:.2e} (relative to the row's largest)",
                      flush=True)
                assert eg <= 1e-10 and ef <= 1e-10, (k, a)
