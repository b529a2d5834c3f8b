"""The cells with atoms of several stored rows at scale, on the GPU, in the
row layout and launch configuration bench.py uses for them:

* the 78646-orbital amorphous Si/O/H cell (8192 atoms, 13/9/4 functions;
  rows in spatial cells, 4-row clusters);
* the 425984-orbital 13-function diamond cell (32768 atoms, 131072 rows;
  rows in bonded groups, a lean system -- no stored L.S and X^T -- on the
  FP64 atom tiles (16, 4), as benchmarked).

The dense oracle does not fit at these sizes; the row-wise oracle's G and F
rows of sampled atoms (every species included) at a seeded L are stored in
tests/golden/<workload>_rows.npz, written by
`tests/golden/make_golden.py rows <workload>` from the oracle only.  The
seeded L = 0.1 (w M + 2I) on L's range is generated on each side from the
same counter definition (the synthetic overlap generator, master seed + 1000,
range R_L, decay 3 bohr).  Tolerance: 1e-12 of the row's largest entry, as
for the 4-function cells.
"""
import os

import numpy as np
import pytest
import torch

import lnv_workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "{}_rows.npz")


@pytest.mark.parametrize("name", ["siOH8192_mixed", "si32768_13f"])
def test_split_eval_at_scale_sampled_rows(gpu, name):
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get(name)
    gold = np.load(GOLD.format(name))
    if name == "si32768_13f":
        s = LNVSystem(w, metric=None, reorder="bonds", lean=True, cluster=None)
        s.set_cluster((16, 4))
        print(f"{name}: {s.n_rows} rows, grid {s.ix_cells.g}, device memory "
              f"{torch.cuda.memory_allocated() / 2**30:.1f} GiB", flush=True)
    else:
        s = LNVSystem(w, metric=None)
    Lm = s.synth_values(0, s.pL, w.R_L, 3.0, w.seed + 1000)
    s.L.val.copy_(0.1 * Lm.val)
    del Lm
    s.eval()
    torch.cuda.synchronize()
    G = s.G.val.cpu().numpy()
    F = s.F.val.cpu().numpy()
    rp, col = s.pL.host()
    atom_of = s.atom_of.cpu().numpy()
    off_of = s.off_of.cpu().numpy()
    nfun = np.asarray(w.nfun)
    for i in gold["atoms"]:
        i = int(i)
        cols = gold[f"cols_{i}"]
        where = {int(j): t for t, j in enumerate(cols)}
        Gr, Fr = gold[f"G_{i}"], gold[f"F_{i}"]
        Gg, Fg = np.zeros_like(Gr), np.zeros_like(Fr)
        seen = set()
        for I in np.nonzero(atom_of == i)[0]:
            oi = off_of[I]
            ni = min(4, nfun[i] - oi)
            for p in range(rp[I], rp[I + 1]):
                J = col[p]
                j, oj = int(atom_of[J]), off_of[J]
                nj = min(4, nfun[j] - oj)
                t = where[j]
                seen.add(j)
                Gg[t, oi:oi + ni, oj:oj + nj] = G[p, :ni, :nj]
                Fg[t, oi:oi + ni, oj:oj + nj] = F[p, :ni, :nj]
        assert seen == set(where), i
        eg = np.abs(Gg - Gr).max() / np.abs(Gr).max()
        ef = np.abs(Fg - Fr).max() / np.abs(Fr).max()
        print(f"atom {i} (nfun {nfun[i]}): |dG|/max {eg:.1e} |dF|/max {ef:.1e}", flush=True)
        assert eg <= 1e-12 and ef <= 1e-12
    del s
    torch.cuda.empty_cache()
