"""The cut of X = H.L.S and Z = S.L.S to R_S + 2 R_L (system.xz_range): every
entry that the L-projected products and the assembly read lies inside it.

X and Z are read by P_L(S.L . X), P_L(S.L . X^T), P_L(S.L . Z) and, on L's own
pattern, by the traces and the assembly.  Entry (k, j) of the right operand
is read when some i has (i, k) in pat(S.L) and (i, j) in pat(L), i.e. the
needed set is pat(L.S . L) (for X^T: its transpose).  Checked with the
oracle's boolean pattern products on 512-atom periodic cells (nearest-image
distances), one with a long H range so that the cut does remove
natural-range entries, one with the 13-function workload's ranges.
"""
import pytest

import lnv_workloads as W
from oracle import structure as ost
from paper_2002_07704_amd.system import xz_range


def _pat(w, R):
    return ost.pattern_matrix(*ost.neighbours(w.pos, w.box, R), w.n)


@pytest.mark.parametrize("cubes, R, cuts", [((4, 4, 4), (8.0, 14.0, 5.0), True),
                                            ((4, 4, 4), (12.0, 14.0, 10.0), False)])
def test_needed_entries_lie_within_the_cut(cubes, R, cuts):
    w = W.diamond_workload("xz", cubes, seed=7, nfun=4, R=R)
    S, H, L = _pat(w, w.R_S), _pat(w, w.R_H), _pat(w, w.R_L)
    M = _pat(w, xz_range(w.R_S, w.R_L))
    SL, _ = ost.pattern_product(S, L)
    LS, _ = ost.pattern_product(L, S)
    X, _ = ost.pattern_product(H, LS)
    Z, _ = ost.pattern_product(S, LS)
    need, _ = ost.pattern_product(LS, L)            # (k, j): (i, k) in S.L, (i, j) in L
    for P in (need, need.T.tocsr(), L):
        outside = P.multiply(M) != P
        assert outside.nnz == 0
    # the cut removes natural-range entries that nothing reads
    cut = X.nnz - X.multiply(M).nnz + Z.nnz - Z.multiply(M).nnz
    print(f"{cubes}: {X.nnz} X and {Z.nnz} Z blocks, {cut} outside the cut", flush=True)
    if cuts:
        assert cut > 0
