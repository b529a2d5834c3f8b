"""Row orders of the atoms (host logic): the bonded groups of the diamond
generator, the validation of an order, and the mapping of a block matrix in a
permuted row order back to the atoms' own order."""
import numpy as np
import pytest

import lnv_workloads as W
from oracle import structure as ost

NN = 10.26 * np.sqrt(3.0) / 4.0          # diamond nearest-neighbour distance (bohr)


@pytest.mark.parametrize("name", ["si8_4x4", "si64_4x4", "si4096_4x4"])
def test_bond_groups_are_bonded_stars(name):
    """Each group is a centre and three atoms a bond length (a quarter of the
    cube diagonal, within the +-0.1 bohr displacements) away from it, and the
    groups hold every atom once."""
    w = W.get(name)
    g = np.asarray(w.groups)
    assert np.array_equal(np.sort(g), np.arange(w.n))
    p = w.pos[g].reshape(-1, 4, 3)
    d = p[:, 1:] - p[:, :1]
    d -= np.round(d / w.box) * w.box
    r = np.linalg.norm(d, axis=2)
    assert np.all(np.abs(r - NN) <= 2 * np.sqrt(3.0) * 0.1 + 1e-12)


def test_row_order_choices():
    from paper_2002_07704_amd.system import row_order
    w = W.get("si64_4x4")
    assert row_order(w, None, False) is None
    assert row_order(w, False, False) is None
    assert np.array_equal(row_order(w, False, True), np.arange(w.n))
    assert np.array_equal(row_order(w, "bonds", False), w.groups)
    o = row_order(w, "cell", False)
    assert np.array_equal(np.sort(o), np.arange(w.n))
    perm = np.random.default_rng(3).permutation(w.n)
    assert np.array_equal(row_order(w, perm, False), perm)
    with pytest.raises(ValueError):
        row_order(w, np.arange(w.n - 1), False)
    with pytest.raises(ValueError):
        row_order(w, np.zeros(w.n, dtype=int), False)
    with pytest.raises(ValueError):
        row_order(w, "spiral", False)
    wa = W.amorphous_workload("siOH48", 48, seed=1)     # no lattice, no bonded groups
    assert wa.groups is None
    with pytest.raises(ValueError):
        row_order(wa, "bonds", True)


def test_atom_order_maps_permuted_rows_back():
    """The range pattern of the atoms in the bonded order, with blocks tagged
    by their atom pair, maps back to the pattern of the atoms' own order with
    each block at its pair."""
    import bench
    w = W.get("si64_4x4")
    g = np.asarray(w.groups)
    rp, col = ost.neighbours(w.pos, w.box, w.R_L)
    rpp, colp = ost.neighbours(w.pos[g], w.box, w.R_L)
    blocks = np.zeros((len(colp), 4, 4))
    for r in range(w.n):
        for t in range(rpp[r], rpp[r + 1]):
            blocks[t] = g[r] * 1000 + g[colp[t]]
    rp2, col2, b2 = bench.atom_order(rpp, colp, blocks, g)
    assert np.array_equal(rp2, rp) and np.array_equal(col2, col)
    for a in range(w.n):
        for t in range(rp[a], rp[a + 1]):
            assert np.all(b2[t] == a * 1000 + col[t])
