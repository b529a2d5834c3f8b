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
