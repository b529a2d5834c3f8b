"""XLBOMD on the GPU (paper_2002_07704_amd/xlbomd.py) against the oracle's
XLBOMD (oracle/xlbomd.py, pinned by energy conservation) on the same seeded
start: 64-atom cell, 300 K, three steps of 20 atomic time units, at most 25
CG iterations per step.  Per step: band energy, electron number, kinetic
energy, CG iterations, positions and velocities.  Then the 4096-atom cell for
four steps: the total energy stays within 1% of the kinetic energy exchanged.
"""
import numpy as np
import pytest

import lnv_workloads as W
from oracle import xlbomd as ox

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("order", [None, "bonds"], ids=["atoms", "bonds"])
def test_xlbomd_matches_oracle_si64(gpu, order):
    """Three MD steps against the oracle's, with the rows in the atoms' own
    order and in groups of four bonded atoms (positions, velocities and forces
    stay in atom order; the row order only relabels the matrices)."""
    from paper_2002_07704_amd.xlbomd import XLBOMD
    w = W.get("si64_4x4")
    m, v = W.masses(w), W.thermal_velocities(w, 300.0, 1)
    ref = ox.run(w, m, v, 20.0, 3, cg_steps=25)
    md = XLBOMD(w, m, v, 20.0, cg_steps=25, reorder=order)
    for k, r in enumerate(ref):
        o = md.step()
        print(f"step {k}: E gpu {o['E']:.12f} oracle {r['E']:.12f} ekin {o['ekin']:.9e} "
              f"iters {o['cg_iters']}/{r['cg_iters']}", flush=True)
        assert o["cg_iters"] == r["cg_iters"], k
        assert abs(o["E"] - r["E"]) / w.n <= 1e-10, k
        assert abs(o["N"] - r["N"]) <= 1e-9 * w.n_elec, k
        assert abs(o["ekin"] - r["ekin"]) <= 1e-9 * r["ekin"], k
        assert np.abs(o["pos"] - r["pos"]).max() <= 1e-11, k
        assert np.abs(o["vel"] - r["vel"]).max() <= 1e-9 * np.abs(r["vel"]).max(), k


def test_xlbomd_energy_conservation_si4096(gpu):
    import time
    from paper_2002_07704_amd.xlbomd import XLBOMD
    w = W.get("si4096_4x4")
    md = XLBOMD(w, W.masses(w), W.thermal_velocities(w, 300.0, 1), 20.0, cg_steps=25,
                reorder="bonds")
    out = []
    for k in range(4):
        t0 = time.perf_counter()
        out.append(md.step())
        o = out[-1]
        print(f"step {k}: E/atom {o['E'] / w.n:.10f} ekin {o['ekin']:.6e} N {o['N']:.6f} "
              f"iters {o['cg_iters']} rebuilds {md.rebuilds} {time.perf_counter() - t0:.2f} s",
              flush=True)
    e0 = out[0]["E"] + out[0]["ekin"]
    dk = abs(out[-1]["ekin"] - out[0]["ekin"])
    for o in out:
        assert abs(o["N"] - w.n_elec) <= 1e-9 * w.n_elec
        assert abs(o["E"] + o["ekin"] - e0) <= 0.01 * dk + 1e-9 * abs(e0)
