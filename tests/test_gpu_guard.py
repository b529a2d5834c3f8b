"""Runaway guard of the CG on the GPU against the oracle.

Occupation bounds (extreme eigenvalues of L S) come from Lanczos in the S
inner product: the Ritz values of the tridiagonal lie inside the spectrum
and approach its ends as the number of steps grows, and once the Krylov
space is exhausted they are the exact extremes.  The guard's decisions (a
restart of the direction, a runaway) are integer results of the trajectory
and must match the oracle's iteration by iteration.
"""
import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost
from paper_2002_07704_amd import lib as L_

pytestmark = pytest.mark.gpu


def _set(sysg, M, pat, A):
    rp, col = pat.host()
    M.val.copy_(torch.as_tensor(ost.dense_to_blocks(A, rp, col, sysg.w.nfun)))


def _system(w, **opts):
    from paper_2002_07704_amd.system import LNVSystem
    s = LNVSystem(w, metric=None)
    for k, v in opts.items():
        setattr(s.opts, k, v)
    return s


@pytest.fixture(scope="module")
def si64_drifted(gpu):
    """64-atom cell with L after 10 identity-metric CG iterations of the oracle
    (occupations in about [-0.041, 1.031])."""
    w = W.get("si64_4x4")
    ref = ost.System(w)
    Lo, _ = olnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, 10)
    sysg = _system(w)
    _set(sysg, sysg.L, sysg.pL, Lo)
    return sysg, olnv.occupations(Lo, ref.S)


def test_occupation_bounds_inside_spectrum_and_converging(si64_drifted):
    sysg, ev = si64_drifted
    lo_ex, hi_ex = ev[0], ev[-1]
    eps = 1e-12 * (hi_ex - lo_ex)
    errs = []
    for steps in (8, 16, 32, 64):
        lo, hi = sysg.occupation_bounds(steps)
        print(f"steps {steps}: lo {lo:.15f} (exact {lo_ex:.15f}) hi {hi:.15f} (exact {hi_ex:.15f})",
              flush=True)
        assert lo >= lo_ex - eps and hi <= hi_ex + eps, steps
        errs.append((lo - lo_ex, hi_ex - hi))
    # Ritz values of the extreme ends move outwards with every step
    for (a0, b0), (a1, b1) in zip(errs, errs[1:]):
        assert a1 <= a0 + eps and b1 <= b0 + eps
    # 64 steps on 256 orbitals: the ends have converged
    assert max(errs[-1]) <= 1e-8
    # the guard's default of 16 steps is far inside its [-0.5, 1.5] margin
    assert max(errs[1]) <= 0.05


def test_occupation_bounds_exhausted_krylov_space(gpu):
    """8 atoms x 4 functions = 32 orbitals: 48 steps exhaust the space, the
    bounds are the exact extreme occupations (closed forms: L = c S^-1 gives
    all occupations c)."""
    w = W.get("si8_4x4")
    ref = ost.System(w)
    Lo, _ = olnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, 10)
    sysg = _system(w)
    _set(sysg, sysg.L, sysg.pL, Lo)
    ev = olnv.occupations(Lo, ref.S)
    lo, hi = sysg.occupation_bounds(48)
    assert abs(lo - ev[0]) <= 1e-10 and abs(hi - ev[-1]) <= 1e-10
    # the range of L covers the cell: L = 0.37 S^-1 on L's pattern is exact
    wf = W.get("si8_4x4", R_L=1000.0)
    reff = ost.System(wf)
    sysf = _system(wf)
    Si = np.linalg.inv(reff.S)
    _set(sysf, sysf.L, sysf.pL, 0.37 * Si * reff.maskL)
    lo, hi = sysf.occupation_bounds(48)
    assert abs(lo - 0.37) <= 1e-12 and abs(hi - 0.37) <= 1e-12


def test_guard_trips_match_oracle_on_a_runaway(gpu):
    """Identity-metric CG on the 8-atom cell drifts to occupations below -0.5:
    the guard restarts the direction at iteration 9 and flags the runaway at
    10 on both sides; E, the occupation bounds and the status bits agree at
    every iteration, and lnv_cg_check reports LNV_ENUMERIC."""
    w = W.get("si8_4x4")
    ref = ost.System(w)
    steps = 12
    _, hist = olnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, steps, occ_every=1)
    sysg = _system(w, occ_every=1, occ_iter=64)
    sysg.cg_init()
    guard = runaway = False
    for k in range(steps):
        sysg.cg_step()
        sc = sysg.scalars_host()
        h = hist[k]
        guard |= h["guard"]
        runaway |= h["runaway"]
        st = int(sc["STATUS"])
        print(f"k={k} E gpu {sc['E']:.13f} oracle {h['E']:.13f} occ gpu "
              f"({sc['OCC_MIN']:.6f}, {sc['OCC_MAX']:.6f}) oracle ({h['occ'][0]:.6f}, "
              f"{h['occ'][1]:.6f}) status {st}", flush=True)
        assert abs(sc["E"] - h["E"]) / w.n <= 1e-10, k
        assert abs(sc["OCC_MIN"] - h["occ"][0]) <= 1e-9, k
        assert abs(sc["OCC_MAX"] - h["occ"][1]) <= 1e-9, k
        assert bool(st & L_.ST_GUARD) == guard, k
        assert bool(st & L_.ST_RUNAWAY) == runaway, k
        assert sc["BETA"] == 0.0 or not h["guard"], k
    assert runaway
    with pytest.raises(L_.LnvError) as e:
        sysg.cg_check()
    assert e.value.status == L_.ENUMERIC


def test_guard_quiet_on_a_healthy_run(gpu):
    """The 64-atom cell with its default guard (bounds every 10th iteration
    from 16 Lanczos steps) never trips in 20 iterations, and lnv_cg_check
    returns the clear status."""
    w = W.get("si64_4x4")
    sysg = _system(w)
    sysg.cg_init()
    for _ in range(20):
        sysg.cg_step()
    assert sysg.cg_check() == 0
    lo, hi = sysg.scalar("OCC_MIN"), sysg.scalar("OCC_MAX")
    assert -0.5 < lo < 0.0 and 1.0 < hi < 1.5
