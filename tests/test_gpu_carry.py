"""S.L and S.L.S carried from one CG step to the next (lnv_cg_step).

A step leaves S.L and S.L.S of its final L in its workspace (by linearity
from the products its line search and electron-number correction already
formed) and the next step starts from them; a reset step (k divisible by the
reset period) forms them afresh, and so does any step after another call
has overwritten them (the workspace's carry flag).  Checked here against the
oracle's CG with a short reset period, by the carried sums against freshly
formed products after a full period, and by an evaluation at another L
between two steps.
"""
import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def si64(gpu):
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get("si64_4x4")
    return LNVSystem(w, metric=None), ost.System(w)


def _scalars_match(sc, h, w, k):
    assert abs(sc["E"] - h["E"]) / w.n <= 1e-10, k
    assert abs(sc["N"] - h["N"]) <= 1e-9, k
    assert abs(sc["MU"] - h["mu"]) <= 1e-9 * max(1.0, abs(h["mu"])), k
    assert abs(sc["BETA"] - h["beta"]) <= 1e-7, k
    assert abs(sc["ALPHA"] - h["alpha"]) <= 1e-8 * abs(h["alpha"]), k
    assert abs(sc["DELTA"] - h["delta"]) <= 1e-8 * max(abs(h["delta"]), 1e-6), k


def test_short_reset_period_against_oracle(si64):
    """Reset period 4 over 12 iterations: the resets at k = 4 and 8 form S.L
    and S.L.S afresh, the other steps carry them; every iteration's scalars
    match the oracle's CG with the same period."""
    sysg, ref = si64
    w = sysg.w
    _, hist = olnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, 12, reset_period=4)
    sysg.opts.reset_period = 4
    try:
        sysg.cg_init()
        for k in range(12):
            sysg.cg_step()
            sc = sysg.scalars_host()
            print(f"k={k} E/atom gpu {sc['E'] / w.n:.13f} oracle {hist[k]['E'] / w.n:.13f} "
                  f"beta {sc['BETA']:.6f} ({hist[k]['beta']:.6f})", flush=True)
            _scalars_match(sc, hist[k], w, k)
            if k % 4 == 0:
                assert sc["BETA"] == 0.0, k
            assert int(sc["STATUS"]) == 0, k
    finally:
        sysg.opts.reset_period = 40


def test_carried_products_equal_fresh_after_a_period(si64):
    """After 39 carried steps (k = 1..39 of a 40-step period) the carried S.L
    and S.L.S equal the products formed afresh at the final L to rounding."""
    from paper_2002_07704_amd.system import Matrix, multiply
    sysg, _ = si64
    sysg.cg_init()
    for _ in range(40):
        sysg.cg_step()
    torch.cuda.synchronize()
    assert int(sysg.scalar("STATUS")) == 0
    assert sysg.ws.ev.carry == 1
    SL_c = sysg.SL2.clone()
    Z_c = sysg.Z.val.clone()
    fresh = Matrix(sysg.pSL)
    multiply(1.0, sysg.S, sysg.L, 0, 0.0, fresh)
    sysg.eval()                               # forms S.L.S afresh in Z
    torch.cuda.synchronize()
    assert sysg.ws.ev.carry == 0
    e_sl = float((SL_c - fresh.val).abs().max() / fresh.val.abs().max())
    e_z = float((Z_c - sysg.Z.val).abs().max() / sysg.Z.val.abs().max())
    print(f"carried vs fresh after 39 steps: S.L {e_sl:.2e}, S.L.S {e_z:.2e}", flush=True)
    assert e_sl <= 1e-12 and e_z <= 1e-12


def test_evaluation_between_steps_clears_the_carry(si64):
    """An lnv_eval at another L on the same workspace between steps 4 and 5
    overwrites Z; step 5 then forms S.L and S.L.S afresh and lands where the
    uninterrupted run does (to rounding), not at the other L's values."""
    sysg, _ = si64
    w = sysg.w
    sysg.cg_init()
    for _ in range(6):
        sysg.cg_step()
    ref = sysg.scalars_host()
    sysg.cg_init()
    for _ in range(5):
        sysg.cg_step()
    G = torch.empty_like(sysg.G.val)
    F = torch.empty_like(sysg.F.val)
    EN = torch.empty(2, dtype=torch.float64, device=sysg.dev)
    sysg.eval_values(1.1 * sysg.L.val, sysg.S.val, sysg.H.val, G, F, EN)
    assert sysg.ws.ev.carry == 0
    sysg.cg_step()
    sc = sysg.scalars_host()
    for key in ("E", "N", "MU", "ALPHA"):
        assert abs(sc[key] - ref[key]) <= 1e-11 * max(1.0, abs(ref[key])), key
    assert abs(sc["E"] - ref["E"]) / w.n <= 1e-12
