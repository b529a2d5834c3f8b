"""Adjoint of the LNV energy on the GPU: dE/dL, dE/dS, dE/dH.

* Against the oracle's closed forms (dense FP64) on the 64-atom cell and on a
  216-atom cell whose rows span several 64-block work pieces, at seeded
  symmetric L: relative 1e-12 of the largest entry, as for G and F.
* Through the autograd wrapper LNVEnergy: E equals lnv_eval's, gradients
  equal the adjoint's and scale with the incoming gradient.
* Central finite differences at the 16384-atom cell (16x16x8 cubes), at the
  L reached by one CG step, on 50 seeded stored entries of each of L, S and H.
  Every input is symmetric, so each entry (i,j,r,c) is perturbed together
  with its mirror (j,i,c,r): the change of E is then G_ij[r,c] + G_ji[c,r].
  E is a cubic polynomial in L, quadratic in S and linear in H, so the central
  difference is exact for S and H and carries only a truncation term
  h^2 E'''/6 = O(1e-10) for L.  What remains is the rounding of E itself:
  |E| is about 1.2e4 Ha at this L and each trace sums ~1e9 products, so E is
  known to ~1e-11 Ha, which over 2h = 2e-5 is ~1e-6 in the difference.  The
  bound is 2e-6 + 1e-6 |dE| (the largest error seen is about a third of it).
"""
import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost

pytestmark = pytest.mark.gpu


def _dense(sysg, V, pat):
    rp, col = pat.host()
    return ost.blocks_to_dense(V.cpu().numpy(), rp, col, sysg.w.nfun)


def _set(sysg, M, pat, A):
    rp, col = pat.host()
    M.val.copy_(torch.as_tensor(ost.dense_to_blocks(A, rp, col, sysg.w.nfun)))


def _rand_sym(n, mask, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n, n)) * scale
    return ((C + C.T) * 0.5) * mask


@pytest.fixture(scope="module")
def si64(gpu):
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get("si64_4x4")
    return LNVSystem(w, metric=None), ost.System(w)


@pytest.fixture(scope="module")
def si216(gpu):
    from paper_2002_07704_amd.system import LNVSystem
    w = W.diamond_workload("si216", (3, 3, 3), seed=7)
    return LNVSystem(w, metric=None), ost.System(w)


@pytest.mark.parametrize("fx", ["si64", "si216"])
def test_adjoint_matches_oracle(fx, request):
    sysg, ref = request.getfixturevalue(fx)
    n = ref.S.shape[0]
    for seed in (3, 11):
        Ld = _rand_sym(n, ref.maskL, seed) + 0.2 * np.eye(n) * ref.maskL
        _set(sysg, sysg.L, sysg.pL, Ld)
        dS = torch.empty_like(sysg.S.val)
        dH = torch.empty_like(sysg.H.val)
        sysg.adjoint(sysg.L.val, sysg.S.val, sysg.H.val, dS=dS, dH=dH)
        torch.cuda.synchronize()
        gS = olnv.grad_S(Ld, ref.S, ref.H, ref.maskS)
        gH = olnv.grad_H(Ld, ref.S, ref.maskH)
        eS = np.abs(_dense(sysg, dS, sysg.pS) - gS).max()
        eH = np.abs(_dense(sysg, dH, sysg.pH) - gH).max()
        print(f"{fx} seed {seed}: dS err {eS:.2e} (max {np.abs(gS).max():.2e}) "
              f"dH err {eH:.2e} (max {np.abs(gH).max():.2e})", flush=True)
        assert eS <= 1e-12 * np.abs(gS).max()
        assert eH <= 1e-12 * np.abs(gH).max()
        # one-sided requests give the same values
        dS1 = torch.empty_like(dS)
        dH1 = torch.empty_like(dH)
        sysg.adjoint(sysg.L.val, sysg.S.val, sysg.H.val, dS=dS1)
        sysg.adjoint(sysg.L.val, sysg.S.val, sysg.H.val, dH=dH1)
        torch.cuda.synchronize()
        assert torch.equal(dS1, dS) and torch.equal(dH1, dH)


def test_adjoint_without_transposes_agrees(si64):
    """The workspace's optional transposes LS, LH only change which operand
    of the restricted products carries the long range (P_H(LS.LSL) for
    P_H(LSL.SL), Y^T for Y): without them the adjoint takes the other
    association, and the results agree to rounding; dN/dS too."""
    from paper_2002_07704_amd import lib as L_
    sysg, ref = si64
    n = ref.S.shape[0]
    Ld = _rand_sym(n, ref.maskL, 7) + 0.2 * np.eye(n) * ref.maskL
    _set(sysg, sysg.L, sysg.pL, Ld)
    out = []
    ws = sysg.adj_ws if sysg.adj_ws is not None else (sysg.adjoint_setup(), sysg.adj_ws)[1]
    saved = (ws.LS, ws.perm_SL, ws.LH, ws.perm_HL)
    try:
        for with_t in (True, False):
            if not with_t:
                ws.LS, ws.perm_SL, ws.LH, ws.perm_HL = L_.LnvBsm(), None, L_.LnvBsm(), None
            dS = torch.empty_like(sysg.S.val)
            dH = torch.empty_like(sysg.H.val)
            dN = torch.empty_like(sysg.S.val)
            sysg.adjoint(sysg.L.val, sysg.S.val, sysg.H.val, dS=dS, dH=dH, dNS=dN)
            torch.cuda.synchronize()
            out.append((dS, dH, dN))
    finally:
        ws.LS, ws.perm_SL, ws.LH, ws.perm_HL = saved
    for a, b in zip(*out):
        assert float((a - b).abs().max()) <= 1e-12 * float(b.abs().max())
    gS = olnv.grad_S(Ld, ref.S, ref.H, ref.maskS)
    assert np.abs(_dense(sysg, out[0][0], sysg.pS) - gS).max() <= 1e-12 * np.abs(gS).max()


def test_lnv_energy_autograd(si64):
    from paper_2002_07704_amd.autograd import LNVEnergy
    sysg, ref = si64
    n = ref.S.shape[0]
    Ld = _rand_sym(n, ref.maskL, 5) + 0.2 * np.eye(n) * ref.maskL
    rp, col = sysg.pL.host()
    Lv = torch.as_tensor(ost.dense_to_blocks(Ld, rp, col, sysg.w.nfun)).cuda().requires_grad_()
    Sv = sysg.S.val.clone().requires_grad_()
    Hv = sysg.H.val.clone().requires_grad_()
    E = LNVEnergy.apply(Lv, Sv, Hv, sysg)
    (3.0 * E).backward()
    torch.cuda.synchronize()
    Er, _, Gr, _ = olnv.evaluate(Ld, ref.S, ref.H, ref.maskL)
    assert abs(float(E.detach()) - Er) / sysg.w.n <= 1e-10
    gS = olnv.grad_S(Ld, ref.S, ref.H, ref.maskS)
    gH = olnv.grad_H(Ld, ref.S, ref.maskH)
    assert np.abs(_dense(sysg, Lv.grad, sysg.pL) - 3.0 * Gr).max() <= 3e-12 * np.abs(Gr).max()
    assert np.abs(_dense(sysg, Sv.grad, sysg.pS) - 3.0 * gS).max() <= 3e-12 * np.abs(gS).max()
    assert np.abs(_dense(sysg, Hv.grad, sysg.pH) - 3.0 * gH).max() <= 3e-12 * np.abs(gH).max()
    # a request for dE/dL alone (S, H constant)
    Lv2 = Lv.detach().clone().requires_grad_()
    E2 = LNVEnergy.apply(Lv2, sysg.S.val, sysg.H.val, sysg)
    E2.backward()
    assert torch.allclose(Lv2.grad, Lv.grad / 3.0, rtol=1e-15, atol=0)


def test_lnv_energy_rejects_bad_values(si64):
    from paper_2002_07704_amd.autograd import LNVEnergy
    sysg, _ = si64
    with pytest.raises(ValueError):
        LNVEnergy.apply(sysg.L.val.float(), sysg.S.val, sysg.H.val, sysg)
    with pytest.raises(ValueError):
        LNVEnergy.apply(sysg.L.val[:-1], sysg.S.val, sysg.H.val, sysg)


def _mirror(pat):
    """Position of block (j, i) for every stored block (i, j)."""
    rp, col = pat.host()
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    key = rows.astype(np.int64) * (len(rp) - 1) + col
    tkey = col.astype(np.int64) * (len(rp) - 1) + rows
    q = np.searchsorted(key, tkey)
    assert np.array_equal(key[q], tkey)
    return q


def test_adjoint_finite_differences_si16384(gpu):
    from paper_2002_07704_amd.autograd import LNVEnergy
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get("si16384_4x4")
    print(f"building {w.name}: {w.n} atoms", flush=True)
    sysg = LNVSystem(w)
    sysg.cg_init()
    sysg.cg_step()
    torch.cuda.synchronize()
    assert int(sysg.scalar("STATUS")) == 0
    Lv = sysg.L.val.clone().requires_grad_()
    Sv = sysg.S.val.clone().requires_grad_()
    Hv = sysg.H.val.clone().requires_grad_()
    E = LNVEnergy.apply(Lv, Sv, Hv, sysg)
    E.backward()
    torch.cuda.synchronize()
    print(f"E/atom {float(E) / w.n:.12f}", flush=True)
    h = 1e-5
    for which, (name, V, pat) in enumerate((("L", Lv, sysg.pL), ("S", Sv, sysg.pS),
                                            ("H", Hv, sysg.pH))):
        grad = V.grad.cpu().numpy()
        q = _mirror(pat)
        ps, rs, cs = W.fd_entries(w.seed, which, pat.nnzb, 50)
        worst = 0.0
        for p, r, c in zip(ps, rs, cs):
            p, r, c = int(p), int(r), int(c)
            pm = int(q[p])
            two = not (pm == p and r == c)
            an = grad[p, r, c] + (grad[pm, c, r] if two else 0.0)
            E2 = []
            for sgn in (1.0, -1.0):
                X = V.detach().clone()
                X[p, r, c] += sgn * h
                if two:
                    X[pm, c, r] += sgn * h
                args = [Lv.detach(), Sv.detach(), Hv.detach()]
                args[which] = X
                with torch.no_grad():
                    E2.append(float(LNVEnergy.apply(*args, sysg)))
            fd = (E2[0] - E2[1]) / (2 * h)
            err = abs(fd - an)
            worst = max(worst, err / (2e-6 + 1e-6 * abs(an)))
            assert err <= 2e-6 + 1e-6 * abs(an), (name, p, r, c, fd, an)
        print(f"dE/d{name}: 50 entries, worst error / bound {worst:.3f}", flush=True)
