"""Synthetic forces on the GPU (lnv_adjoint + lnv_forces).

* Against the oracle (oracle/forces.py, itself pinned by central differences
  of the dense energy in the positions): the 8-atom cube (every pair has many
  periodic images inside the ranges) and the 48-atom Si/O/H cell (atoms split
  over several stored rows), at a seeded L, plain (-dE/dx at fixed L) and in
  the constrained-minimum form with a chemical potential, -(dE/dx - mu dN/dx).
  Relative 1e-12 of the largest component.
* At the 4096-atom benchmark cell: central differences of the GPU energy with
  S and H generated again at displaced positions (same patterns), for
  components of three atoms; and the forces sum to zero (translation).
"""
import numpy as np
import pytest
import torch

import lnv_workloads as W
from oracle import forces as of
from oracle import lnv as olnv
from oracle import structure as ost

pytestmark = pytest.mark.gpu


def _rand_sym(n, mask, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((n, n)) * scale
    return ((C + C.T) * 0.5) * mask


def _blocks_for(sysg, A):
    """Stored L blocks of the dense orbital matrix A (either layout)."""
    rp, col = sysg.pL.host()
    if not sysg.split:
        return torch.as_tensor(ost.dense_to_blocks(A, rp, col, sysg.w.nfun))
    nfun = np.asarray(sysg.w.nfun)
    atom = sysg.atom_of.cpu().numpy()
    offr = sysg.off_of.cpu().numpy()
    base = ost.offsets(nfun)[atom] + offr
    nv = np.minimum(4, nfun[atom] - offr)
    out = np.zeros((len(col), 4, 4))
    for i in range(len(rp) - 1):
        for p in range(rp[i], rp[i + 1]):
            j = col[p]
            out[p, :nv[i], :nv[j]] = A[base[i]:base[i] + nv[i], base[j]:base[j] + nv[j]]
    return torch.as_tensor(out)


@pytest.mark.parametrize("name", ["si8_4x4", "siOH48"])
def test_forces_match_oracle(gpu, name):
    from paper_2002_07704_amd.system import LNVSystem
    w = W.amorphous_workload("siOH48", 48, seed=21) if name == "siOH48" else W.get(name)
    sysg = LNVSystem(w, metric=None)
    ref = ost.System(w)
    n = ref.S.shape[0]
    Ld = _rand_sym(n, ref.maskL, 4) + 0.2 * np.eye(n) * ref.maskL
    sysg.L.val.copy_(_blocks_for(sysg, Ld))
    gS = olnv.grad_S(Ld, ref.S, ref.H, ref.maskS)
    gH = olnv.grad_H(Ld, ref.S, ref.maskH)
    dEdx = of.energy_gradient_positions(w, gS, gH)
    dNdx = of.energy_gradient_positions(w, olnv.grad_N_S(Ld, ref.S, ref.maskS), 0.0 * gH)
    for mu in (None, 0.3):
        F = sysg.forces(mu=mu).cpu().numpy()
        Fr = -dEdx if mu is None else -(dEdx - mu * dNdx)
        err = np.abs(F - Fr).max() / np.abs(Fr).max()
        print(f"{name} mu={mu}: max |F| {np.abs(Fr).max():.3e}, relative error {err:.1e}",
              flush=True)
        assert err <= 1e-12


def test_forces_finite_differences_si4096(gpu):
    from paper_2002_07704_amd.system import LNVSystem, neighbours
    w = W.get("si4096_4x4")
    sysg = LNVSystem(w)
    sysg.cg_init()
    torch.cuda.synchronize()
    F = sysg.forces().cpu().numpy()
    assert np.abs(F.sum(axis=0)).max() <= 1e-10 * np.abs(F).max()
    pats = {R: sysg.pS if R == w.R_S else sysg.pH for R in (w.R_S, w.R_H)}
    h = 1e-4
    worst = 0.0
    for a in (0, 1234, 4095):
        for k in range(3):
            E = []
            for sg in (1.0, -1.0):
                pos = w.pos.copy()
                pos[a, k] += sg * h
                sysg.move_atoms(pos)
                for R, P in pats.items():      # same range patterns after the move
                    Q = neighbours(sysg.pos, w.box, R)
                    assert torch.equal(Q.row_ptr, P.row_ptr) and torch.equal(Q.col, P.col)
                sysg.eval()
                torch.cuda.synchronize()
                E.append(float(sysg.EN[0]))
            fd = -(E[0] - E[1]) / (2 * h)
            err = abs(fd - F[a, k])
            worst = max(worst, err / (1e-6 * np.abs(F).max()))
            assert err <= 1e-6 * np.abs(F).max(), (a, k, fd, F[a, k])
    sysg.move_atoms(w.pos)
    print(f"FD forces at 4096 atoms: worst error / bound {worst:.3f}", flush=True)
