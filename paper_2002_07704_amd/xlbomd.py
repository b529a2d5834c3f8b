"""Extended-Lagrangian Born-Oppenheimer molecular dynamics with the LNV
minimisation on the GPU (Sec. III.C, moving atoms).

An auxiliary matrix X associated with LS (on the natural pattern of L.S)
is propagated in a harmonic potential centred on the minimised L(t)S(t),

  X(t+dt) = 2X(t) - X(t-dt) + kappa (L(t)S(t) - X(t)) + alpha sum_m c_m X(t - m dt),

and the minimisation at the new geometry starts from the symmetric part of
P_L(X T), T ~ S^-1 (Hotelling; X T is not symmetric, L is).  kappa = 1.82, alpha = 0.018, c = (-6, 14, -8, -3, 4, -1) are
the published dissipative coefficients (Niklasson et al., J. Chem. Phys. 130,
214109 (2009)) for the dissipation term the paper adds.  Each minimisation
runs at most cg_steps CG iterations and stops after the iteration whose
||g||_F <= 1e-6 sqrt(entries of L).  Ions move by velocity Verlet under the
synthetic forces at the minimised L in the constrained form (lnv_forces with
mu of the last CG iteration).

When a pair crosses a range cutoff the system is built again for the new
geometry and the X history and L(t)S(t) are carried over to the new pattern
of L.S (lnv_bsm_remap: blocks present in both kept, new blocks zero).  All
matrix work runs in liblnv's kernels; the host integrates the positions.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np
import torch

from . import lib as L_
from .pm import _lincomb, pm_initial_L
from .system import LNVSystem, Matrix, _stream, multiply, neighbours, transpose, transpose_map

KAPPA = 1.82
ALPHA = 0.018
COEFFS = (-6.0, 14.0, -8.0, -3.0, 4.0, -1.0)


def _remap(A, B):
    L_.call("lnv_bsm_remap", ctypes.byref(A.struct), ctypes.byref(B.struct), _stream())
    return B


class XLBOMD:
    def __init__(self, w, masses, vel, dt, cg_steps=10, pm_steps=60, n_hotelling=16,
                 kappa=KAPPA, alpha=ALPHA, coeffs=COEFFS, **system_kw):
        self.w = w
        self.m = np.asarray(masses, dtype=np.float64)[:, None]
        self.vel = np.array(vel, dtype=np.float64)
        self.dt = float(dt)
        self.cg_steps = int(cg_steps)
        self.n_hotelling = int(n_hotelling)
        self.kappa, self.alpha, self.coeffs = kappa, alpha, tuple(coeffs)
        self.system_kw = dict(system_kw)
        self.rebuilds = 0
        self.s = self._build(w)
        pm_initial_L(self.s, pm_steps)
        self.cg_iters = self._minimise()
        self.F = self._forces()
        self.LS = self._ls()
        self.hist = [Matrix(self.pLS, self.LS.val.clone()) for _ in self.coeffs]

    # ----------------------------------------------------------- pieces
    def _build(self, w):
        s = LNVSystem(w, metric="hotelling", n_hotelling=self.n_hotelling, **self.system_kw)
        self.pLS = s.pLS
        if self.pLS.items is None:
            self.pLS.build_items()
        return s

    def _ls(self):
        """L S on the natural pattern of L.S."""
        out = Matrix(self.pLS)
        multiply(1.0, self.s.L, self.s.S, 0, 0.0, out)
        return out

    def _minimise(self):
        s = self.s
        tol = 1e-6 * float(np.sqrt(s.pL.nnzb * 16))
        s.cg_restart()
        for k in range(self.cg_steps):
            s.cg_step()
            if s.scalar("GNORM") <= tol:
                return k + 1
        return self.cg_steps

    def _forces(self):
        return self.s.forces(mu=self.s.scalar("MU")).cpu().numpy()

    def _same_patterns(self, pos_rows):
        s = self.s
        for R, P in ((s.R_S, s.pS), (s.R_H, s.pH), (s.R_L, s.pL)):
            Q = neighbours(pos_rows, s.box, R)
            if not (torch.equal(Q.row_ptr, P.row_ptr) and torch.equal(Q.col, P.col)):
                return False
        return True

    # ----------------------------------------------------------- one MD step
    def step(self):
        """One velocity-Verlet step with the XLBOMD start; returns the band
        energy, electron number, kinetic energy and CG iterations."""
        dt, m = self.dt, self.m
        self.vel = self.vel + 0.5 * dt * self.F / m
        pos = np.mod(self.w.pos + dt * self.vel, self.w.box)
        self.w = dataclasses.replace(self.w, pos=pos)
        s = self.s
        rows = pos if s.atom_of is None else pos[s.atom_of.cpu().numpy()]
        rows_t = torch.as_tensor(np.ascontiguousarray(rows), dtype=torch.float64, device=s.dev)
        if self._same_patterns(rows_t):
            s.move_atoms(pos)
            L_.call("lnv_hotelling", ctypes.byref(s.S.struct), ctypes.byref(s.T.struct),
                    self.n_hotelling, ctypes.byref(s.ws), _stream())
        else:
            old_pLS, old_hist, old_LS = self.pLS, self.hist, self.LS
            old_pLS.build_index()
            self.s = s = self._build(self.w)
            self.hist = [_remap(h, Matrix(self.pLS)) for h in old_hist]
            self.LS = _remap(old_LS, Matrix(self.pLS))
            del old_pLS, old_hist, old_LS
            self.rebuilds += 1
        # X(t+dt) from the history and L(t)S(t)
        h = self.hist
        X = Matrix(self.pLS)
        _lincomb(2.0 - self.kappa, h[0], -1.0, h[1], self.kappa, self.LS, X)
        for q in range(0, len(self.coeffs), 2):
            c1 = self.alpha * self.coeffs[q]
            if q + 1 < len(self.coeffs):
                _lincomb(1.0, X, c1, h[q], self.alpha * self.coeffs[q + 1], h[q + 1], X)
            else:
                _lincomb(1.0, X, c1, h[q], 0.0, None, X)
        self.hist = [X] + h[:-1]
        # start of the minimisation: the symmetric part of P_L(X T)
        multiply(1.0, X, s.T, 0, 0.0, s.L)
        if getattr(s, "_perm_L", None) is None:
            s._perm_L = transpose_map(s.pL, s.pL)
        LT = Matrix(s.pL)
        transpose(s.L, s._perm_L, LT)
        _lincomb(0.5, s.L, 0.5, LT, 0.0, None, s.L)
        iters = self._minimise()
        self.F = self._forces()          # mu of the last CG iteration (before eval)
        s.eval()
        E, N = (float(v) for v in s.EN.cpu())
        self.vel = self.vel + 0.5 * dt * self.F / m
        self.LS = self._ls()
        ekin = 0.5 * float(np.sum(m * self.vel * self.vel))
        return dict(E=E, N=N, ekin=ekin, cg_iters=iters, pos=pos.copy(), vel=self.vel.copy())
