"""Extended-Lagrangian Born-Oppenheimer MD with the LNV minimisation --
test infrastructure (plain dense FP64).

Sec. III.C (moving atoms): reusing the previous L as the start of each MD
step breaks time reversibility; the code instead propagates an auxiliary
matrix X associated with LS in a harmonic potential centred on the ground
state,
    X(t+dt) = 2X(t) - X(t-dt) + dt^2 w^2 [L(t)S(t) - X(t)]
            + alpha sum_{m=0..M} c_m X(t - m dt)      (dissipation),
and starts the minimisation at the new geometry from L = X S^-1.  Readings
(the paper gives the scheme, not its constants): kappa = dt^2 w^2 = 1.82,
alpha = 0.018 and c = (-6, 14, -8, -3, 4, -1) (M = 5), the published
dissipative coefficients of Niklasson, Steneteg, Odell, Bock, Challacombe,
Tymczak, Holmstrom, Zheng and Weber (J. Chem. Phys. 130, 214109 (2009));
S^-1 is the Hotelling approximate inverse T on L's range and the start is
the symmetric part of P_L(X T) (X ~ LS is not symmetric, nor is X T for an
approximate T, and L is symmetric, stored in both triangles); X
lives on the pattern of L.S (the natural range of LS) of the current
geometry; the history starts at rest (X(-m dt) = L(0)S(0)).

Each minimisation runs at most cg_steps CG iterations and stops after the
iteration whose projected gradient has ||g||_F <= 1e-6 sqrt(entries of L)
(a convergence test the paper leaves undefined: iterated on rounding noise
past convergence, the CG eventually leaves the minimum).

Ions: velocity Verlet with the forces of the synthetic S(x), H(x) at the
minimised L in the constrained form -(dE/dx - mu dN/dx) (oracle.forces), mu
the chemical potential of the last CG iteration.  Units: bohr, Hartree, m_e,
atomic time.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import forces as of
from . import lnv
from . import pm
from . import structure as st

KAPPA = 1.82
ALPHA = 0.018
COEFFS = (-6.0, 14.0, -8.0, -3.0, 4.0, -1.0)


def propagate(hist, LS, kappa=KAPPA, alpha=ALPHA, coeffs=COEFFS):
    """X(t+dt) from hist = [X(t), X(t-dt), ...] (len >= len(coeffs)) and
    LS = L(t) S(t)."""
    X = 2.0 * hist[0] - hist[1] + kappa * (LS - hist[0])
    for m, c in enumerate(coeffs):
        X = X + alpha * c * hist[m]
    return X


def ls_mask(sy, w):
    """Orbital mask of the natural pattern of L.S."""
    n = w.n
    P, _ = st.pattern_product(st.pattern_matrix(*sy.pat["L"], n), st.pattern_matrix(*sy.pat["S"], n))
    return st.block_mask(P.indptr, P.indices, w.nfun)


def g_tol(sy):
    return 1e-6 * float(np.sqrt(np.count_nonzero(sy.maskL)))


def ground_state(sy, w, L0, T, cg_steps):
    """CG from L0 with metric T; returns (L, mu of the last iteration, hist)."""
    L, hist = lnv.cg(sy.S, sy.H, sy.maskL, w.n_elec, cg_steps, L0=L0, T=T, stop_g=g_tol(sy))
    return L, hist[-1]["mu"], hist


def forces(w, sy, L, mu):
    gS = lnv.grad_S(L, sy.S, sy.H, sy.maskS)
    gH = lnv.grad_H(L, sy.S, sy.maskH)
    gN = lnv.grad_N_S(L, sy.S, sy.maskS)
    dEdx = of.energy_gradient_positions(w, gS, gH)
    dNdx = of.energy_gradient_positions(w, gN, np.zeros_like(gH))
    return -(dEdx - mu * dNdx)


def run(w, masses, vel, dt, n_steps, cg_steps=4, pm_steps=60, n_hotelling=16,
        kappa=KAPPA, alpha=ALPHA, coeffs=COEFFS):
    """XLBOMD trajectory; returns a list of per-step dicts (E band energy,
    kinetic energy, N, positions, velocities)."""
    m = np.asarray(masses, dtype=np.float64)[:, None]
    pos = np.array(w.pos, dtype=np.float64)
    vel = np.array(vel, dtype=np.float64)
    sy = st.System(w)
    T = lnv.hotelling(sy.S, sy.maskL, n_hotelling)
    K, _, _ = pm.purify(sy.S, sy.H, T, sy.maskL, w.n_elec, pm_steps)
    L, mu, h = ground_state(sy, w, K, T, cg_steps)
    F = forces(w, sy, L, mu)
    maskLS = ls_mask(sy, w)
    LS = (L @ sy.S) * maskLS
    xh = [LS.copy() for _ in coeffs]
    out = []
    for step in range(n_steps):
        vel = vel + 0.5 * dt * F / m
        pos = np.mod(pos + dt * vel, w.box)
        w = dataclasses.replace(w, pos=pos)
        sy = st.System(w)
        maskLS = ls_mask(sy, w)
        X = propagate(xh, LS, kappa, alpha, coeffs) * maskLS
        xh = [X] + [x * maskLS for x in xh[:-1]]
        T = lnv.hotelling(sy.S, sy.maskL, n_hotelling)
        L0 = (X @ T) * sy.maskL
        L0 = (L0 + L0.T) * 0.5
        L, mu, h = ground_state(sy, w, L0, T, cg_steps)
        E, N, _, _ = lnv.evaluate(L, sy.S, sy.H, sy.maskL)
        F = forces(w, sy, L, mu)
        vel = vel + 0.5 * dt * F / m
        LS = (L @ sy.S) * maskLS
        ekin = 0.5 * float(np.sum(m * vel * vel))
        out.append(dict(step=step, E=E, N=N, ekin=ekin, pos=pos.copy(), vel=vel.copy(),
                        mu=mu, alpha0=h[0]["alpha"], cg_iters=len(h)))
    return out
