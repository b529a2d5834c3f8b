"""Initial density matrix by canonical purification -- test infrastructure.

Sec. II.C.2 generates the starting density matrix from the Hamiltonian with
an iterative generalisation of the McWeeny transform (Palser and
Manolopoulos' canonical purification, extended to a non-orthogonal basis),
with an approximate inverse overlap T ~ S^-1.  In terms of K (support-
function basis) and the projector rho = K S:

  start   K0 = (lambda/n) (mu T - T H T) + (theta/n) T,
          theta = N_e/2 occupied states of n orbitals, mu = Tr[T H]/n,
          lambda = min(theta/(b - mu), (n - theta)/(mu + b)), b >= the
          spectral radius of T H (here ||T||_inf ||H||_inf), so that the
          eigenvalues of rho0 lie in [0, 1] with trace theta (theta Tr[TS]/n
          for an approximate T);
  step    c = Tr[rho^2 - rho^3] / Tr[rho - rho^2],
          K <- ((1 + c) KSK - KSKSK) / c                  if c >= 1/2,
          K <- ((1 - 2c) K + (1 + c) KSK - KSKSK)/(1 - c)  otherwise,
          every product truncated to L's range (mask), and K replaced by
          its symmetric part after each step: the truncated KSKSK =
          P_L(P_L(KSK) S K) is not symmetric, and the step multiplies any
          antisymmetric part of K by about 3 (from rounding level to 1e-1
          within 20 steps), while K must stay symmetric (stored in both
          triangles);
  stop    when Tr[rho - rho^2] <= tol * theta, after n_iter steps, or --
          with truncation the spectrum leaves [0, 1] -- before a step whose
          c falls outside [0, 1] or whose Tr[rho - rho^2] exceeds the
          previous step's (that K is returned, not updated).

The trace Tr[rho] = theta is kept by every step (exactly, without
truncation), the spectrum moves to {0, 1}, and K converges to the density
matrix of the theta lowest states; K is then a valid L for the LNV
functional (its McWeeny transform is itself).
"""
from __future__ import annotations

import numpy as np


def norm_inf(A):
    return float(np.max(np.sum(np.abs(A), axis=1)))


def purify(S, H, T, mask, n_elec, n_iter=100, tol=1e-12):
    """Returns (K, history); history[k] = dict(c, t1, t2, t3) of step k with
    t_p = Tr[rho^p] before the step."""
    n = S.shape[0]
    theta = n_elec / 2.0
    T = T * mask
    mu = float(np.sum(T * H)) / n
    b = norm_inf(T) * norm_inf(H)
    lam = min(theta / (b - mu), (n - theta) / (mu + b))
    K = ((lam / n) * (mu * T - T @ H @ T) + (theta / n) * T) * mask
    hist = []
    prev = None
    for _ in range(n_iter):
        SK = S @ K
        K2 = (K @ SK) * mask
        K3 = (K2 @ SK) * mask
        t1, t2, t3 = (float(np.sum(M * S)) for M in (K, K2, K3))
        idem = t1 - t2
        c = (t2 - t3) / idem if idem != 0.0 else None
        stop = (idem <= tol * theta or c is None or not 0.0 <= c <= 1.0
                or (prev is not None and idem > prev))
        if stop:
            hist.append(dict(c=None, t1=t1, t2=t2, t3=t3))
            break
        prev = idem
        if c >= 0.5:
            K = ((1.0 + c) * K2 - K3) / c
        else:
            K = ((1.0 - 2.0 * c) * K + (1.0 + c) * K2 - K3) / (1.0 - c)
        K = (K + K.T) * 0.5
        hist.append(dict(c=c, t1=t1, t2=t2, t3=t3))
    return K, hist, dict(mu=mu, b=b, lam=lam)
