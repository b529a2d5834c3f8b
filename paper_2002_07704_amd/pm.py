"""Initial L by canonical purification on the GPU (generalised McWeeny).

Sec. II.C.2 starts the minimisation from a density matrix generated from the
Hamiltonian by an iterative generalisation of the McWeeny transform, with
the approximate inverse overlap T of the metric.  With rho = K S, theta =
N_e/2 occupied states of n orbitals (functions present, padding excluded):

  K0 = (lambda/n) (mu T - T H T) + (theta/n) T,  mu = <T, H>/n,
       lambda = min(theta/(b - mu), (n - theta)/(mu + b)),  b = ||T||_inf ||H||_inf
  c  = Tr[rho^2 - rho^3] / Tr[rho - rho^2]   (Tr[rho^p] = <K (SK)^(p-1), S>)
  K  <- ((1 + c) KSK - KSKSK)/c  (c >= 1/2),  ((1 - 2c) K + (1 + c) KSK - KSKSK)/(1 - c)

with KSK = P_L(K . SK), KSKSK = P_L(KSK . SK) truncated to L's range and K
replaced by its symmetric part after each step (truncation leaves KSKSK
unsymmetric, and the step amplifies any antisymmetric part).  It
stops when Tr[rho - rho^2] <= tol theta, after n_iter steps, or before a
step whose c leaves [0, 1] or whose Tr[rho - rho^2] grew (truncation pushes
the spectrum out of [0, 1]).  Every product, trace and update runs in
liblnv's kernels; the host evaluates c and the stopping test.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import lib as L_
from .system import (BLK, Matrix, _ptr, _stream, multiply, product_pattern, transpose,
                     transpose_map)


def _dot(system, A, B):
    part = torch.empty(L_.DOT_PARTIALS, dtype=torch.float64, device=system.dev)
    out = torch.zeros(1, dtype=torch.float64, device=system.dev)
    L_.call("lnv_bsm_dot", ctypes.byref(A.struct), ctypes.byref(B.struct), _ptr(part), _ptr(out),
            _stream())
    return out


def _norm_inf(system, A):
    part = torch.empty(A.pat.n, dtype=torch.float64, device=system.dev)
    out = torch.zeros(1, dtype=torch.float64, device=system.dev)
    L_.call("lnv_bsm_norm_inf", ctypes.byref(A.struct), _ptr(part), _ptr(out), _stream())
    return out


def _lincomb(a, X, b, Y, c, Z, out):
    ref = [ctypes.byref(M.struct) if M is not None else None for M in (Y, Z)]
    L_.call("lnv_bsm_lincomb", float(a), ctypes.byref(X.struct), float(b), ref[0], float(c),
            ref[1], ctypes.byref(out.struct), _stream())


def _pattern_HL(system):
    """pat(H.L) with its index, work list and the system's cluster plan (the
    adjoint's, when it has been set up)."""
    if getattr(system, "pHL", None) is not None:
        return system.pHL
    P = product_pattern(system.pH, system.pL, triples=False).build_index().build_items()
    if system.cluster is not None:
        P.build_cluster(*system.cluster)
    return P


def pm_initial_L(system, n_iter=100, tol=1e-12):
    """Purified K written to system.L; returns the history [dict(c, t1, t2, t3)]
    and the start parameters (mu, b, lambda)."""
    if system.metric is None:
        raise ValueError("canonical purification needs the metric T ~ S^-1")
    system.pH.build_index()
    n = float(np.sum(system.w.nfun)) if system.w is not None else float(system.fun_rows.sum())
    theta = system.n_elec / 2.0
    T, S, H = system.T, system.S, system.H
    mu = float(_dot(system, T, H)) / n
    b = float(_norm_inf(system, T)) * float(_norm_inf(system, H))
    lam = min(theta / (b - mu), (n - theta) / (mu + b))
    HT = Matrix(_pattern_HL(system))             # H.T on pat(H.L), dropped after use
    multiply(1.0, H, T, 0, 0.0, HT)
    K = Matrix(system.pL)
    K2 = Matrix(system.pL)
    K3 = Matrix(system.pL)
    KT = Matrix(system.pL)
    perm_L = transpose_map(system.pL, system.pL)
    multiply(1.0, T, HT, 0, 0.0, K2)             # P_L(T H T)
    del HT
    _lincomb((lam * mu + theta) / n, T, -lam / n, K2, 0.0, None, K)
    SK = system.SL                               # S.K on pat(S.L)
    hist = []
    prev = None
    for _ in range(n_iter):
        multiply(1.0, S, K, 0, 0.0, SK)
        multiply(1.0, K, SK, 0, 0.0, K2)
        multiply(1.0, K2, SK, 0, 0.0, K3)
        t = torch.cat([_dot(system, M, S) for M in (K, K2, K3)]).cpu().numpy()
        t1, t2, t3 = (float(x) for x in t)
        idem = t1 - t2
        c = (t2 - t3) / idem if idem != 0.0 else None
        if (idem <= tol * theta or c is None or not 0.0 <= c <= 1.0
                or (prev is not None and idem > prev)):
            hist.append(dict(c=None, t1=t1, t2=t2, t3=t3))
            break
        prev = idem
        if c >= 0.5:
            _lincomb(0.0, K, (1.0 + c) / c, K2, -1.0 / c, K3, K)
        else:
            _lincomb((1.0 - 2.0 * c) / (1.0 - c), K, (1.0 + c) / (1.0 - c), K2,
                     -1.0 / (1.0 - c), K3, K)
        transpose(K, perm_L, KT)
        _lincomb(0.5, K, 0.5, KT, 0.0, None, K)
        hist.append(dict(c=c, t1=t1, t2=t2, t3=t3))
    system.L.val.copy_(K.val)
    torch.cuda.synchronize()
    assert K.val.shape[1] == BLK
    return hist, dict(mu=mu, b=b, lam=lam)
