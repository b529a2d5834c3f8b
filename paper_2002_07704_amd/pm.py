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
the spectrum out of [0, 1]).  Every product, trace, update and decision
(c, the stopping test, the coefficients) runs in liblnv (lnv_pm_start,
lnv_pm_step): the steps are queued without synchronising, and the history
is read once at the end.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import lib as L_
from .system import BLK, Matrix, _stream, product_pattern, transpose_map


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
    (c None for the step that stopped) and the start parameters (mu, b, lambda).
    For a batch of cells every cell is purified with its own scalars
    (lnv_pm_start_batch, lnv_pm_step_batch), and both are lists, one entry
    per cell."""
    if system.metric is None:
        raise ValueError("canonical purification needs the metric T ~ S^-1")
    system.pH.build_index()
    batch = system.cells is not None
    ncell = len(system.cells) if batch else 1
    n = float(np.sum(system.w.nfun)) if system.w is not None else float(system.fun_rows.sum())
    dev = system.dev
    T, S, H = system.T, system.S, system.H
    K = Matrix(system.pL)
    K2 = torch.zeros_like(K.val)
    K3 = torch.zeros_like(K.val)
    KT = torch.zeros_like(K.val)
    perm_L = transpose_map(system.pL, system.pL)
    plen = int(L_.load().lnv_partials_len(max(system.pL.struct.n_items,
                                              system.pL.struct.n_cl_items)))
    part = torch.zeros(plen, dtype=torch.float64, device=dev)
    sc = torch.zeros(ncell, L_.PM_NSCALARS, dtype=torch.float64, device=dev)
    hist_d = torch.zeros(ncell, 4 * max(1, n_iter), dtype=torch.float64, device=dev)
    ws = L_.LnvPmWs()
    ws.SK = system.SL.struct                      # S.K on pat(S.L)
    ws.K2, ws.K3, ws.KT = K2.data_ptr(), K3.data_ptr(), KT.data_ptr()
    ws.perm_L = perm_L.data_ptr()
    ws.partials, ws.partials_len = part.data_ptr(), plen
    ws.scalars, ws.hist, ws.hist_len = sc.data_ptr(), hist_d.data_ptr(), int(n_iter)
    HT = Matrix(_pattern_HL(system))             # H.T on pat(H.L), dropped after use
    ref = ctypes.byref
    if batch:
        b = ref(system.batch())
        L_.call("lnv_pm_start_batch", ref(K.struct), ref(T.struct), ref(H.struct), ref(HT.struct),
                b, ref(ws), _stream())
        for _ in range(n_iter):
            L_.call("lnv_pm_step_batch", ref(K.struct), ref(S.struct), b, float(tol), ref(ws),
                    _stream())
    else:
        L_.call("lnv_pm_start", ref(K.struct), ref(T.struct), ref(H.struct), ref(HT.struct), n,
                float(system.n_elec), ref(ws), _stream())
        for _ in range(n_iter):
            L_.call("lnv_pm_step", ref(K.struct), ref(S.struct), float(system.n_elec),
                    float(tol), ref(ws), _stream())
    system.L.val.copy_(K.val)
    v = sc.cpu().numpy()
    h = hist_d.cpu().numpy().reshape(ncell, -1, 4)
    del HT
    assert K.val.shape[1] == BLK
    hists, infos = [], []
    for c in range(ncell):
        hists.append([dict(c=None if np.isnan(r[0]) else float(r[0]), t1=float(r[1]),
                           t2=float(r[2]), t3=float(r[3]))
                      for r in h[c][:int(v[c, L_.PM["STEPS"]])]])
        infos.append(dict(mu=float(v[c, L_.PM["MU"]]), b=float(v[c, L_.PM["B"]]),
                          lam=float(v[c, L_.PM["LAMBDA"]])))
    return (hists, infos) if batch else (hists[0], infos[0])
