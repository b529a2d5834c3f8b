"""Trace identities behind the CG step's cubics (host-side pins).

Along a direction P the energy and the electron number are cubics whose
coefficients need T0 = Tr[PMPS], T1 = Tr[LSPSPM], T2 = Tr[PSPSPM] and
T3 = Tr[PSLSPM] (M = H - mu S, or S).  The device takes T3 = <L, Q>,
T2 = <P, Q> and T1 = <P, S L X_P> with the symmetric Q = S P M P S formed on
the half of L's pattern only (weight 2 for pairs of row groups).  Here the cubics so
formed are checked against the oracle's E and N at points along the line.
"""
import numpy as np

import lnv_workloads as W
from oracle import lnv as olnv
from oracle import structure as ost


def _half_weights(rp, col, n):
    """Weight of each block of the symmetric pattern under the device's half:
    1 inside a row group (both (i, j) and (j, i) kept), 2 for the kept block
    of a pair from two groups, 0 outside (rows grouped in fours, cyclic group
    offset below m/2, as in_half)."""
    g = 2 if n % 4 == 0 else 0
    m = n >> g
    wts = np.zeros((n, n))
    for i in range(n):
        for j in col[rp[i]:rp[i + 1]]:
            A, B = i >> g, j >> g
            if A == B:
                wts[i, j] = 1.0
                continue
            D = (B - A) % m
            if 2 * D < m or (2 * D == m and A < B):
                wts[i, j] = 2.0
    return wts


def test_cubic_traces_from_half_products():
    w = W.get("si64_4x4")
    ref = ost.System(w)
    S, H, maskL = ref.S, ref.H, ref.maskL
    rng = np.random.default_rng(5)
    n = len(S)
    C = rng.standard_normal((n, n)) * 0.02
    L = ((C + C.T) * 0.5 + 0.25 * np.eye(n)) * maskL
    C = rng.standard_normal((n, n)) * 0.01
    P = ((C + C.T) * 0.5) * maskL
    mu = -0.3
    rp, col = ref.pat["L"]
    wb = _half_weights(rp, col, w.n)
    wt = np.kron(wb, np.ones((4, 4)))            # per-entry weights of 4x4 blocks

    def cubic(M):
        XP = M @ P @ S
        Q = S @ P @ XP                           # S P M P S, symmetric
        T0 = float((P * XP).sum())
        T3 = float((wt * L * Q).sum())           # <L, Q> from the half
        T2 = float((wt * P * Q).sum())           # <P, Q> from the half
        T1 = float((P * (S @ L @ XP)).sum())     # <P, S L X_P> in full
        return T0, T1, T2, T3

    def poly(L0, T, lin):
        T0, T1, T2, T3 = T
        return [L0, lin, 2 * (3 * T0 - 2 * (2 * T1 + T3)), -4 * T2]

    E0, N0, G, F = olnv.evaluate(L, S, H, maskL)
    cE = poly(E0 - mu * N0, cubic(H - mu * S), float(((G - mu * F) * P).sum()))
    T = cubic(S)
    assert abs(T[1] - T[3]) <= 1e-12 * abs(T[1])          # T1 = T3 for M = S
    cN = poly(N0, T, float((F * P).sum()))
    for a in (-1.5, -0.4, 0.3, 1.0, 2.0):
        E, N, _, _ = olnv.evaluate(L + a * P, S, H, maskL)
        om = sum(c * a ** k for k, c in enumerate(cE))
        nn = sum(c * a ** k for k, c in enumerate(cN))
        assert abs(om - (E - mu * N)) <= 1e-10 * max(1.0, abs(E)), a
        assert abs(nn - N) <= 1e-10 * max(1.0, abs(N)), a
