"""LNV density-matrix functional, gradients and CG minimisation (dense FP64).

Test infrastructure only (see the package docstring).  Every matrix here is a
dense N_orb x N_orb numpy array; range truncation is a 0/1 orbital mask.

Sec. II.C.2 of the paper defines the method:
  * the density matrix is written through an auxiliary matrix L of restricted
    range with the McWeeny form  K = 3LSL - 2LSLSL ;
  * the band energy E = 2 Tr[KH] is minimised with respect to the elements of
    L, using the gradient dE/dL, under a constraint on the electron number,
    N = 2 Tr[KS] (spin-degenerate occupation, the same factor 2 as in E);
  * K has the range of H; it is L whose range is restricted.
Sec. V.C (gramicidin A run) states that the search direction of the density
matrix minimisation is reset every 40 iterations.

The paper does not spell out the electron-number scheme, the CG flavour, the
line search or the initial L beyond naming their sources; the readings taken
here are: gradient projection against dN/dL, Polak-Ribiere (clamped at zero)
directions with the 40-step reset, exact minimisation of the cubic
Omega(alpha) = (E - mu N)(L + alpha D), a cubic electron-number correction
along dN/dL after each step, L0 = lambda * T on L's range with lambda the
smallest positive root of N(lambda T) = N_e, and a runaway guard: two
consecutive rises of E, or occupation numbers (eigenvalues of L S) outside
[-0.5, 1.5], restart the direction, and a second trip within one reset
period marks the minimisation as running away (the McWeeny form 3x^2 - 2x^3
is bounded only for occupations x near [0, 1]).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def tr_prod(A, B):
    """Tr[A B] = sum_ab A_ab B_ba."""
    return float(np.einsum("ab,ba->", A, B))


def dot(A, B):
    """<A, B> = sum_ab A_ab B_ab."""
    return float(np.sum(A * B))


# ------------------------------------------------------------------ functional
def mcweeny(L, S):
    """K = 3LSL - 2LSLSL (Sec. II.C.2)."""
    LSL = L @ S @ L
    return 3.0 * LSL - 2.0 * (LSL @ S @ L)


def evaluate(L, S, H, maskL):
    """E = 2Tr[KH], N = 2Tr[KS], G = dE/dL and F = dN/dL on L's range.

    With E = 6 Tr[LSLH] - 4 Tr[LSLSLH], differentiating each entry of L:
      G = 2 [3 (SLH + HLS) - 2 (SLSLH + SLHLS + HLSLS)]
      F = 12 (SLS - SLSLS)
    both restricted to the range of L (the free variables).
    """
    K = mcweeny(L, S)
    E = 2.0 * tr_prod(K, H)
    N = 2.0 * tr_prod(K, S)
    SLH = S @ L @ H
    HLS = H @ L @ S
    SLSLH = S @ L @ S @ L @ H
    SLHLS = S @ L @ H @ L @ S
    HLSLS = H @ L @ S @ L @ S
    G = 2.0 * (3.0 * (SLH + HLS) - 2.0 * (SLSLH + SLHLS + HLSLS)) * maskL
    SLS = S @ L @ S
    SLSLS = S @ L @ S @ L @ S
    F = 12.0 * (SLS - SLSLS) * maskL
    return E, N, G, F


def grad_S(L, S, H, maskS):
    """dE/dS on S's range: 2 [3 LHL - 2 (LSLHL + LHLSL)]."""
    LHL = L @ H @ L
    return 2.0 * (3.0 * LHL - 2.0 * (L @ S @ LHL + LHL @ S @ L)) * maskS


def grad_N_S(L, S, maskS):
    """dN/dS on S's range: N = 2 Tr[KS] = 6 Tr[LSLS] - 4 Tr[LSLSLS], so
    dN/dS = 12 (LSL - LSLSL)."""
    LSL = L @ S @ L
    return 12.0 * (LSL - LSL @ S @ L) * maskS


def grad_H(L, S, maskH):
    """dE/dH on H's range: 2K (E = 2 Tr[KH] is linear in H)."""
    return 2.0 * mcweeny(L, S) * maskH


def k_coeffs(L, D, S):
    """Matrix coefficients of K(L + a D) = K0 + a K1 + a^2 K2 + a^3 K3."""
    LS, DS = L @ S, D @ S
    K0 = 3.0 * (LS @ L) - 2.0 * (LS @ LS @ L)
    K1 = 3.0 * (DS @ L + LS @ D) - 2.0 * (DS @ LS @ L + LS @ DS @ L + LS @ LS @ D)
    K2 = 3.0 * (DS @ D) - 2.0 * (DS @ DS @ L + DS @ LS @ D + LS @ DS @ D)
    K3 = -2.0 * (DS @ DS @ D)
    return K0, K1, K2, K3


def line_coeffs(L, D, S, M):
    """c_m with 2 Tr[K(L + a D) M] = c0 + c1 a + c2 a^2 + c3 a^3."""
    return np.array([2.0 * tr_prod(K, M) for K in k_coeffs(L, D, S)])


# ------------------------------------------------------------------ scalar roots
def cubic_min(c):
    """Local minimum of c0 + c1 a + c2 a^2 + c3 a^3: the real root of
    3 c3 a^2 + 2 c2 a + c1 = 0 where 2 c2 + 6 c3 a > 0; None if there is none."""
    _, c1, c2, c3 = (float(x) for x in c)
    if c3 == 0.0 and c2 == 0.0:
        return None
    r = np.roots([3.0 * c3, 2.0 * c2, c1])
    best = None
    for x in r:
        if np.isreal(x):
            x = float(np.real(x))
            if 2.0 * c2 + 6.0 * c3 * x > 0.0:
                best = x
    return best


def newton_polish(coef, x, iters=8):
    """Refine a root of the polynomial coef (highest degree first) with
    Newton's method; eigenvalues of the companion matrix carry an absolute
    error of order eps times the largest root, which is large relative to a
    small root."""
    p = np.poly1d(coef)
    dp = p.deriv()
    for _ in range(iters):
        d = dp(x)
        if d == 0.0:
            break
        x = x - p(x) / d
    return float(x)


def cubic_smallest_root(c, target):
    """Real root of c0 + c1 d + c2 d^2 + c3 d^3 = target with the smallest |d|."""
    c0, c1, c2, c3 = (float(x) for x in c)
    coef = [c3, c2, c1, c0 - target]
    while coef and coef[0] == 0.0:
        coef = coef[1:]
    if len(coef) < 2:
        return None
    r = [float(np.real(x)) for x in np.roots(coef) if np.isreal(x)]
    if not r:
        return None
    return newton_polish(coef, min(r, key=abs))


# ------------------------------------------------------------------ initial L
def initial_L(S, maskL, n_elec, T=None):
    """L0 = lambda * T on L's range (T = identity by default), lambda the
    smallest positive real root of N(lambda T) = N_e (a cubic in lambda)."""
    Tm = (np.eye(S.shape[0]) if T is None else T) * maskL
    c = line_coeffs(np.zeros_like(S), Tm, S, S)
    coef = [c[3], c[2], c[1], c[0] - n_elec]
    roots = [float(np.real(x)) for x in np.roots(coef) if np.isreal(x) and np.real(x) > 0]
    if not roots:
        raise ValueError("no positive lambda with N(lambda T) = N_e")
    lam = newton_polish(coef, min(roots))
    return lam * Tm, lam


# ------------------------------------------------------------------ CG
def pr_plus_beta(g, gc, g_prev, gc_prev):
    """Polak-Ribiere coefficient clamped at zero (PR+) in the metric of the
    preconditioner: beta = max(0, <g, g_c - g_c,prev> / <g_prev, g_c,prev>),
    g the projected gradient and g_c = P_L(T g T) its preconditioned form.
    With T = I this is the textbook PR+ of nonlinear CG."""
    return max(0.0, dot(g, gc - gc_prev) / dot(g_prev, gc_prev))


def occupations(L, S):
    """Occupation numbers: the eigenvalues of L S, ascending.  L S is similar
    to C^T L C with S = C C^T (Cholesky), which is symmetric."""
    C = np.linalg.cholesky(S)
    return np.linalg.eigvalsh(C.T @ L @ C)


RISE_TOL = 1e-11          # a rise of E beyond this fraction of |E| counts
OCC_RANGE = (-0.5, 1.5)   # occupations outside trip the guard


def guard_step(state, k, E, occ, reset_period):
    """Runaway guard of the CG (reading of the paper's silence on divergence):
    two consecutive rises of E, or occupation bounds occ = (min, max) outside
    OCC_RANGE, restart the direction; a second trip within reset_period
    iterations of the last one marks the run as running away.  state: dict
    with E_prev, rises, guard_k (updated in place).  Returns (reset, runaway)."""
    Ep = state["E_prev"]
    rises = state["rises"] + 1 if (Ep is not None and E > Ep + RISE_TOL * max(1.0, abs(Ep))) else 0
    occ_bad = occ is not None and not (occ[0] >= OCC_RANGE[0] and occ[1] <= OCC_RANGE[1])
    reset = runaway = False
    if rises >= 2 or occ_bad:
        runaway = k - state["guard_k"] <= reset_period
        reset = True
        state["guard_k"] = k
        rises = 0
    state["rises"] = rises
    state["E_prev"] = E
    return reset, runaway


def cg(S, H, maskL, n_elec, n_iter, L0=None, T=None, reset_period=40,
       n_tol=1e-11, step_cap=0.1, stop_g=None, stop_de=None, n_atoms=None, occ_every=0,
       beta_rule=pr_plus_beta, callback=None):
    """Conjugate-gradient LNV minimisation; returns (L, history).

    Iteration k at the current L:
      1. E, N, G, F = evaluate(L)
      2. metric: G_c = P_L(T G T), F_c = P_L(T F T) (identity when T is None)
      3. mu = <G, F_c> / <F, F_c>;  g = G - mu F;  g_c = G_c - mu F_c
      4. beta = 0 when k % reset_period == 0 or after a failed line search,
         otherwise max(0, <g, g_c - g_c_prev> / <g_prev, g_c_prev>)
      5. D = -g_c + beta D_prev;  D <- D - (<D, F> / <F, F_c>) F_c
      6. alpha = local minimiser of Omega(L + alpha D), Omega = E - mu N
         (an exact cubic); none -> alpha = 0 and a reset next iteration
      7. L <- L + alpha D
      8. if |N(L) - N_e| > n_tol N_e: delta = smallest-|delta| real root of
         N(L + delta F_c) = N_e, applied when |delta| ||F_c|| <= step_cap ||L||
    Between 3 and 4 the runaway guard (guard_step) may force beta = 0, with
    the exact occupations of L S every occ_every-th iteration (0: never).
    History entries carry guard (the direction was restarted) and runaway.
    beta_rule(g, g_c, g_prev, g_c,prev) gives beta outside the resets
    (pr_plus_beta; other rules only serve tests that tell them apart);
    callback(entry, G, F), if given, sees each history entry with the
    gradients of that iteration's evaluation (before its step).
    """
    if L0 is None:
        L, _ = initial_L(S, maskL, n_elec, T)
    else:
        L = L0.copy()
    hist = []
    D_prev = g_prev = gc_prev = None
    force_reset = False
    e_hist = []
    gstate = dict(E_prev=None, rises=0, guard_k=-10 ** 9)
    for k in range(n_iter):
        E, N, G, F = evaluate(L, S, H, maskL)
        occ = None
        if occ_every and k % occ_every == 0:
            ev = occupations(L, S)
            occ = (float(ev[0]), float(ev[-1]))
        if T is None:
            Gc, Fc = G, F
        else:
            Gc = (T @ G @ T) * maskL
            Fc = (T @ F @ T) * maskL
        FF = dot(F, Fc)
        mu = dot(G, Fc) / FF
        g = G - mu * F
        gc = Gc - mu * Fc
        guard, runaway = guard_step(gstate, k, E, occ, reset_period)
        if k % reset_period == 0 or force_reset or guard or g_prev is None:
            beta = 0.0
        else:
            beta = beta_rule(g, gc, g_prev, gc_prev)
        D = -gc + beta * D_prev if beta != 0.0 else -gc
        D = D - (dot(D, F) / FF) * Fc
        c = line_coeffs(L, D, S, H - mu * S)
        alpha = cubic_min(c)
        force_reset = alpha is None
        if alpha is None:
            alpha = 0.0
        L = L + alpha * D
        nc = line_coeffs(L, Fc, S, S)
        N1 = nc[0]
        delta = 0.0
        if abs(N1 - n_elec) > n_tol * n_elec:
            d = cubic_smallest_root(nc, n_elec)
            if d is not None and abs(d) * np.sqrt(dot(Fc, Fc)) <= step_cap * np.sqrt(dot(L, L)):
                delta = d
                L = L + delta * Fc
        g_prev, gc_prev, D_prev = g, gc, D
        gnorm = float(np.sqrt(dot(g, g)))
        hist.append(dict(k=k, E=E, N=N, mu=mu, beta=beta, alpha=alpha, delta=delta,
                         c=c.tolist(), nc=nc.tolist(), gnorm=gnorm, N_after_step=N1,
                         guard=guard, runaway=runaway, occ=occ))
        if callback is not None:
            callback(hist[-1], G, F)
        if stop_g is not None and gnorm <= stop_g:
            break
        if stop_de is not None and n_atoms:
            e_hist.append(E)
            if len(e_hist) >= 4 and all(abs(e_hist[-m] - e_hist[-m - 1]) / n_atoms < stop_de
                                        for m in (1, 2, 3)):
                break
    return L, hist


# ------------------------------------------------------------------ exact reference
def exact_density(H, S, n_elec):
    """Exact diagonalisation at Gamma with step occupation (Sec. II.C.1):
    H c = eps S c, K = sum_{n < N_e/2} c_n c_n^T, E = 2 sum_{n < N_e/2} eps_n."""
    eps, C = sla.eigh(H, S)
    nocc = n_elec // 2
    K = C[:, :nocc] @ C[:, :nocc].T
    E = 2.0 * float(np.sum(eps[:nocc]))
    gap = float(eps[nocc] - eps[nocc - 1]) if nocc < len(eps) else float("inf")
    return K, E, gap, eps


# ------------------------------------------------------------------ metric
def gershgorin_scale(S):
    """sigma = 1 / max_a sum_b |S_ab|: 1/sigma bounds the spectrum of S from
    above, so T0 = sigma I gives ||I - T0 S|| < 1 for SPD S."""
    return 1.0 / float(np.max(np.sum(np.abs(S), axis=1)))


def hotelling(S, mask, n_iter, sigma=None):
    """Sparse approximate inverse of S by Hotelling's iteration, truncated to
    the range pattern `mask` after every step (Sec. II.C.2 uses such an
    approximate inverse overlap as the metric of the minimisation):
        T0 = sigma I,   T_{n+1} = P_mask(2 T_n - T_n S T_n)."""
    if sigma is None:
        sigma = gershgorin_scale(S)
    T = sigma * np.eye(S.shape[0]) * mask
    for _ in range(n_iter):
        T = (2.0 * T - T @ S @ T) * mask
    return T
