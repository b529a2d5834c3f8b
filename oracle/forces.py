"""Synthetic forces -- test infrastructure (plain dense FP64).

The paper obtains forces as the exact derivative of the energy, Pulay terms
included (Sec. III.A); with the synthetic matrices of this work the
positions enter only through the image weights of the generator:

  S_ij = w_S(i,j) M^S_ij + 2 I delta_ij,   H_ij = -w_H(i,j) M^H_ij,
  w(i,j) = sum over images T with d_T <= R of exp(-d_T / a),
  d_T = |x_j - x_i + T|  (T = integer multiples of the cell edges).

At fixed L, for atoms a != b,

  dw(a,b)/dx_a = sum_T exp(-d_T/a) / a * (x_b - x_a + T) / d_T,
  dE/dx_a = sum over stored blocks (a,b) and (b,a), b != a, of
            <dE/dS_ab, M^S_ab> dw_S(a,b)/dx_a - <dE/dH_ab, M^H_ab> dw_H(a,b)/dx_a
            (the (b,a) block contributes with M_ba = M_ab^T),

and the force is -dE/dx.  At a minimum of E under the constraint N = N_e
the same formula with dE/dS - mu dN/dS (dN/dS = 12 (LSL - LSLSL)) gives the
force of the constrained minimum.  Diagonal blocks do not depend on the
positions (their images are lattice vectors).
"""
from __future__ import annotations

import numpy as np

import lnv_workloads as W

from . import structure as st


def weight_grad(dx, box, R, decay):
    """d w / d x_i for pairs with separation dx = x_j - x_i ([..., 3]):
    sum over in-range images of exp(-d/a)/a * (dx + T)/d."""
    dx = np.asarray(dx, dtype=np.float64)
    out = np.zeros(dx.shape)
    m = [int(np.ceil(R / b)) + 1 for b in box]
    R2 = R * R
    for tx in range(-m[0], m[0] + 1):
        for ty in range(-m[1], m[1] + 1):
            for tz in range(-m[2], m[2] + 1):
                v = dx + np.array([tx * box[0], ty * box[1], tz * box[2]])
                d2 = (v[..., 0] * v[..., 0] + v[..., 1] * v[..., 1]) + v[..., 2] * v[..., 2]
                ok = (d2 <= R2) & (d2 > 0.0)
                d = np.sqrt(np.where(ok, d2, 1.0))
                f = np.where(ok, np.exp(-(d / decay)) / decay / d, 0.0)
                out = out + f[..., None] * v
    return out


def energy_gradient_positions(w, gS, gH):
    """dE/dx [n, 3] at fixed L from the dense gradients gS = dE/dS, gH = dE/dH
    (orbital matrices, each stored entry independent)."""
    nf = np.asarray(w.nfun)
    off = st.offsets(nf)
    out = np.zeros((w.n, 3))
    for kind, g, stream, decay, R, sign in (("S", gS, W.STREAM_S, 3.0, w.R_S, 1.0),
                                            ("H", gH, W.STREAM_H, 2.5, w.R_H, -1.0)):
        rp, col = st.neighbours(w.pos, w.box, R)
        for i in range(w.n):
            js = [int(j) for j in col[rp[i]:rp[i + 1]] if j != i]
            if not js:
                continue
            dws = weight_grad(w.pos[js] - w.pos[i], w.box, R, decay)
            for j, dw in zip(js, dws):
                M = st.random_block(w.seed, stream, i, j, int(nf[i]), int(nf[j]), w.scale)
                c = sign * float(np.sum(g[off[i]:off[i + 1], off[j]:off[j + 1]] * M))
                # block (i, j) depends on x_i through dw and on x_j through -dw
                out[i] += c * dw
                out[j] -= c * dw
    return out
