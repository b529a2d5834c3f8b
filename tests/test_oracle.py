"""Pins of the CPU oracle against mathematics, not against itself.

Each test checks a property that the paper's definitions (Sec. II.C.2, Eq. for
K = 3LSL - 2LSLSL, E = 2Tr[KH]) or plain mathematics fix independently of how
the oracle is coded: finite differences, homogeneity, invariances, closed forms
at special points, exact diagonalisation, lattice shell counts and the
published SplitMix64 outputs.
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

import lnv_workloads as W
from oracle import lnv
from oracle import structure as st


# ------------------------------------------------------------------ helpers
def random_system(seed=0, n_atoms=6, nf=4, density=0.7):
    rng = np.random.default_rng(seed)
    n = n_atoms * nf
    am = rng.random((n_atoms, n_atoms)) < density
    am = am | am.T | np.eye(n_atoms, dtype=bool)
    mask = np.kron(am.astype(float), np.ones((nf, nf)))
    A = rng.standard_normal((n, n)) * 0.15
    S = (A + A.T) * 0.5 * mask + 2.0 * np.eye(n)
    assert np.linalg.eigvalsh(S).min() > 0.1
    B = rng.standard_normal((n, n))
    H = -(B + B.T) * 0.25 * mask
    C = rng.standard_normal((n, n)) * 0.05
    L = ((C + C.T) * 0.5 + 0.2 * np.eye(n)) * mask
    return L, S, H, mask


# ------------------------------------------------------------------ RNG
def test_splitmix64_published_outputs():
    # First outputs of SplitMix64 seeded with 0, as published with the
    # reference implementation (Vigna's splitmix64.c / Steele-Lea-Flood).
    x = W.splitmix64_at(0, np.arange(3))
    assert [int(v) for v in x] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


# ------------------------------------------------------------------ neighbour lists
def _diamond_shell_count(R, a):
    """Number of diamond-lattice sites within R of a site, counted from exact
    integer lattice vectors in units of a/4 (fcc vectors, plus (1,1,1) for the
    other sublattice)."""
    unit2 = (a / 4.0) ** 2
    m = int(R / (a / 4.0)) + 2
    cnt = 0
    rng = range(-m, m + 1)
    for x in rng:
        for y in rng:
            for z in rng:
                same = x % 2 == 0 and y % 2 == 0 and z % 2 == 0 and (x + y + z) % 4 == 0
                xs, ys, zs = x - 1, y - 1, z - 1
                other = xs % 2 == 0 and ys % 2 == 0 and zs % 2 == 0 and (xs + ys + zs) % 4 == 0
                if (same or other) and (x * x + y * y + z * z) * unit2 <= R * R:
                    cnt += 1
    return cnt


def test_neighbours_perfect_diamond_shell_counts():
    w = W.diamond_workload("perfect", (4, 4, 4), seed=1, disp=0.0)
    for R, expect in ((12.0, 47), (14.0, 87), (16.0, 123)):
        assert _diamond_shell_count(R, 10.26) == expect
        rp, col = st.neighbours(w.pos, w.box, R)
        assert np.all(np.diff(rp) == expect)


@pytest.mark.parametrize("name", ["si64_4x4", "si8_4x4"])
def test_neighbours_match_periodic_kdtree(name):
    w = W.get(name)
    tree = cKDTree(w.pos, boxsize=w.box)
    for R in (w.R_S, w.R_H, w.R_L, 5.0):
        rp, col = st.neighbours(w.pos, w.box, R)
        for i in range(w.n):
            got = set(col[rp[i]:rp[i + 1]].tolist())
            ref = set(tree.query_ball_point(w.pos[i], R))
            assert got == ref
            assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)
            assert i in got


# ------------------------------------------------------------------ synthetic S, H
def test_synthetic_matrices_structure():
    w = W.get("si64_4x4")
    sy = st.System(w)
    S, H = sy.S, sy.H
    assert np.array_equal(S, S.T) and np.array_equal(H, H.T)
    ev = np.linalg.eigvalsh(S)
    assert ev.min() > 0.5
    # zero outside the range patterns
    assert np.all(S[sy.maskS == 0] == 0) and np.all(H[sy.maskH == 0] == 0)
    # image sum: a pair with two images in range (cell edge 20.52 < 2 R_S)
    i = 0
    found = False
    for j in range(1, w.n):
        dx = w.pos[j] - w.pos[i]
        ds = []
        for t in np.ndindex(5, 5, 5):
            v = dx + (np.array(t) - 2) * w.box
            d = math.sqrt(float(v @ v))
            if d <= w.R_S:
                ds.append(d)
        if len(ds) >= 2:
            found = True
            wt = sum(math.exp(-d / 3.0) for d in ds)
            Mref = st.random_block(w.seed, W.STREAM_S, i, j, 4, 4, w.scale)
            got = S[0:4, 4 * j:4 * j + 4]
            assert np.allclose(got, wt * Mref, rtol=1e-13, atol=0)
            break
    assert found


# ------------------------------------------------------------------ functional and gradients
def test_gradients_central_finite_differences():
    L, S, H, mask = random_system(1)
    E, N, G, F = lnv.evaluate(L, S, H, mask)
    gS = lnv.grad_S(L, S, H, np.ones_like(S))
    gH = lnv.grad_H(L, S, np.ones_like(S))
    rng = np.random.default_rng(7)
    idx = np.argwhere(mask > 0)
    h = 1e-5
    for a, b in idx[rng.choice(len(idx), 12, replace=False)]:
        for Mname in ("L", "S", "H"):
            Mp = {"L": L.copy(), "S": S.copy(), "H": H.copy()}
            Mm = {"L": L.copy(), "S": S.copy(), "H": H.copy()}
            Mp[Mname][a, b] += h
            Mm[Mname][a, b] -= h
            Ep, Np, _, _ = lnv.evaluate(Mp["L"], Mp["S"], Mp["H"], mask)
            Em, Nm, _, _ = lnv.evaluate(Mm["L"], Mm["S"], Mm["H"], mask)
            dE = (Ep - Em) / (2 * h)
            dN = (Np - Nm) / (2 * h)
            if Mname == "L":
                assert abs(dE - G[a, b]) < 1e-7 * max(1, abs(G[a, b]))
                assert abs(dN - F[a, b]) < 1e-7 * max(1, abs(F[a, b]))
            elif Mname == "S":
                assert abs(dE - gS[a, b]) < 1e-7 * max(1, abs(gS[a, b]))
            else:
                assert abs(dE - gH[a, b]) < 1e-7 * max(1, abs(gH[a, b]))


def test_euler_homogeneity_identity():
    # E = 6 Tr[LSLH] - 4 Tr[LSLSLH] has parts of degree 2 and 3 in L, so
    # <L, dE/dL> = 12 Tr[LSLH] - 12 Tr[LSLSLH].
    L, S, H, mask = random_system(2)
    E, N, G, F = lnv.evaluate(L, S, H, mask)
    t2 = np.trace(L @ S @ L @ H)
    t3 = np.trace(L @ S @ L @ S @ L @ H)
    assert abs(lnv.dot(G, L) - 12 * (t2 - t3)) < 1e-10 * abs(12 * t2)
    assert abs(E - (6 * t2 - 4 * t3)) < 1e-12 * abs(E)


def test_energy_with_H_equal_S_is_electron_number():
    L, S, H, mask = random_system(3)
    E, N, G, F = lnv.evaluate(L, S, S, mask)
    assert abs(E - N) < 1e-12 * abs(N)
    assert np.allclose(G, F, atol=1e-12 * np.abs(F).max())


def test_per_atom_rotation_invariance():
    L, S, H, mask = random_system(4)
    rng = np.random.default_rng(5)
    blocks = [np.linalg.qr(rng.standard_normal((4, 4)))[0] for _ in range(6)]
    U = np.zeros_like(S)
    for k, Q in enumerate(blocks):
        U[4 * k:4 * k + 4, 4 * k:4 * k + 4] = Q
    E, N, _, _ = lnv.evaluate(L, S, H, mask)
    E2, N2, _, _ = lnv.evaluate(U.T @ L @ U, U.T @ S @ U, U.T @ H @ U, mask)
    assert abs(E - E2) < 1e-13 * abs(E) and abs(N - N2) < 1e-13 * abs(N)


def test_mcweeny_closed_forms():
    L, S, H, mask = random_system(6)
    Si = np.linalg.inv(S)
    for c in (0.3, 0.5, 0.9):
        K = lnv.mcweeny(c * Si, S)
        assert np.allclose(K, (3 * c * c - 2 * c ** 3) * Si, atol=1e-12)
    # S = I: K = V diag(3x^2 - 2x^3) V^T for L = V diag(x) V^T
    rng = np.random.default_rng(8)
    V = np.linalg.qr(rng.standard_normal((12, 12)))[0]
    x = rng.uniform(-0.3, 1.2, 12)
    K = lnv.mcweeny(V @ np.diag(x) @ V.T, np.eye(12))
    assert np.allclose(K, V @ np.diag(3 * x * x - 2 * x ** 3) @ V.T, atol=1e-12)


def test_exact_projector_is_stationary():
    L, S, H, mask = random_system(9)
    full = np.ones_like(S)
    n_elec = 8
    P, E, gap, eps = lnv.exact_density(H, S, n_elec)
    assert np.allclose(lnv.mcweeny(P, S), P, atol=1e-11)
    E2, N2, G, F = lnv.evaluate(P, S, H, full)
    assert abs(E2 - E) < 1e-11 * abs(E)
    assert abs(N2 - n_elec) < 1e-11
    assert np.abs(G).max() < 1e-10 and np.abs(F).max() < 1e-10


def test_line_coefficients_are_exact_cubic():
    L, S, H, mask = random_system(10)
    rng = np.random.default_rng(11)
    C = rng.standard_normal(S.shape)
    D = (C + C.T) * mask * 0.1
    mu = -0.37
    c = lnv.line_coeffs(L, D, S, H - mu * S)
    E0, N0, G, F = lnv.evaluate(L, S, H, mask)
    assert abs(c[0] - (E0 - mu * N0)) < 1e-12 * abs(c[0])
    assert abs(c[1] - lnv.dot(G - mu * F, D)) < 1e-11 * max(1, abs(c[1]))
    for a in (0.3, -0.7, 1.1, 2.5):
        Ea, Na, _, _ = lnv.evaluate(L + a * D, S, H, mask)
        poly = c[0] + c[1] * a + c[2] * a * a + c[3] * a ** 3
        assert abs((Ea - mu * Na) - poly) < 1e-11 * max(1, abs(poly))


def test_cubic_root_helpers():
    # (a - 1)^2 (a + 2) = a^3 - 3a + 2: local min at a = 1
    assert abs(lnv.cubic_min([2, -3, 0, 1]) - 1.0) < 1e-14
    # -(a^3) + 3a: local min at a = -1
    assert abs(lnv.cubic_min([0, 3, 0, -1]) + 1.0) < 1e-14
    # convex quadratic (c3 = 0): min at -c1 / (2 c2)
    assert abs(lnv.cubic_min([0, -4, 2, 0]) - 1.0) < 1e-14
    # monotone cubic: no local minimum
    assert lnv.cubic_min([0, 1, 0, 1]) is None
    # (d - 0.1)(d - 2)(d + 3) roots 0.1, 2, -3 -> smallest |d| is 0.1
    c = np.poly([0.1, 2.0, -3.0])[::-1]
    assert abs(lnv.cubic_smallest_root(c, 0.0) - 0.1) < 1e-13


def test_initial_L_has_target_electron_number():
    w = W.get("si64_4x4")
    sy = st.System(w)
    L0, lam = lnv.initial_L(sy.S, sy.maskL, w.n_elec)
    _, N, _, _ = lnv.evaluate(L0, sy.S, sy.H, sy.maskL)
    assert abs(N - w.n_elec) < 1e-10 * w.n_elec
    assert 0.2 < lam < 0.3


def test_cg_projection_and_descent_si64():
    w = W.get("si64_4x4")
    sy = st.System(w)
    L, hist = lnv.cg(sy.S, sy.H, sy.maskL, w.n_elec, 20)
    E = [h["E"] for h in hist]
    assert all(E[k + 1] < E[k] for k in range(len(E) - 1))
    assert all(abs(h["N"] - w.n_elec) < 1e-9 for h in hist)
    assert all(h["alpha"] > 0 for h in hist)
    K, Ex, gap, _ = lnv.exact_density(sy.H, sy.S, w.n_elec)
    # truncated range and 20 steps: above the exact energy, within 1e-3 Ha/atom
    assert 0 < (E[-1] - Ex) / w.n < 1e-3


def test_check_a_converged_lnv_equals_exact_diagonalisation():
    """Untruncated L on the 8-atom cell with the exact inverse-overlap metric
    reproduces the exact Gamma-point density matrix and band energy, and the
    converged K is idempotent in the S metric with 2Tr[KS] = N_e."""
    w = W.get("si8_4x4", R_L=1000.0)
    sy = st.System(w)
    K, Ex, gap, _ = lnv.exact_density(sy.H, sy.S, w.n_elec)
    assert gap > 1e-2
    T = np.linalg.inv(sy.S)
    nnz = sy.maskL.sum()
    L, hist = lnv.cg(sy.S, sy.H, sy.maskL, w.n_elec, 150, T=T,
                     stop_g=1e-6 * math.sqrt(nnz), stop_de=1e-13, n_atoms=w.n)
    assert len(hist) < 150
    Kl = lnv.mcweeny(L, sy.S)
    E, N, _, _ = lnv.evaluate(L, sy.S, sy.H, sy.maskL)
    assert abs(E - Ex) / w.n < 1e-9
    assert np.abs(Kl - K).max() < 1e-8
    assert abs(2 * lnv.tr_prod(Kl, sy.S) - w.n_elec) <= 1e-9 * w.n_elec
    assert np.abs(Kl @ sy.S @ Kl - Kl).max() < 1e-8


# ------------------------------------------------------------------ metric
def test_hotelling_reaches_inverse_when_range_covers_cell():
    w = W.get("si8_4x4", R_L=1000.0)
    sy = st.System(w)
    T = lnv.hotelling(sy.S, sy.maskL, 16)
    assert np.abs(T - np.linalg.inv(sy.S)).max() < 1e-12


def test_hotelling_truncated_is_symmetric_approximate_inverse():
    w = W.get("si64_4x4")
    sy = st.System(w)
    sig = lnv.gershgorin_scale(sy.S)
    assert sig <= 1.0 / np.linalg.eigvalsh(sy.S).max()
    T = lnv.hotelling(sy.S, sy.maskL, 16)
    assert np.abs(T - T.T).max() < 1e-14
    assert np.all(T[sy.maskL == 0] == 0)
    assert np.abs((T @ sy.S - np.eye(len(T))) * sy.maskL).max() < 1e-3


def test_cg_with_hotelling_metric_descends_si216():
    w = W.diamond_workload("si216", (3, 3, 3), seed=7)
    sy = st.System(w)
    T = lnv.hotelling(sy.S, sy.maskL, 16)
    L, hist = lnv.cg(sy.S, sy.H, sy.maskL, w.n_elec, 8, T=T)
    E = [h["E"] for h in hist]
    assert all(E[k + 1] < E[k] for k in range(len(E) - 1))
    assert all(abs(h["N"] - w.n_elec) < 1e-9 for h in hist[1:])
    assert all(h["alpha"] > 0 for h in hist)


@pytest.mark.parametrize("name", ["si8_4x4", "siOH24"])
def test_synth_blocks_follow_random_block_definition(name):
    """The vectorised generator gives, bit for bit, w(d) M_ij (+ 2I on the S
    diagonal, negated for H) with M_ij from random_block's per-block
    definition, for uniform and for mixed 13/9/4 block sizes."""
    w = W.amorphous_workload("siOH24", 24, seed=5) if name == "siOH24" else W.get(name)
    nf = w.nfun
    for kind, stream, decay, R in (("S", W.STREAM_S, 3.0, w.R_S), ("H", W.STREAM_H, 2.5, w.R_H)):
        rp, col = st.neighbours(w.pos, w.box, R)
        got = st.synth_blocks(w, kind, rp, col)
        for i in range(w.n):
            for t in range(rp[i], rp[i + 1]):
                j = int(col[t])
                M = st.random_block(w.seed, stream, i, j, int(nf[i]), int(nf[j]), w.scale)
                wt = st.image_weight((w.pos[j] - w.pos[i])[None], w.box, R, decay)[0]
                want = wt * M + (2.0 * np.eye(nf[i]) if (kind == "S" and i == j) else 0.0)
                if kind == "H":
                    want = -(wt * M)
                assert np.array_equal(got[t, :nf[i], :nf[j]], want), (kind, i, j)
                assert not got[t, nf[i]:, :].any() and not got[t, :, nf[j]:].any()


@pytest.mark.parametrize("name", ["si64_4x4", "siOH24"])
def test_row_oracle_equals_dense_oracle(name):
    """The row-wise oracle (sparse row panels, for cells too large to be
    dense) reproduces the dense evaluation: per-atom energy and electron
    contributions sum to E and N, and every row of G and F matches."""
    from oracle import rows as orows
    w = W.amorphous_workload("siOH24", 24, seed=5) if name == "siOH24" else W.get(name)
    sysd = st.System(w)
    n_orb = sysd.S.shape[0]
    rng = np.random.default_rng(3)
    C = rng.standard_normal((n_orb, n_orb)) * 0.05
    Ld = ((C + C.T) * 0.5 + 0.2 * np.eye(n_orb)) * sysd.maskL
    E, N, G, F = lnv.evaluate(Ld, sysd.S, sysd.H, sysd.maskL)
    pL = sysd.pat["L"]
    ro = orows.RowOracle(w, sysd.Sb, sysd.Hb, sysd.blocks(Ld, "L"), sysd.pat["S"],
                         sysd.pat["H"], pL)
    off = st.offsets(w.nfun)
    es = ns = 0.0
    for i in range(w.n):
        e, nn, Gb, Fb, cols = ro.row(i)
        es += e
        ns += nn
        assert np.array_equal(cols, pL[1][pL[0][i]:pL[0][i + 1]])
        for t, j in enumerate(cols):
            nj = w.nfun[j]
            ref_g = G[off[i]:off[i + 1], off[j]:off[j + 1]]
            ref_f = F[off[i]:off[i + 1], off[j]:off[j + 1]]
            assert np.abs(Gb[t, :, :nj] - ref_g).max() <= 1e-12 * np.abs(G).max()
            assert np.abs(Fb[t, :, :nj] - ref_f).max() <= 1e-12 * np.abs(F).max()
    assert abs(es - E) <= 1e-11 * abs(E) and abs(ns - N) <= 1e-11 * abs(N)


@pytest.mark.parametrize("name", ["si8_4x4", "siOH24"])
def test_synthetic_forces_central_differences(name):
    """dE/dx at fixed L (oracle.forces) against central differences of the
    dense energy with S and H regenerated at displaced positions; the 8-atom
    cell has many periodic images of each pair inside the ranges."""
    import dataclasses
    from oracle import forces as of
    w = W.amorphous_workload("siOH24", 24, seed=5) if name == "siOH24" else W.get(name)
    sysd = st.System(w)
    n = sysd.S.shape[0]
    rng = np.random.default_rng(7)
    C = rng.standard_normal((n, n)) * 0.05
    L = ((C + C.T) * 0.5 + 0.2 * np.eye(n)) * sysd.maskL
    gS = lnv.grad_S(L, sysd.S, sysd.H, sysd.maskS)
    gH = lnv.grad_H(L, sysd.S, sysd.maskH)
    dEdx = of.energy_gradient_positions(w, gS, gH)
    h = 1e-5
    for a in (0, 3, w.n - 1):
        for k in range(3):
            E = []
            for sg in (1.0, -1.0):
                pos = w.pos.copy()
                pos[a, k] += sg * h
                w2 = dataclasses.replace(w, pos=pos)
                s2 = st.System(w2)
                for key in ("S", "H", "L"):
                    assert all(np.array_equal(x, y) for x, y in zip(s2.pat[key], sysd.pat[key]))
                E.append(lnv.evaluate(L, s2.S, s2.H, sysd.maskL)[0])
            fd = (E[0] - E[1]) / (2 * h)
            assert abs(fd - dEdx[a, k]) <= 1e-7 * max(1.0, np.abs(dEdx).max()), (a, k, fd, dEdx[a, k])
    # translation invariance: the gradient sums to zero
    assert np.abs(dEdx.sum(axis=0)).max() <= 1e-11 * np.abs(dEdx).max()


def test_dN_dS_central_differences():
    w = W.get("si8_4x4")
    sysd = st.System(w)
    n = sysd.S.shape[0]
    rng = np.random.default_rng(11)
    C = rng.standard_normal((n, n)) * 0.05
    L = ((C + C.T) * 0.5 + 0.2 * np.eye(n)) * sysd.maskL
    g = lnv.grad_N_S(L, sysd.S, sysd.maskS)
    h = 1e-6
    for (a, b) in ((0, 0), (1, 5), (7, 30), (12, 3)):
        Sp, Sm = sysd.S.copy(), sysd.S.copy()
        Sp[a, b] += h
        Sm[a, b] -= h
        fd = (lnv.evaluate(L, Sp, sysd.H, sysd.maskL)[1]
              - lnv.evaluate(L, Sm, sysd.H, sysd.maskL)[1]) / (2 * h)
        assert abs(fd - g[a, b]) <= 1e-7 * max(1.0, abs(g[a, b])), (a, b, fd, g[a, b])


def test_purification_reaches_exact_density_untruncated():
    """Canonical purification (oracle/pm.py) with T = S^-1 and L covering the
    8-atom cube: K becomes the exact Gamma-point density matrix (the theta
    lowest generalised eigenvectors), so 2 Tr[KS] = N_e, KSK = K, E = 2 Tr[KH]
    is the exact band energy and the LNV gradient vanishes there."""
    from oracle import pm as opm
    w = W.get("si8_4x4", R_L=1000.0)
    sy = st.System(w, R_L=1000.0)
    T = np.linalg.inv(sy.S)
    K, hist, info = opm.purify(sy.S, sy.H, T, sy.maskL, w.n_elec, 200)
    Kx, Ex, gap, _ = lnv.exact_density(sy.H, sy.S, w.n_elec)
    assert gap >= 1e-2 and hist[-1]["c"] is None and len(hist) < 60
    assert np.abs(K - Kx).max() <= 1e-10
    assert abs(2.0 * np.sum(K * sy.S) - w.n_elec) <= 1e-10 * w.n_elec
    assert np.abs(K @ sy.S @ K - K).max() <= 1e-10
    E, N, G, F = lnv.evaluate(K, sy.S, sy.H, sy.maskL)
    assert abs(E - Ex) <= 1e-10 * abs(Ex) and np.abs(G).max() <= 1e-9
    assert all(h["c"] is None or 0.0 <= h["c"] <= 1.0 for h in hist)


def test_xlbomd_recursion_properties():
    """The X recursion of oracle/xlbomd.py: a constant history at the harmonic
    centre stays there (the dissipation coefficients sum to zero); without
    dissipation the recursion is time reversible (X(t+dt) + X(t-dt) depends
    only on X(t) and LS); the dissipation vanishes on a history linear in
    time (sum c_m = sum m c_m = 0) and the K = 5 coefficients are the
    published ones."""
    from oracle import xlbomd as ox
    rng = np.random.default_rng(2)
    A = rng.standard_normal((6, 6))
    assert np.allclose(ox.propagate([A] * 6, A), A, atol=1e-14)
    X0, X1, LS = (rng.standard_normal((6, 6)) for _ in range(3))
    hist = [X1, X0] + [X0] * 4
    fwd = ox.propagate(hist, LS, alpha=0.0)
    back = ox.propagate([X1, fwd] + [X0] * 4, LS, alpha=0.0)
    assert np.allclose(back, X0, atol=1e-12)
    c = np.array(ox.COEFFS)
    assert c.sum() == 0.0 and (np.arange(6) * c).sum() == 0.0
    assert (ox.KAPPA, ox.ALPHA) == (1.82, 0.018)


def test_xlbomd_conserves_energy_si64():
    """Three velocity-Verlet steps of XLBOMD on the 64-atom cell at 300 K with
    25 CG iterations per step: the total energy (band energy + kinetic) stays
    within 1% of the kinetic energy exchanged, which wrong forces (a sign, a
    missing term) would violate by order one."""
    from oracle import xlbomd as ox
    w = W.get("si64_4x4")
    out = ox.run(w, W.masses(w), W.thermal_velocities(w, 300.0, 1), 20.0, 3, cg_steps=25)
    e0 = out[0]["E"] + out[0]["ekin"]
    dk = abs(out[-1]["ekin"] - out[0]["ekin"])
    assert dk > 1e-4
    for o in out:
        assert abs(o["N"] - w.n_elec) <= 1e-9 * w.n_elec
        assert abs(o["E"] + o["ekin"] - e0) <= 0.01 * dk


# ------------------------------------------------------------------ runaway guard
def test_occupations_closed_forms():
    """Occupations (eigenvalues of L S): L = c S^-1 gives L S = c I; the exact
    Gamma-point density matrix K of the 8-atom cell satisfies K S K = K, so
    its occupations are exactly 0 (empty states) and 1 (N_e / 2 of them)."""
    w = W.get("si8_4x4")
    ref = st.System(w)
    Si = np.linalg.inv(ref.S)
    occ = lnv.occupations(0.37 * Si, ref.S)
    assert np.abs(occ - 0.37).max() <= 1e-12
    K, _, _, _ = lnv.exact_density(ref.H, ref.S, w.n_elec)
    occ = lnv.occupations(K, ref.S)
    nocc = w.n_elec // 2
    assert np.abs(occ[-nocc:] - 1.0).max() <= 1e-10
    assert np.abs(occ[:-nocc]).max() <= 1e-10


def test_guard_rule():
    """Two consecutive rises of E restart the direction; a trip within one
    reset period of the last is a runaway; occupations outside [-0.5, 1.5]
    trip at once; a descent clears the count of rises."""
    st = dict(E_prev=None, rises=0, guard_k=-10 ** 9)
    seq = [(-1.0, None), (-2.0, None), (-1.5, None), (-1.2, None), (-1.3, None),
           (-1.1, None), (-1.0, None), (-2.0, (-0.6, 1.0)), (-3.0, (0.0, 1.0))]
    got = [lnv.guard_step(st, k, E, occ, 40) for k, (E, occ) in enumerate(seq)]
    assert got == [(False, False), (False, False), (False, False), (True, False),
                   (False, False), (False, False), (True, True), (True, True), (False, False)]
    st = dict(E_prev=None, rises=0, guard_k=-10 ** 9)
    lnv.guard_step(st, 0, 0.0, (0.0, 1.6), 40)
    assert lnv.guard_step(st, 41, -1.0, (0.0, 1.6), 40) == (True, False)   # 41 > 40 apart


def test_guard_trips_on_the_runaway_identity_metric_cell():
    """The 8-atom cell minimised with the identity metric drifts to
    occupations below -0.5 (the non-physical state the plain LNV functional
    admits): the guard restarts the direction at iteration 9 and flags the
    runaway at 10.  With the Hotelling metric it never trips."""
    w = W.get("si8_4x4")
    ref = st.System(w)
    _, hist = lnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, 12, occ_every=1)
    trips = [h["k"] for h in hist if h["guard"]]
    runaway = [h["k"] for h in hist if h["runaway"]]
    assert trips[:2] == [9, 10] and runaway[0] == 10
    assert hist[9]["occ"][0] < -0.5 and hist[8]["occ"][0] > -0.5
    T = lnv.hotelling(ref.S, ref.maskL, 16)
    _, hist = lnv.cg(ref.S, ref.H, ref.maskL, w.n_elec, 30, T=T, occ_every=1)
    assert not any(h["guard"] for h in hist)


# ------------------------------------------------------------------ CG direction
def test_pr_plus_beta_hand_values():
    """The Polak-Ribiere coefficient clamped at zero, in the preconditioner's
    metric, on hand-worked vectors (each case is computed in its comment; the
    listed wrong rules give other values):
      g = (1, 2), g_prev = (2, 1), no metric:  <g, g - g_prev> = -1 + 2 = 1,
        |g_prev|^2 = 5  ->  0.2   (Fletcher-Reeves |g|^2/|g_prev|^2 = 1)
      g = (1, 0), g_prev = (2, 1):  <g, g - g_prev> = -1  ->  max(0, -0.2) = 0
        (unclamped -0.2, Fletcher-Reeves 0.2)
      g = (2, 1), g_c = (4, 1), g_prev = (1, 1), g_c,prev = (2, 1):
        <g, g_c - g_c,prev> = <(2, 1), (2, 0)> = 4, <g_prev, g_c,prev> = 3
        ->  4/3   (g for g_c: 1;  g_c for g: 8/3;  FR in the metric 9/3 = 3;
        <g_c,prev, g_c,prev> = 5 below: 4/5)."""
    v = lambda *x: np.array(x, dtype=float).reshape(1, -1)  # noqa: E731
    g, gp = v(1, 2), v(2, 1)
    assert lnv.pr_plus_beta(g, g, gp, gp) == pytest.approx(0.2, rel=1e-15)
    g, gp = v(1, 0), v(2, 1)
    assert lnv.pr_plus_beta(g, g, gp, gp) == 0.0
    g, gc, gp, gcp = v(2, 1), v(4, 1), v(1, 1), v(2, 1)
    assert lnv.pr_plus_beta(g, gc, gp, gcp) == pytest.approx(4.0 / 3.0, rel=1e-15)


def test_cg_direction_rule_sets_the_convergence_rate():
    """Check (a)'s 8-atom cell (untruncated L, exact inverse-overlap metric):
    with the preconditioned PR+ directions the minimisation is within 5e-6
    Ha/atom of the exact band energy after 30 iterations (1.3e-6 measured)
    and stops (||g|| test) before 60; the plausible wrong rules -- steepest
    descent (beta = 0), Fletcher-Reeves, PR+ without the metric, g_c in
    place of g in the numerator -- are all further than 5e-6 from it at
    iteration 30 (3e-5 for Fletcher-Reeves, 2e-3 to 1e-2 for the others), so
    the rule the CG actually applies is the PR+ of test_pr_plus_beta_hand_values."""
    w = W.get("si8_4x4", R_L=1000.0)
    sy = st.System(w)
    T = np.linalg.inv(sy.S)
    _, Ex, _, _ = lnv.exact_density(sy.H, sy.S, w.n_elec)
    nnz = sy.maskL.sum()
    dot = lnv.dot
    wrong = {
        "zero": lambda g, gc, gp, gcp: 0.0,
        "fletcher_reeves": lambda g, gc, gp, gcp: dot(g, gc) / dot(gp, gcp),
        "no_metric": lambda g, gc, gp, gcp: max(0.0, dot(g, g - gp) / dot(gp, gp)),
        "gc_numerator": lambda g, gc, gp, gcp: max(0.0, dot(gc, gc - gcp) / dot(gp, gcp)),
    }

    def err30(rule=None):
        kw = {} if rule is None else {"beta_rule": rule}
        _, hist = lnv.cg(sy.S, sy.H, sy.maskL, w.n_elec, 60, T=T, stop_g=1e-6 * math.sqrt(nnz),
                         stop_de=1e-13, n_atoms=w.n, **kw)
        return (hist[30]["E"] - Ex) / w.n if len(hist) > 30 else 0.0, len(hist)

    e, n = err30()
    assert 0.0 <= e < 5e-6 and n < 60, (e, n)
    for name, rule in wrong.items():
        e_w, _ = err30(rule)
        assert e_w > 5e-6, (name, e_w)


def test_row_oracle_region_patterns_give_the_same_rows():
    """The row-wise oracle on patterns holding only the rows within reach of
    the sampled atoms (region_patterns) gives exactly the rows it gives on the
    full patterns: every row its product chains read is kept.  A 216-atom cell
    with short ranges, so that the reach (R_H + R_S + 2 R_L) covers only part
    of the box."""
    import dataclasses
    from oracle import rows as orows
    w = dataclasses.replace(W.diamond_workload("si216", (3, 3, 3), seed=7),
                            R_S=4.5, R_H=5.0, R_L=4.0)
    atoms = [0, 100]
    (rS, rH, rL), nrow = orows.region_patterns(w, atoms)
    assert 0 < nrow < w.n
    full = [st.neighbours(w.pos, w.box, R) for R in (w.R_S, w.R_H, w.R_L)]

    def oracle(pS, pH, pL):
        Lb = 0.1 * st.synth_blocks(dataclasses.replace(w, seed=w.seed + 1000, R_S=w.R_L), "S", *pL)
        return orows.RowOracle(w, st.synth_blocks(w, "S", *pS), st.synth_blocks(w, "H", *pH),
                               Lb, pS, pH, pL)

    a, b = oracle(rS, rH, rL), oracle(*full)
    for i in atoms:
        ra, rb = a.row(i), b.row(i)
        assert np.array_equal(ra[4], rb[4])
        for x, y in zip(ra[:4], rb[:4]):
            assert np.allclose(x, y, rtol=1e-14, atol=1e-14 * np.abs(y).max())
