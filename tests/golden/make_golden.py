"""Write the stored expected values of the at-scale parity tests.

Calls only `oracle/` (dense FP64 numpy) and `lnv_workloads`; nothing here
reads any GPU result.  The 4096-atom cell (16384 orbitals) needs ~25 GB of
RAM and tens of minutes on 8 cores per CG step, which is why its values are
stored instead of recomputed inside the GPU tests.

usage: python tests/golden/make_golden.py si4096_4x4 [n_cg_steps]
       python tests/golden/make_golden.py rows siOH8192_mixed
       python tests/golden/make_golden.py rows si32768_13f
       python tests/golden/make_golden.py cgtraj si4096_4x4 [n_cg_steps]

The third form writes <workload>_cg.json and <workload>_cg_rows.npz: the
minimisation the benchmark times, from the oracle alone -- Hotelling's
approximate inverse overlap T (16 steps) as the metric, the canonical
purification start (oracle/pm.py, at most 60 steps), then CG iterations in
that metric -- with every iteration's scalars (E, N, mu, beta, alpha, delta)
and the G and F rows of a few atoms at selected iterations.  Each iteration
is written as soon as it is done (a dense step at 16384 orbitals takes about
20 minutes on 8 cores), so an interrupted run still leaves its first steps.

The second form writes <workload>_rows.npz: the row-wise oracle's G and F
rows (and per-atom energy / electron contributions) of a few sampled atoms at
the seeded test matrix L = 0.1 (w M + 2I) on L's range -- the synthetic
overlap generator with master seed + 1000, range R_L and decay 3 bohr -- for
the cells where no dense matrix fits (the 78646-orbital Si/O/H cell, the
425984-orbital 13-function cell); the oracle's matrices hold only the rows
within reach of the sampled atoms (region_patterns), which the sampled rows
depend on (oracle/rows.py, region_patterns).
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import lnv_workloads as W  # noqa: E402
from oracle import lnv as olnv  # noqa: E402
from oracle import structure as ost  # noqa: E402


L_SEED_OFFSET = 1000
L_SCALE = 0.1


def test_L_blocks(w, patL):
    """The seeded L of the sampled-row tests (oracle side)."""
    import dataclasses
    w2 = dataclasses.replace(w, seed=w.seed + L_SEED_OFFSET, R_S=w.R_L)
    return L_SCALE * ost.synth_blocks(w2, "S", *patL)


def sample_atoms(w):
    """The first atom of each species and three seeded picks (stream 4)."""
    at = [int(np.nonzero(w.species == s)[0][0]) for s in np.unique(w.species)]
    u = W.uniform01(w.seed, W.STREAM_FD, 99, np.arange(3), 0)
    at += [int(x) for x in (u * w.n).astype(int)]
    return sorted(set(at))


def rows_main(name):
    from oracle import rows as orows
    w = W.get(name)
    t0 = time.time()
    atoms = sample_atoms(w)
    (pS, pH, pL), nrow = orows.region_patterns(w, atoms)
    ro = orows.RowOracle(w, ost.synth_blocks(w, "S", *pS), ost.synth_blocks(w, "H", *pH),
                         test_L_blocks(w, pL), pS, pH, pL)
    print(f"set-up {time.time() - t0:.1f}s ({nrow} of {w.n} rows in reach)", flush=True)
    out = {"atoms": np.array(atoms), "e": [], "n": []}
    for i in atoms:
        e, nn, Gb, Fb, cols = ro.row(i)
        out["e"].append(e)
        out["n"].append(nn)
        out[f"G_{i}"], out[f"F_{i}"], out[f"cols_{i}"] = Gb, Fb, cols
        print(f"atom {i} (nfun {w.nfun[i]}) {time.time() - t0:.1f}s", flush=True)
    out["e"], out["n"] = np.array(out["e"]), np.array(out["n"])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}_rows.npz")
    np.savez_compressed(path, **out)
    print("wrote", path, flush=True)


CG_ROW_ATOMS = (0, 1365, 2730, 4095)
CG_ROW_ITERS = (0, 4, 9)


def cgtraj_main(name, steps):
    from oracle import pm as opm
    w = W.get(name)
    here = os.path.dirname(os.path.abspath(__file__))
    jpath = os.path.join(here, f"{name}_cg.json")
    npath = os.path.join(here, f"{name}_cg_rows.npz")
    t0 = time.time()
    sy = ost.System(w)
    T = olnv.hotelling(sy.S, sy.maskL, 16)
    print(f"system + metric {time.time() - t0:.1f}s", flush=True)
    K, pm_hist, info = opm.purify(sy.S, sy.H, T, sy.maskL, w.n_elec, 60)
    print(f"purification: {len(pm_hist)} entries {time.time() - t0:.1f}s", flush=True)
    out = {"workload": name, "n_atoms": w.n, "metric": "hotelling 16", "start": "purify 60",
           "pm_steps": len(pm_hist), "pm_lambda": info["lam"], "cg": [],
           "row_atoms": [a for a in CG_ROW_ATOMS if a < w.n], "row_iters": list(CG_ROW_ITERS)}
    rows = {}
    off = ost.offsets(w.nfun)
    rp, col = ost.neighbours(w.pos, w.box, w.R_L)

    def save():
        out["seconds"] = time.time() - t0
        with open(jpath + ".tmp", "w") as f:
            json.dump(out, f, indent=1)
        os.replace(jpath + ".tmp", jpath)
        if rows:
            np.savez_compressed(npath + ".tmp.npz", **rows)
            os.replace(npath + ".tmp.npz", npath)

    def callback(h, G, F):
        out["cg"].append({k: h[k] for k in ("k", "E", "N", "mu", "beta", "alpha", "delta",
                                            "gnorm", "N_after_step")})
        if h["k"] in CG_ROW_ITERS:
            for a in out["row_atoms"]:
                cols = col[rp[a]:rp[a + 1]]
                r = slice(off[a], off[a + 1])
                rows[f"G_{h['k']}_{a}"] = np.stack([G[r, off[j]:off[j + 1]] for j in cols])
                rows[f"F_{h['k']}_{a}"] = np.stack([F[r, off[j]:off[j + 1]] for j in cols])
                rows[f"cols_{a}"] = cols
        save()
        print(h["k"], h["E"] / w.n, h["alpha"], h["delta"], f"{time.time() - t0:.0f}s", flush=True)

    olnv.cg(sy.S, sy.H, sy.maskL, w.n_elec, steps, L0=K, T=T, callback=callback)
    print("wrote", jpath, npath, flush=True)


def main():
    if len(sys.argv) > 2 and sys.argv[1] == "rows":
        return rows_main(sys.argv[2])
    if len(sys.argv) > 2 and sys.argv[1] == "cgtraj":
        return cgtraj_main(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 10)
    name = sys.argv[1] if len(sys.argv) > 1 else "si4096_4x4"
    steps = int(sys.argv[2]) if len(sys.argv) > 2 else 2
    w = W.get(name)
    t0 = time.time()
    sy = ost.System(w)
    print(f"system {time.time() - t0:.1f}s", flush=True)
    L0, lam = olnv.initial_L(sy.S, sy.maskL, w.n_elec)
    E, N, G, F = olnv.evaluate(L0, sy.S, sy.H, sy.maskL)
    print(f"eval {time.time() - t0:.1f}s E/atom {E / w.n:.15f} N {N:.12f}", flush=True)
    out = {"workload": name, "n_atoms": w.n, "lambda": lam, "E0": E, "N0": N,
           "G0_fro": float(np.sqrt(np.sum(G * G))), "F0_fro": float(np.sqrt(np.sum(F * F))),
           "cg": []}
    del G, F
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name}.json")
    if steps > 0:
        _, hist = olnv.cg(sy.S, sy.H, sy.maskL, w.n_elec, steps, L0=L0)
        for h in hist:
            out["cg"].append({k: h[k] for k in ("k", "E", "N", "mu", "beta", "alpha", "delta",
                                                "gnorm", "N_after_step")})
            print(h["k"], h["E"] / w.n, h["alpha"], h["delta"], flush=True)
    out["seconds"] = time.time() - t0
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
