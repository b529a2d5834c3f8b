"""Write the stored expected values of the at-scale parity tests.

Calls only `oracle/` (dense FP64 numpy) and `lnv_workloads`; nothing here
reads any GPU result.  The 4096-atom cell (16384 orbitals) needs ~25 GB of
RAM and tens of minutes on 8 cores per CG step, which is why its values are
stored instead of recomputed inside the GPU tests.

usage: python tests/golden/make_golden.py si4096_4x4 [n_cg_steps]
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


def main():
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
