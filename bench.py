"""Benchmark of the LNV hot path on one MI355X.

Headline workload (the largest configuration, the one the FP64-vs-mixed
metric is about): 32768-atom periodic diamond-Si cell (16x16x16 conventional
cubes, a = 10.26 bohr, +-0.1 bohr seeded displacements), 13 support
functions per atom stored as 4 rows of 4 (16x16 padded atom tiles, 425984
orbitals, 131072 block rows), ranges S/H/L = 12/14/10 bohr, H.L.S and
S.L.S formed within R_S + 2 R_L = 32 bohr (every entry that the products
onto L's range read), rows in groups of four bonded atoms.  Set-up per geometry
(not timed): neighbour lists, synthetic S and H, symbolic products, spatial
index, Hotelling metric, canonical-purification start.  One step = one
energy + gradient evaluation at that L: E, N, G = dE/dL and F = dN/dL from
the six block-sparse products (S.L, H.L.S and the half of S.L.S within 32
bohr; L-restricted S.L.S.L.H, halves of S.L.H.L.S and S.L.S.L.S) on the
atom tiles and their FP64 assembly and traces.  `value` is FP64 evaluations
per second (FP64 matrix-core tiles); the same evaluation with FP32 MFMA and
with the FP16 hi/lo split is timed beside it, with its energy, electron
number and gradient errors against the FP64 evaluation at the same L (the
1e-6 Ha/atom gate).  The system is "lean" (no stored L.S and X^T, FP32
intermediates in the FP64 ones' memory): both orientations of the
intermediates would not fit in the GPU's memory.

`si4096_cg` reports the 4096-atom, 4-function cell (the plain-FP64 workload
"one evaluation plus 10 CG steps"): consecutive CG iterations from the
purified start (evaluation, metric, projection, PR+ direction, exact cubic
line minimisation, electron-number correction), its evaluation alone, the
mixed-precision evaluation and CG, the adjoint; `other_configs` the
amorphous Si/O/H cell and the batch of 32 cells.

Inputs are resident in HBM before every timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "LNV energy+grad evals/s & block-sparse GFLOP/s, FP64 vs mixed at 1e-6 Ha/atom"
PEAK_FP64 = 78.6e12       # MI355X FP64 vector = FP64 matrix peak, FLOP/s
PEAK_FP32_MFMA = 157.3e12  # dense FP32 matrix peak
PEAK_FP16_MFMA = 2.5e15   # dense FP16 matrix peak
PEAK_HBM = 8.0e12         # bytes/s
HEADLINE = "si32768_13f"
CG_WORKLOAD = "si4096_4x4"


def host_info():
    """Cores this process may use and the CPU model."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, model


def cpu_baseline_rows(name, budget_s=25.0):
    """The row-wise oracle, as it stands, on sampled atom rows of the
    workload, with every host core (BLAS threads); scaled to whole
    evaluations per second.  The oracle's matrices hold the rows within
    reach of the sample (oracle/rows.py region_patterns; set-up not timed),
    which makes each sampled row cheaper than a row of a full evaluation,
    whose chains run over the full matrices: the rate is an upper bound of
    the oracle's."""
    import dataclasses

    import lnv_workloads as W
    from oracle import rows as orows
    from oracle import structure as ost
    w = W.get(name)
    atoms = [0, w.n // 3, (2 * w.n) // 3]
    t0 = time.perf_counter()
    (pS, pH, pL), nrow = orows.region_patterns(w, atoms)
    w2 = dataclasses.replace(w, seed=w.seed + 1000, R_S=w.R_L)
    ro = orows.RowOracle(w, ost.synth_blocks(w, "S", *pS), ost.synth_blocks(w, "H", *pH),
                         0.1 * ost.synth_blocks(w2, "S", *pL), pS, pH, pL)
    setup = time.perf_counter() - t0
    done = 0
    t0 = time.perf_counter()
    for i in atoms:
        ro.row(int(i))
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    per_row = (time.perf_counter() - t0) / done
    _, model = host_info()
    return {"value": 1.0 / (per_row * w.n), "unit": "evals/s", "cores": baseline_threads(),
            "kind": "oracle",
            "cpu": model,
            "sample": f"{done} atom rows of one evaluation of {name} (row-wise oracle, "
                      f"{per_row:.2f} s/row, matrices holding the {nrow} rows within reach of "
                      f"the sample; set-up {setup:.0f} s not timed), scaled by {w.n}/{done}"}


def baseline_threads():
    """Host cores for the CPU baseline: all but two, which stay with the
    process that feeds the GPU while the baseline runs beside it."""
    cores, _ = host_info()
    return max(1, cores - 2)


def start_cpu_baseline(name):
    """The CPU baseline in a child process at low priority, beside the GPU
    work (it touches no GPU)."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = str(baseline_threads())
    env["HIP_VISIBLE_DEVICES"] = ""
    return subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only",
                             name], stdout=subprocess.PIPE, stderr=subprocess.PIPE, env=env,
                            text=True, preexec_fn=lambda: os.nice(10))


def finish_cpu_baseline(proc, timeout=600):
    try:
        out, err = proc.communicate(timeout=timeout)
    except subprocess.TimeoutExpired:
        proc.kill()
        proc.communicate()
        return None
    for line in out.splitlines()[::-1]:
        if line.startswith("{"):
            return json.loads(line)
    sys.stderr.write(err[-2000:])
    return None


# ------------------------------------------------------------------ traffic records
KERNEL_SRC = [os.path.join(ROOT, "paper_2002_07704_amd", "csrc", f)
              for f in ("multiply.hip", "lnv_core.hip", "internal.h")]
COPY_BYTES = 1 << 30


def kernel_hash():
    import hashlib
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(path, key, row_order):
    """HBM bytes per launch of the multiply from profiles/traffic.json when
    they were taken on the current kernel sources and row layout (else
    None: stale counters are not reported)."""
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            tj = json.load(f).get(key)
        if (tj and tj.get("kernel_src_sha256_16") == kernel_hash()
                and tj.get("row_order", "atoms") == row_order):
            return tj
    except (OSError, ValueError, KeyError):
        return None
    return None


def summarize_pmc(fetch_dir, write_dir, out_path, key, kernel, row_order):
    """Per-launch HBM bytes of the multiply kernel (name contains `kernel`)
    from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE, KiB per dispatch),
    each scaled by what the same counter reads for the device copy of
    COPY_BYTES bytes made by --pmc-probe, over the dispatches after it."""
    import csv
    import glob

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        per = {}
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            k = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            per[k] = per.get(k, 0.0) + float(r["Counter_Value"]) * 1024.0
        return per

    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = load(d, counter)
        copies = [(i, v) for (i, n), v in per.items() if "copyBuffer" in n and v > 0.4 * COPY_BYTES]
        if not copies:
            raise SystemExit(f"no calibration copy found in {d}")
        # the calibration copy is the last large copy before the timed work
        copy_id, copy_v = max(copies, key=lambda x: x[0])
        factor = COPY_BYTES / copy_v
        mul = [v for (i, n), v in per.items() if kernel in n and i > copy_id]
        out[counter] = {"factor": factor, "launches": len(mul),
                        "bytes_per_launch": factor * sum(mul) / max(1, len(mul))}
    res = {}
    if os.path.exists(out_path):
        res = json.load(open(out_path))
    res[key] = {
        "kernel": kernel, "kernel_src_sha256_16": kernel_hash(), "row_order": row_order,
        "fetch_bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"],
        "write_bytes_per_launch": out["WRITE_SIZE"]["bytes_per_launch"],
        "bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"],
        "calibration": {"copy_bytes": COPY_BYTES, "fetch_factor": out["FETCH_SIZE"]["factor"],
                        "write_factor": out["WRITE_SIZE"]["factor"]},
        "launches": out["FETCH_SIZE"]["launches"],
    }
    with open(out_path, "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res[key]))


def roofline(kernel, flops, ms_total, launches, peak, unit_peak, traffic_rec):
    """Roofline object of the dominant kernel: achieved algorithmic FLOP/s of
    its launches (HIP events) against the compute peak; with a current
    traffic record, the calibrated HBM bytes per launch against 8 TB/s, and
    the bound is whichever fraction is larger."""
    achieved = flops / (ms_total * 1e-3)
    avg_ms = ms_total / max(1, launches)
    frac = achieved / peak
    traffic = traffic_rec["bytes_per_launch"] if traffic_rec else None
    hbm_frac = traffic / (avg_ms * 1e-3) / PEAK_HBM if traffic else None
    bound = unit_peak
    if hbm_frac is not None and hbm_frac > frac:
        bound = "hbm"
    return {"kernel": kernel, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": frac, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "hbm_GBps": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
            "hbm_frac": hbm_frac, "avg_launch_ms": avg_ms, "launches": launches,
            "flops_per_launch": flops / max(1, launches)}


def event_timed(lib, fn, reps):
    """Run fn reps times with HIP events around every multiply launch;
    (summed kernel ms, launches)."""
    import ctypes

    import torch
    torch.cuda.synchronize()
    lib.lnv_timing_reset()
    lib.lnv_timing_enable(1)
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    lib.lnv_timing_enable(0)
    ms_tot = ctypes.c_double(0.0)
    launches = ctypes.c_int64(0)
    st = lib.lnv_timing_read(ctypes.byref(ms_tot), ctypes.byref(launches))
    if st != 0:
        raise RuntimeError(f"lnv_timing_read failed ({st})")
    return ms_tot.value, launches.value


def wall_timed(fn, reps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / reps


# ------------------------------------------------------------------ headline
def build_headline():
    """The 32768-atom 13-function cell on the atom tiles (16, 4), lean, rows
    in bonded groups, purified start; (system, set-up s, purification info)."""
    import torch

    import lnv_workloads as W
    from paper_2002_07704_amd.pm import pm_initial_L
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get(HEADLINE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s = LNVSystem(w, reorder="bonds", metric="hotelling", lean=True, cluster=None)
    s.set_cluster((16, 4))
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    pm_hist, _ = pm_initial_L(s, 60)
    torch.cuda.synchronize()
    return s, setup, {"steps": len(pm_hist), "s": time.perf_counter() - t0}


def headline_shape(s, acc):
    """Atom-tile shape of the headline cell for an arithmetic (acc -1 FP64,
    else the FP32 accumulation mode, which the caller has set): 4 x 4 tiles
    per wave (16, 4) or 4 x 2 (16, 8), whichever evaluates faster; (shape,
    {shape: ms})."""
    from paper_2002_07704_amd import autotune
    shp, tried = autotune.tune(s, candidates=s.tile_shapes(), reps=2, mixed=acc >= 0,
                               acc=max(acc, 0))
    return shp, {str(k): v for k, v in tried.items()}


def bench_headline(args, lib):
    import torch

    from paper_2002_07704_amd import lib as L_
    s, setup_s, pm = build_headline()
    w = s.w
    torch.cuda.reset_peak_memory_stats()
    f_alg, f_pad = s.flops("eval"), s.flops("eval", padded=True)
    # atom-tile shape per arithmetic (timed here, outside the timed steps)
    shapes = {}
    shape64, tried = headline_shape(s, -1)
    shapes["f64"] = {"shape": str(shape64), "eval_ms": tried}
    for _ in range(args.warmup):
        s.eval()
    ms64 = wall_timed(s.eval, args.steps)
    E64, N64 = (float(x) for x in s.EN.cpu())
    G64, F64 = s.G.val.clone(), s.F.val.clone()
    ms_k, nl = event_timed(lib, s.eval, args.steps)
    rl64 = roofline("k_tile16 (16x16 atom tiles, FP64 MFMA v_mfma_f64_16x16x4_f64; the six "
                    "multiply launches of each timed evaluation)", args.steps * f_alg, ms_k, nl,
                    PEAK_FP64, "mfma", traffic_record(args.traffic_json, f"{HEADLINE}:f64:{shape64}",
                                                 "bonds"))
    rl64["padded_tflops"] = args.steps * f_pad / (ms_k * 1e-3) / 1e12
    s.mixed_setup()
    mixed = {}
    modes = ((0, "fp32_mfma", PEAK_FP32_MFMA, 1), (2, "fp16_hilo_mfma", PEAK_FP16_MFMA, 3))
    for acc, label, peak, mult in modes:
        L_.call("lnv_set_f32_accumulation", acc)
        try:
            shp, tried = headline_shape(s, acc)
            shapes[label] = {"shape": str(shp), "eval_ms": tried}
            for _ in range(max(1, args.warmup)):
                s.eval_mixed()
            ms = wall_timed(s.eval_mixed, args.steps)
            E, N = (float(x) for x in s.EN.cpu())
            dG = float(torch.linalg.vector_norm(s.G.val - G64) / torch.linalg.vector_norm(G64))
            dF = float(torch.linalg.vector_norm(s.F.val - F64) / torch.linalg.vector_norm(F64))
            msk, nlk = event_timed(lib, s.eval_mixed, args.steps)
        finally:
            L_.call("lnv_set_f32_accumulation", 0)
        rl = roofline(f"k_tile16 ({label})", args.steps * f_alg, msk, nlk, peak, "mfma",
                      traffic_record(args.traffic_json, f"{HEADLINE}:{label}:{shp}", "bonds"))
        # matrix-core utilisation: padded tile flops (x3 for the hi/lo split's
        # three products) against the mode's matrix peak
        rl["mfma_util"] = mult * args.steps * f_pad / (msk * 1e-3) / peak
        mixed[label] = {"evals_per_s": 1e3 / ms, "ms": ms,
                        "gflops_per_s": f_alg / (ms * 1e-3) / 1e9,
                        "speedup_vs_fp64_eval": ms64 / ms,
                        "dE_per_atom": abs(E - E64) / w.n, "dN_rel": abs(N - N64) / N64,
                        "dG_rel": dG, "dF_rel": dF,
                        "within_1e-6_Ha_per_atom": abs(E - E64) / w.n <= 1e-6,
                        "tile_shape": str(shp), "roofline": rl}
    rl64["mfma_util"] = args.steps * f_pad / (ms_k * 1e-3) / PEAK_FP64
    out = {
        "metric": METRIC,
        "value": 1e3 / ms64,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms64,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {w.n}-atom diamond Si (16x16x16 cubes), 13 support "
                        f"functions/atom as 16x16 padded atom tiles ({w.n_orb} orbitals, "
                        f"{s.n_rows} block rows), R_S/R_H/R_L {w.R_S:g}/{w.R_H:g}/{w.R_L:g} "
                        f"bohr, H.L.S and S.L.S within R_S + 2 R_L",
            "step": "one energy+gradient evaluation (E, N, G = dE/dL, F = dN/dL: six block-sparse "
                    "products on the FP64 atom tiles, FP64 assembly and traces) at the purified L",
            "row_order": "bonds", "tile_shape": str(shape64), "lean": True,
            "metric_T": "Hotelling T ~ S^-1 on L's range (16 steps, set-up)",
            "start": f"canonical purification, {pm['steps']} steps, {pm['s']:.1f} s (set-up)",
            "spatial_index_grid": list(s.ix_cells.g),
            "atoms": w.n, "n_elec": w.n_elec,
            "E_per_atom": E64 / w.n, "N": N64,
        },
        "gflop_per_eval": f_alg / 1e9,
        "gflop_per_eval_padded": f_pad / 1e9,
        "gflops_per_s": f_alg / (ms64 * 1e-3) / 1e9,
        "setup_s": setup_s,
        "tile_shapes_tried": shapes,
        "mixed": mixed,
        "peak_device_memory_GiB": torch.cuda.max_memory_allocated() / 2**30,
        "roofline": rl64,
    }
    del s, G64, F64
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------------ 4096-atom CG
def bench_cg(args, lib):
    """Consecutive CG iterations on the 4096-atom 4-function cell from the
    purified start, its evaluation alone, the mixed-precision evaluation and
    CG, the adjoint; roofline of the pipelined 4x4 multiply."""
    import math

    import torch

    import lnv_workloads as W
    from paper_2002_07704_amd import lib as L_
    from paper_2002_07704_amd.pm import pm_initial_L
    from paper_2002_07704_amd.system import LNVSystem
    w = W.get(CG_WORKLOAD)
    steps = args.cg_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sysg = LNVSystem(w, reorder=args.row_order)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    pm_hist, _ = pm_initial_L(sysg, 60)
    torch.cuda.synchronize()
    pm_s = time.perf_counter() - t0
    L_start = sysg.L.val.clone()
    sysg.eval()
    e_start = float(sysg.EN[0].item())

    def restart():
        sysg.L.val.copy_(L_start)
        sysg.cg_restart()

    restart()
    for _ in range(2):
        sysg.cg_step()
    restart()
    torch.cuda.synchronize()
    sysg.scalars[L_.SC["NCORR"]] = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        sysg.cg_step()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    status = int(sysg.scalar("STATUS"))
    n_corr = int(sysg.scalar("NCORR"))
    # the first step and every reset step form S.L and S.L.S afresh
    n_fresh = math.ceil(steps / sysg.opts.reset_period)
    flops_run = (steps * sysg.flops("step_base") + n_fresh * sysg.flops("first_extra")
                 + n_corr * sysg.flops("ncorr"))
    sysg.eval()
    torch.cuda.synchronize()
    e_end = float(sysg.EN[0])

    def cg_run():
        restart()
        for _ in range(steps):
            sysg.cg_step()

    ms_k, nl = event_timed(lib, cg_run, 1)
    rl = roofline("k_mul44c1 (pipelined 4-row clustered block SpGEMM, FP64 VALU; all multiply "
                  "launches of the timed iterations)", flops_run, ms_k, nl, PEAK_FP64, "alu",
                  traffic_record(args.traffic_json, CG_WORKLOAD, args.row_order))
    ms_eval = wall_timed(sysg.eval, args.eval_reps)
    flops_eval = sysg.flops("eval")
    # mixed precision at the L of the last FP64 step
    sysg.mixed_setup()
    sysg.eval()
    torch.cuda.synchronize()
    E64, N64 = (float(x) for x in sysg.EN.cpu())
    G64, F64 = sysg.G.val.clone(), sysg.F.val.clone()
    mixed = {}
    for acc, name in ((0, "fp32_accumulate"), (1, "fp64_accumulate")):
        L_.call("lnv_set_f32_accumulation", acc)
        sysg.eval_mixed()
        torch.cuda.synchronize()
        E32, N32 = (float(x) for x in sysg.EN.cpu())
        dG = float(torch.linalg.vector_norm(sysg.G.val - G64) / torch.linalg.vector_norm(G64))
        dF = float(torch.linalg.vector_norm(sysg.F.val - F64) / torch.linalg.vector_norm(F64))
        ms = wall_timed(sysg.eval_mixed, args.eval_reps)
        mixed[name] = {"evals_per_s": 1e3 / ms, "ms": ms,
                       "gflops_per_s": flops_eval / (ms * 1e-3) / 1e9,
                       "speedup_vs_fp64_eval": ms_eval / ms,
                       "dE_per_atom": abs(E32 - E64) / w.n, "dN_rel": abs(N32 - N64) / N64,
                       "dG_rel": dG, "dF_rel": dF,
                       "within_1e-6_Ha_per_atom": abs(E32 - E64) / w.n <= 1e-6}
    L_.call("lnv_set_f32_accumulation", 0)
    del G64, F64
    sysg.opts.mixed = True
    restart()
    sysg.cg_step()
    restart()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sysg.cg_step()
    torch.cuda.synchronize()
    ms_mcg = (time.perf_counter() - t0) * 1e3 / steps
    status_m = int(sysg.scalar("STATUS"))
    sysg.opts.mixed = False
    sysg.eval()
    torch.cuda.synchronize()
    e_mcg, n_mcg = (float(x) for x in sysg.EN.cpu())
    # adjoint at the same L
    sysg.adjoint_setup()
    dS = torch.empty_like(sysg.S.val)
    dH = torch.empty_like(sysg.H.val)
    sysg.adjoint(sysg.L.val, sysg.S.val, sysg.H.val, dS=dS, dH=dH)
    ms_adj = wall_timed(lambda: sysg.adjoint(sysg.L.val, sysg.S.val, sysg.H.val, dS=dS, dH=dH),
                        args.eval_reps)
    flops_adj = sysg.adjoint_flops()
    out = {
        "what": f"{w.name}: {w.n}-atom diamond Si, 4x4 FP64 blocks ({w.n_orb} orbitals), "
                f"R_S/R_H/R_L {w.R_S:g}/{w.R_H:g}/{w.R_L:g} bohr, Hotelling metric, purified "
                f"start ({len(pm_hist)} steps, {pm_s:.2f} s), rows {args.row_order}",
        "step": "one CG iteration: evaluation (6 products) + metric P_L(TGT), P_L(TFT) + "
                "projection + PR+ direction + exact cubic line search + electron-number "
                f"correction; {steps} consecutive iterations from the purified start",
        "cg_steps_per_s": 1e3 / ms_step, "ms_per_step": ms_step,
        "gflop_per_step": flops_run / steps / 1e9,
        "gflops_per_s": flops_run / steps / (ms_step * 1e-3) / 1e9,
        "n_corrections": n_corr, "cg_status_bits": status,
        "E_per_atom_start": e_start / w.n, "E_per_atom_after_steps": e_end / w.n,
        "setup_s": setup_s,
        "eval_only": {"evals_per_s": 1e3 / ms_eval, "ms": ms_eval, "gflop": flops_eval / 1e9,
                      "gflops_per_s": flops_eval / (ms_eval * 1e-3) / 1e9},
        "mixed": mixed,
        "mixed_cg": {"ms_per_step": ms_mcg, "steps_per_s": 1e3 / ms_mcg,
                     "speedup_vs_fp64_step": ms_step / ms_mcg,
                     "E_per_atom_after_steps": e_mcg / w.n,
                     "dE_per_atom_vs_fp64_cg": abs(e_mcg - e_end) / w.n,
                     "N_after_steps": n_mcg, "cg_status_bits": status_m},
        "adjoint_dS_dH": {"ms": ms_adj, "gflop": flops_adj / 1e9,
                          "gflops_per_s": flops_adj / (ms_adj * 1e-3) / 1e9},
        "roofline": rl,
    }
    del sysg
    torch.cuda.empty_cache()
    return out


def extra_configs(reps):
    """Evaluation rates of the amorphous Si/O/H cell (13/9/4 support
    functions, atoms split into 4x4-blocked rows) and of a batch of 32
    independent cells: FP64 and mixed-precision evaluation at L0 (for the
    batch: per-cell E and N, identity start) after the autotuner's choice of
    the multiply's shape; CG iterations of the Si/O/H cell from the
    purified start."""
    import numpy as np
    import torch

    import lnv_workloads as W
    from paper_2002_07704_amd import autotune
    from paper_2002_07704_amd.system import LNVSystem
    cells = [
        ("siOH8192_mixed", W.get("siOH8192_mixed"),
         "amorphous Si/O/H 40/40/20 %, 13/9/4 functions/atom, rho 0.0074 bohr^-3"),
        ("siOH_batch32", W.get_batch("siOH_batch32"),
         "32 independent amorphous Si/O/H cells of 64-512 atoms (13/9/4 functions), one "
         "block-diagonal system, one launch per product for all cells, every CG scalar per cell"),
    ]
    res = {}
    for name, w, what in cells:
        t0 = time.perf_counter()
        batch = isinstance(w, list)
        s = LNVSystem(w, metric="hotelling")
        s.cg_init()
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        shape, tried = autotune.tune(s)
        if batch:
            ms64 = wall_timed(s.cell_energies, reps)
            E64 = float(s.EN[0])
            s.mixed_setup()
            ms32 = wall_timed(lambda: s.cell_energies(mixed=True), reps)
        else:
            ms64 = wall_timed(s.eval, reps)
            E64 = float(s.EN[0])
            s.mixed_setup()
            ms32 = wall_timed(s.eval_mixed, reps)
        E32 = float(s.EN[0])
        f_alg, f_pad = s.flops("eval"), s.flops("eval", padded=True)
        cg = None
        if batch:
            # every cell minimised at once: per-cell mu, beta, alpha, delta in
            # the same launches, Hotelling metric, each cell purified
            from paper_2002_07704_amd.pm import pm_initial_L
            t1 = time.perf_counter()
            pm_hists, _ = pm_initial_L(s, 60)
            pm_s = time.perf_counter() - t1
            s.cg_restart()
            s.cg_step()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                s.cg_step()
            torch.cuda.synchronize()
            ms_cg = (time.perf_counter() - t1) * 1e3 / 3
            scs = s.cell_scalars_host()
            bits = [int(x["STATUS"]) for x in scs]
            cg = {"start": "canonical purification per cell (Hotelling metric per cell)",
                  "purification_steps_per_cell": [len(h) for h in pm_hists],
                  "purification_s": pm_s, "cells": len(scs),
                  "cg_step_ms": ms_cg, "cg_steps_per_s": 1e3 / ms_cg,
                  "E_per_atom_after_4_steps": sum(x["E"] for x in scs) / s.n,
                  "cells_correction_capped": sum(1 for b in bits if b & 8),
                  "status_bits_or": int(np.bitwise_or.reduce(bits))}
        else:
            from paper_2002_07704_amd.pm import pm_initial_L
            t1 = time.perf_counter()
            pm_hist, _ = pm_initial_L(s, 60)
            pm_s = time.perf_counter() - t1
            L_pm = s.L.val.clone()

            def cg_run():
                s.L.val.copy_(L_pm)
                s.cg_restart()
                s.cg_step()
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                for _ in range(3):
                    s.cg_step()
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t2) * 1e3 / 3
                st = int(s.scalar("STATUS"))
                s.eval()
                torch.cuda.synchronize()
                return ms, float(s.EN[0]), float(s.EN[1]), st

            ms_cg, e_cg, n_cg4, st_cg = cg_run()
            cg = {"purification_steps": len(pm_hist), "purification_s": pm_s,
                  "cg_step_ms": ms_cg, "cg_steps_per_s": 1e3 / ms_cg,
                  "E_per_atom_after_4_steps": e_cg / s.n,
                  "N_after_4_steps": n_cg4, "n_elec": s.n_elec, "cg_status_bits": st_cg}
            s.opts.mixed = True
            try:
                ms_m, e_m, n_m, st_m = cg_run()
            finally:
                s.opts.mixed = False
            cg["mixed"] = {"cg_step_ms": ms_m, "cg_steps_per_s": 1e3 / ms_m,
                           "speedup_vs_fp64_step": ms_cg / ms_m,
                           "E_per_atom_after_4_steps": e_m / s.n,
                           "dE_per_atom_vs_fp64_cg": abs(e_m - e_cg) / s.n,
                           "N_after_4_steps": n_m, "cg_status_bits": st_m}
        res[name] = {"what": what, "atoms": s.n,
                     "orbitals": int(sum(int(c.nfun.sum()) for c in (w if batch else [w]))),
                     "rows": s.n_rows, "setup_s": setup, "cluster_shape": str(shape),
                     "autotune_eval_ms": {str(k): v for k, v in tried.items()},
                     "eval_ms": ms64, "evals_per_s": 1e3 / ms64,
                     "gflop_algorithmic": f_alg / 1e9, "gflop_padded": f_pad / 1e9,
                     "tflops_algorithmic": f_alg / (ms64 * 1e-3) / 1e12,
                     "mixed_eval_ms": ms32, "mixed_evals_per_s": 1e3 / ms32,
                     "mixed_dE_per_atom": abs(E32 - E64) / s.n,
                     ("cg" if batch else "cg_from_purified_start"): cg}
        print(f"[bench] {name}: {json.dumps(res[name])}", file=sys.stderr, flush=True)
        del s
        torch.cuda.empty_cache()
    return res


def profile_headline(acc, reps=3):
    """The headline cell (set-up and purification as benchmarked) and reps
    evaluations: acc -1 FP64 tiles, 0 FP32 MFMA, 2 FP16 hi/lo (a short
    program for rocprofv3)."""
    import torch

    from paper_2002_07704_amd import lib as L_
    s, _, _ = build_headline()
    if acc >= 0:
        s.mixed_setup()
        L_.call("lnv_set_f32_accumulation", acc)
    shp, _ = headline_shape(s, acc)
    torch.cuda.synchronize()
    print(json.dumps({"profile_headline": acc, "tile_shape": str(shp), "reps": reps}), flush=True)
    for _ in range(reps):
        s.eval_mixed() if acc >= 0 else s.eval()
    torch.cuda.synchronize()
    L_.call("lnv_set_f32_accumulation", 0)
    print(json.dumps({"profile_headline": acc, "E": float(s.EN[0]), "N": float(s.EN[1])}),
          flush=True)


def pmc_probe(args, acc):
    """Counter program: the workload's set-up, a COPY_BYTES device copy (the
    calibration), then the timed work only (headline: evaluations in the
    given arithmetic; si4096_4x4: CG iterations)."""
    import torch

    from paper_2002_07704_amd import lib as L_
    if args.workload == HEADLINE:
        s, _, _ = build_headline()
        if acc >= 0:
            s.mixed_setup()
            L_.call("lnv_set_f32_accumulation", acc)
        shp, _ = headline_shape(s, acc)
        print(json.dumps({"pmc_probe_tile_shape": str(shp)}), flush=True)
        fn = s.eval_mixed if acc >= 0 else s.eval
        fn()
    else:
        import lnv_workloads as W
        from paper_2002_07704_amd.pm import pm_initial_L
        from paper_2002_07704_amd.system import LNVSystem
        s = LNVSystem(W.get(args.workload), reorder=args.row_order)
        pm_initial_L(s, 60)
        s.cg_restart()
        fn = s.cg_step
    torch.cuda.synchronize()
    a = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b
    for _ in range(args.steps):
        fn()
    torch.cuda.synchronize()
    L_.call("lnv_set_f32_accumulation", 0)
    print(json.dumps({"pmc_probe": args.workload, "acc": acc, "steps": args.steps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed evaluations of the headline cell (per arithmetic mode)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cg-steps", type=int, default=10,
                    help="consecutive CG iterations timed on the 4096-atom cell")
    ap.add_argument("--row-order", default="bonds", choices=("bonds", "cell", "atoms"),
                    help="row order of the 4096-atom cell (bonds: groups of four bonded atoms)")
    ap.add_argument("--eval-reps", type=int, default=10)
    ap.add_argument("--workload", default=HEADLINE, help="workload of --pmc-probe")
    ap.add_argument("--acc", type=int, default=-1,
                    help="--pmc-probe / --profile arithmetic: -1 FP64, 0 FP32 MFMA, 2 FP16 hi/lo")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cg", action="store_true", help="skip the 4096-atom CG workload")
    ap.add_argument("--no-extra-configs", action="store_true",
                    help="skip the Si/O/H cell and the batch of 32 cells")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"))
    ap.add_argument("--pmc-probe", action="store_true")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "KEY", "KERNEL"))
    ap.add_argument("--profile", action="store_true",
                    help="only the headline cell's set-up and 3 evaluations (for rocprofv3)")
    ap.add_argument("--cpu-baseline-only", metavar="WORKLOAD")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_rows(args.cpu_baseline_only)), flush=True)
        return
    if args.summarize_pmc:
        fd, wd, key, kern = args.summarize_pmc
        summarize_pmc(fd, wd, args.traffic_json, key, kern, args.row_order)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library drives one device per process "
              "and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.profile:
        profile_headline(args.acc)
        return
    if args.pmc_probe:
        pmc_probe(args, args.acc)
        return

    import torch

    from paper_2002_07704_amd import lib as L_
    lib = L_.load()
    out = bench_headline(args, lib)
    print(f"[bench] headline: {out['value']:.3f} evals/s", file=sys.stderr, flush=True)
    # the CPU baseline runs beside the secondary workloads, so that its host
    # load cannot reach the headline's timed evaluations
    cpu = None if args.no_cpu_baseline else start_cpu_baseline(HEADLINE)
    if not args.no_cg:
        out["si4096_cg"] = bench_cg(args, lib)
        print(f"[bench] si4096_cg: {out['si4096_cg']['cg_steps_per_s']:.2f} CG steps/s",
              file=sys.stderr, flush=True)
    if not args.no_extra_configs:
        out["other_configs"] = extra_configs(args.eval_reps)
    if cpu is not None:
        cb = finish_cpu_baseline(cpu)
        if cb is not None:
            out["cpu_baseline"] = cb
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
