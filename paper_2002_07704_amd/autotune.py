"""Work-decomposition autotuner for the block multiply.

The multiply's one tunable is the row-cluster shape of its output-stationary
work decomposition (4-row clusters, one lane per output column, or one row
per wavefront), and, for
cells whose atoms all carry 13 support functions (4 stored rows each), the
atom-tile shapes that multiply whole 16x16 atom tiles on the matrix cores.
Which one is fastest depends on the register budget of the value type, the
arithmetic mode and on how similar the rows of a cluster are (the cluster's
contraction list is the union of its rows'), so the tuner times a full
evaluation with each candidate on the actual system and keeps the fastest.
Results are cached per pattern signature and accumulation mode for the life
of the process.
"""
from __future__ import annotations

import time

import torch

CANDIDATES = ((4, 1), None)
_CACHE: dict = {}


def signature(system, mixed, acc=0):
    return (system.n_rows, system.pL.nnzb, system.pS.nnzb, system.pH.nnzb, bool(mixed),
            int(acc))


def tune(system, candidates=None, reps=3, mixed=False, acc=0):
    """Time one evaluation (FP64, or mixed precision) per cluster shape
    (default: the row clusters plus the system's atom-tile shapes), leave the
    system on the fastest; returns (shape, {shape: ms}).  acc: the FP32
    accumulation mode the caller has set (lnv_set_f32_accumulation), part of
    the cache key."""
    if candidates is None:
        candidates = CANDIDATES + system.tile_shapes()
    key = signature(system, mixed, acc)
    if key in _CACHE:
        best, res = _CACHE[key]
        system.set_cluster(best)
        return best, res
    if mixed:
        system.mixed_setup()
    fn = system.eval_mixed if mixed else system.eval
    res = {}
    for shape in candidates:
        system.set_cluster(shape)
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        res[shape] = (time.perf_counter() - t0) * 1e3 / reps
    best = min(res, key=res.get)
    system.set_cluster(best)
    _CACHE[key] = (best, res)
    return best, res
