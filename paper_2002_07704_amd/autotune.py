"""Work-decomposition autotuner for the block multiply.

The multiply's one tunable is the row-cluster shape of its output-stationary
work decomposition (how many output rows a wavefront accumulates per
gathered right-operand block, and how many lanes share a column).  Which one
is fastest depends on the register budget of the value type and on how
similar the rows of a cluster are (the cluster's contraction list is the
union of its rows'), so the tuner times a full evaluation with each
candidate on the actual system and keeps the fastest.  Results are cached per
pattern signature for the life of the process.
"""
from __future__ import annotations

import time

import torch

CANDIDATES = ((4, 1), (8, 2), None)
_CACHE: dict = {}


def signature(system, mixed):
    return (system.n_rows, system.pL.nnzb, system.pS.nnzb, system.pH.nnzb, bool(mixed))


def tune(system, candidates=CANDIDATES, reps=3, mixed=False):
    """Time one evaluation (FP64, or mixed precision) per cluster shape, leave
    the system on the fastest; returns (shape, {shape: ms})."""
    key = signature(system, mixed)
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
