"""ctypes binding of liblnv.so (the C ABI declared in include/lnv.h).

Argument marshalling only: every computation happens in the HIP kernels of
the library.  `load()` fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblnv.so")

# status codes (lnv_status)
OK, EINVAL, ECAPACITY, EPATTERN, EHIP, ENUMERIC, EUNSUPPORTED = range(7)
F64 = 0
F32 = 1
DOT_PARTIALS = 1024
NOALLOC_PARTIALS = 1 << 19
NSLOTS = 12

# device scalar block indices (LNV_SC_*)
SC = dict(E=0, N=1, MU=2, BETA=3, ALPHA=4, DELTA=5, FF=6, GG=7, C1=8, C2=9, C3=10,
          N0=11, N1=12, N2=13, N3=14, FORCE_RESET=15, SKIP_NCORR=16, GNORM=17,
          N_AFTER=18, LAMBDA=19, STATUS=20, LL=21, GF=22, DF=23, FCFC=32, SIGMA=33, GGN=34, NCORR=35,
          E_PREV=36, RISES=37, GUARD_K=38, OCC_MIN=39, OCC_MAX=40)
NSCALARS = 48
ST_NONFINITE, ST_NO_ALPHA, ST_NO_DELTA, ST_DELTA_CAPPED = 1, 2, 4, 8
ST_GUARD, ST_RUNAWAY = 16, 32


class LnvIndex(ctypes.Structure):
    _fields_ = [("tab", c_void_p), ("cell", c_void_p), ("slot", c_void_p),
                ("g", c_int32 * 3), ("r", c_int32 * 3), ("w", c_int32 * 3),
                ("occ", c_int32), ("qs", c_int32), ("stride", c_int64)]


class LnvPattern(ctypes.Structure):
    _fields_ = [("n", c_int32), ("n_items", c_int32), ("nnzb", c_int64),
                ("row_ptr", c_void_p), ("col", c_void_p), ("ix", LnvIndex),
                ("items", c_void_p),
                ("cl_m", c_int32), ("cl_g", c_int32), ("n_cl_items", c_int32), ("tile4", c_int32),
                ("cl_ptr", c_void_p), ("cl_col", c_void_p), ("cl_pos", c_void_p),
                ("cl_items", c_void_p), ("cl_cell", c_void_p)]


class LnvBsm(ctypes.Structure):
    _fields_ = [("pat", POINTER(LnvPattern)), ("blk", c_int32), ("dtype", c_int32),
                ("val", c_void_p)]


class LnvEvalWs(ctypes.Structure):
    _fields_ = [("SL", LnvBsm), ("LS", LnvBsm), ("X", LnvBsm), ("XT", LnvBsm), ("Z", LnvBsm),
                ("perm_SL", c_void_p), ("perm_X", c_void_p), ("YT", c_void_p),
                ("W", c_void_p), ("V", c_void_p), ("partials", c_void_p),
                ("partials_len", c_int64), ("scalars", c_void_p), ("Zu", LnvBsm), ("Lu", LnvBsm),
                ("Vu", c_void_p), ("carry", c_int32)]


class LnvCgWs(ctypes.Structure):
    _fields_ = [("ev", LnvEvalWs), ("LL", LnvBsm), ("SL2", c_void_p), ("Hp", c_void_p),
                ("G", c_void_p), ("F", c_void_p), ("Gc", c_void_p), ("Fc", c_void_p),
                ("g", c_void_p), ("gc", c_void_p), ("gc_prev", c_void_p), ("D", c_void_p),
                ("D_prev", c_void_p), ("lanczos", c_void_p)]


class LnvEval32Ws(ctypes.Structure):
    _fields_ = [("L", LnvBsm), ("S", LnvBsm), ("H", LnvBsm), ("SL", LnvBsm), ("LS", LnvBsm),
                ("X", LnvBsm), ("XT", LnvBsm), ("Z", LnvBsm), ("perm_SL", c_void_p),
                ("perm_X", c_void_p), ("YT", c_void_p), ("W", c_void_p), ("V", c_void_p),
                ("partials", c_void_p), ("partials_len", c_int64), ("scalars", c_void_p),
                ("Zu", LnvBsm), ("Lu", LnvBsm), ("Vu", c_void_p)]


class LnvAdjWs(ctypes.Structure):
    _fields_ = [("SL", LnvBsm), ("LSL", LnvBsm), ("HL", LnvBsm), ("YS", c_void_p),
                ("LSLu", LnvBsm), ("Hu", LnvBsm), ("Su", LnvBsm),
                ("LS", LnvBsm), ("perm_SL", c_void_p), ("LH", LnvBsm), ("perm_HL", c_void_p)]


class LnvOpts(ctypes.Structure):
    _fields_ = [("reset_period", c_int32), ("n_tol", c_double), ("step_cap", c_double),
                ("eval32", c_void_p), ("occ_every", c_int32), ("occ_iter", c_int32)]


class LnvAtoms(ctypes.Structure):
    _fields_ = [("n_atoms", c_int32), ("n_rows", c_int32), ("nfun", c_void_p),
                ("row_start", c_void_p), ("atom_of", c_void_p), ("off_of", c_void_p)]


class LnvVbsm(ctypes.Structure):
    _fields_ = [("atoms", POINTER(LnvAtoms)), ("row_ptr", c_void_p), ("col", c_void_p),
                ("val_off", c_void_p), ("nnz", c_int64), ("dtype", c_int32), ("val", c_void_p)]


class LnvBatch(ctypes.Structure):
    _fields_ = [("n_cells", c_int32), ("item_ptr", c_void_p), ("val_ptr", c_void_p),
                ("row_cell", c_void_p), ("n_elec", c_void_p), ("scalars", c_void_p),
                ("row_off", c_void_p), ("n_orb", c_void_p)]


class LnvPmWs(ctypes.Structure):
    _fields_ = [("SK", LnvBsm), ("K2", c_void_p), ("K3", c_void_p), ("KT", c_void_p),
                ("perm_L", c_void_p), ("partials", c_void_p), ("partials_len", c_int64),
                ("scalars", c_void_p), ("hist", c_void_p), ("hist_len", c_int32)]


PM = dict(MU=0, B=1, LAMBDA=2, STOPPED=11, STEPS=12)
PM_NSCALARS = 32

PPat = POINTER(LnvPattern)
PBsm = POINTER(LnvBsm)
PAtoms = POINTER(LnvAtoms)
PVbsm = POINTER(LnvVbsm)

# name -> (restype, argtypes); the exported symbols of include/lnv.h
SIGNATURES = {
    "lnv_strerror": (c_char_p, [c_int]),
    "lnv_last_hip_error": (c_int, []),
    "lnv_sync_check": (c_int, [c_void_p]),
    "lnv_cg_check": (c_int, [c_void_p, POINTER(c_int32), c_void_p]),
    "lnv_lanczos_len": (c_int64, [c_int32]),
    "lnv_occupation_bounds": (c_int, [PBsm, PBsm, c_int32, c_void_p, c_void_p, c_void_p]),
    "lnv_neighbours": (c_int, [c_void_p, c_int32, POINTER(c_double), c_double, c_void_p,
                               c_void_p, c_int64, POINTER(c_int64), c_void_p]),
    "lnv_pattern_product": (c_int, [PPat, PPat, PPat, c_void_p, c_void_p, c_int64,
                                    POINTER(c_int64), c_void_p, POINTER(c_int64), c_void_p]),
    "lnv_cells": (c_int, [c_void_p, c_int32, POINTER(c_double), POINTER(c_int32),
                          POINTER(c_double), c_void_p, c_void_p, POINTER(c_int32), c_void_p]),
    "lnv_pattern_index": (c_int, [PPat, c_void_p, c_void_p, POINTER(c_int32), c_int32, c_int32,
                                  c_void_p, c_int64, POINTER(c_int64), c_void_p]),
    "lnv_pattern_half": (c_int, [PPat, c_void_p, c_void_p, c_int64, POINTER(c_int64), c_void_p]),
    "lnv_pattern_flops": (c_int, [PPat, PPat, PPat, c_void_p, POINTER(c_int64), c_void_p]),
    "lnv_pattern_items": (c_int, [PPat, c_void_p, c_int64, POINTER(c_int32), c_void_p]),
    "lnv_pattern_transpose_map": (c_int, [PPat, PPat, c_void_p, c_void_p]),
    "lnv_pattern_cluster": (c_int, [PPat, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                    c_void_p, c_int64, c_void_p, c_int64, POINTER(c_int64),
                                    POINTER(c_int32), c_void_p]),
    "lnv_pattern_tile4": (c_int, [PPat, POINTER(c_int32), c_void_p]),
    "lnv_bsm_transpose": (c_int, [PBsm, c_void_p, PBsm, c_void_p]),
    "lnv_atoms_layout": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_int64, POINTER(c_int32), c_void_p]),
    "lnv_atoms_rows": (c_int, [PAtoms, c_void_p, c_void_p, c_void_p]),
    "lnv_vbsm_offsets": (c_int, [PAtoms, c_void_p, c_void_p, c_int64, c_void_p,
                                 POINTER(c_int64), c_void_p]),
    "lnv_vbsm_pack": (c_int, [PVbsm, PBsm, c_void_p]),
    "lnv_vbsm_unpack": (c_int, [PBsm, PVbsm, c_void_p]),
    "lnv_multiply_ws_bytes": (c_int, [PBsm, PBsm, c_int32, PBsm, c_int32, POINTER(c_int64)]),
    "lnv_synth_blocks": (c_int, [c_void_p, POINTER(c_double), c_void_p, c_void_p, c_void_p, PBsm,
                                 c_int32, c_double, c_double, c_uint64, c_double, c_void_p]),
    "lnv_bsm_multiply": (c_int, [c_double, PBsm, PBsm, c_int32, c_double, PBsm, c_void_p]),
    "lnv_bsm_multiply_dot": (c_int, [c_double, PBsm, PBsm, c_int32, c_double, PBsm, c_int32,
                                     PBsm, PBsm, c_void_p, c_void_p, c_void_p]),
    "lnv_bsm_multiply_dot_noalloc": (c_int, [c_double, PBsm, PBsm, c_int32, c_double, PBsm,
                                             c_int32, PBsm, PBsm, c_void_p, c_void_p]),
    "lnv_bsm_dot": (c_int, [PBsm, PBsm, c_void_p, c_void_p, c_void_p]),
    "lnv_partials_len": (c_int64, [c_int32]),
    "lnv_eval": (c_int, [PBsm, PBsm, PBsm, PBsm, PBsm, c_void_p, POINTER(LnvEvalWs), c_void_p]),
    "lnv_eval_mixed": (c_int, [PBsm, PBsm, PBsm, PBsm, PBsm, c_void_p, POINTER(LnvEval32Ws),
                               c_void_p]),
    "lnv_bsm_convert": (c_int, [PBsm, PBsm, c_void_p]),
    "lnv_neighbours_cells": (c_int, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                     c_double, c_void_p, c_void_p, c_int64, POINTER(c_int64),
                                     c_void_p]),
    "lnv_synth_blocks_cells": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p, PBsm, c_int32, c_double, c_double, c_double,
                                       c_void_p]),
    "lnv_cell_traces": (c_int, [PPat, POINTER(LnvEvalWs), c_int32, c_void_p, c_void_p, c_void_p]),
    "lnv_adjoint": (c_int, [PBsm, PBsm, PBsm, PBsm, PBsm, PBsm, POINTER(LnvAdjWs), c_void_p]),
    "lnv_forces": (c_int, [c_void_p, POINTER(c_double), c_void_p, c_void_p, c_void_p, c_uint64,
                           c_double, PBsm, PBsm, c_double, c_double, c_double, PBsm, c_double,
                           c_double, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "lnv_hotelling": (c_int, [PBsm, PBsm, c_int32, POINTER(LnvCgWs), c_void_p]),
    "lnv_cg_init": (c_int, [PBsm, PBsm, PBsm, c_double, POINTER(LnvCgWs), c_void_p]),
    "lnv_cg_step": (c_int, [PBsm, PBsm, PBsm, PBsm, c_double, c_int64, POINTER(LnvOpts),
                            POINTER(LnvCgWs), c_void_p]),
    "lnv_pm_start": (c_int, [PBsm, PBsm, PBsm, PBsm, c_double, c_double, POINTER(LnvPmWs),
                             c_void_p]),
    "lnv_pm_step": (c_int, [PBsm, PBsm, c_double, c_double, POINTER(LnvPmWs), c_void_p]),
    "lnv_hotelling_batch": (c_int, [PBsm, PBsm, c_int32, POINTER(LnvBatch), POINTER(LnvCgWs),
                                    c_void_p]),
    "lnv_pm_start_batch": (c_int, [PBsm, PBsm, PBsm, PBsm, POINTER(LnvBatch), POINTER(LnvPmWs),
                                   c_void_p]),
    "lnv_pm_step_batch": (c_int, [PBsm, PBsm, POINTER(LnvBatch), c_double, POINTER(LnvPmWs),
                                  c_void_p]),
    "lnv_cg_init_batch": (c_int, [PBsm, PBsm, PBsm, POINTER(LnvBatch), POINTER(LnvCgWs),
                                  c_void_p]),
    "lnv_cg_step_batch": (c_int, [PBsm, PBsm, PBsm, PBsm, POINTER(LnvBatch), c_int64,
                                  POINTER(LnvOpts), POINTER(LnvCgWs), c_void_p]),
    "lnv_bsm_lincomb": (c_int, [c_double, PBsm, c_double, PBsm, c_double, PBsm, PBsm, c_void_p]),
    "lnv_bsm_norm_inf": (c_int, [PBsm, c_void_p, c_void_p, c_void_p]),
    "lnv_bsm_remap": (c_int, [PBsm, PBsm, c_void_p]),
    "lnv_set_f32_accumulation": (c_int, [c_int32]),
    "lnv_timing_enable": (c_int, [c_int32]),
    "lnv_timing_read": (c_int, [POINTER(c_double), POINTER(c_int64)]),
    "lnv_timing_reset": (c_int, []),
}

_LIB = None


class LnvError(RuntimeError):
    def __init__(self, fn, status, lib):
        msg = lib.lnv_strerror(status).decode()
        if status == EHIP:
            msg += f" (hipError_t {lib.lnv_last_hip_error()})"
        super().__init__(f"{fn} failed: {msg} [status {status}]")
        self.status = status


def load(path=None):
    """Load liblnv.so once and declare its signatures; raises when missing."""
    global _LIB
    if _LIB is not None and path is None:
        return _LIB
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _LIB = lib
    return lib


def check(lib, fn, status):
    if status != OK:
        raise LnvError(fn, status, lib)
    return status


def call(fn, *args):
    lib = load()
    return check(lib, fn, getattr(lib, fn)(*args))
