"""ctypes declarations of include/stagmi.h and the loader of libstagmi.so.

Argument marshalling only: every step of the operator and the solvers runs in
the library's HIP kernels.  The loader fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstagmi.so")

# status codes
STG_OK = 0
STG_NOT_CONVERGED = 1
STG_BREAKDOWN = 2
STG_INVALID_ARG = -1
STG_HIP_ERROR = -2
STG_WORKSPACE_TOO_SMALL = -3

# link formats
STG_LINK_C128_18 = 0
STG_LINK_C128_12 = 1
STG_LINK_C64_12 = 2
STG_LINK_BF16_12 = 3

# field types
STG_C128 = 0
STG_C64 = 1

# tuning keys
STG_TUNE_XCD_REMAP = 0
STG_TUNE_SITES_PER_THREAD = 1
STG_TUNE_STAGE_NEIGHBOURS = 2
STG_TUNE_THREADS_PER_SITE = 3
STG_TUNE_STAPLE_THREADS = 4
STG_TUNE_PENCIL_TILE = 5
STG_TUNE_FIELDS_PER_LAUNCH = 6
STG_TUNE_LAYER_GROUP = 7
STG_TUNE_SPREAD_EPILOGUE = 8
STG_TUNE_FIELD_SPLIT = 9
STG_TUNE_CG_FORM = 10

# solver modes
STG_CG_F64 = 0
STG_CG_MIXED = 1


class StgLattice(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4)]


class StgGauge(ctypes.Structure):
    _fields_ = [("links", ctypes.c_void_p), ("fmt", ctypes.c_int), ("phases", ctypes.c_void_p)]


class StgCgParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("mode", ctypes.c_int),
                ("delta", ctypes.c_double), ("poll_every", ctypes.c_int),
                ("restart", ctypes.c_int)]


class StgCgStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int),
                ("status", ctypes.c_int), ("converged_iter", ctypes.c_int),
                ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double),
                ("ms_iters", ctypes.c_int), ("pad_", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StgTuneChoice(ctypes.Structure):
    _fields_ = [("xcd_remap", ctypes.c_int), ("sites_per_thread", ctypes.c_int),
                ("stage_neighbours", ctypes.c_int), ("threads_per_site", ctypes.c_int),
                ("us", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StgSolveDesc(ctypes.Structure):
    _fields_ = [("lat", StgLattice), ("hi", StgGauge), ("lo", StgGauge), ("mass", ctypes.c_double),
                ("nrhs", ctypes.c_int), ("b", ctypes.c_void_p), ("x", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_S = ctypes.c_size_t
_LAT = ctypes.POINTER(StgLattice)
_G = ctypes.POINTER(StgGauge)

# name -> (restype, argtypes); the exported surface of include/stagmi.h
SIGNATURES = {
    "stg_version": (_I, []),
    "stg_status_string": (ctypes.c_char_p, [_I]),
    "stg_last_error": (ctypes.c_char_p, []),
    "stg_set_tuning": (_I, [_I, _I]),
    "stg_get_tuning": (_I, [_I, ctypes.POINTER(_I)]),
    "stg_autotune": (_I, [_LAT, _G, _I, _I, _P, _P, ctypes.c_char_p, _P]),
    "stg_autotune_load": (_I, [ctypes.c_char_p, ctypes.POINTER(_I)]),
    "stg_autotune_lookup": (_I, [_LAT, _I, _I, ctypes.POINTER(StgTuneChoice)]),
    "stg_autotune_fields_lookup": (_I, [_LAT, _I, ctypes.POINTER(ctypes.c_int)]),
    "stg_autotune_clear": (None, []),
    "stg_links_bytes": (_I, [_LAT, _I, ctypes.POINTER(_S)]),
    "stg_pack_links": (_I, [_LAT, _P, _I, _P, _P]),
    "stg_pack_phases": (_I, [_LAT, _P, _I, _P, _P]),
    "dirac_apply_eo": (_I, [_LAT, _G, _I, _I, _P, _P, _P]),
    "dirac_apply_oe": (_I, [_LAT, _G, _I, _I, _P, _P, _P]),
    "gauge_staples": (_I, [_LAT, _G, _D, _D, _P, _P]),
    "fermion_force": (_I, [_LAT, _G, _I, ctypes.POINTER(_D), _P, _P, _P, _P]),
    "stout_smear": (_I, [_LAT, _G, _D, _P, _P]),
    "gauge_momentum_update": (_I, [_LAT, _G, _D, _D, _D, _D, _P, _P]),
    "gauge_link_update": (_I, [_LAT, _I, _P, _D, _P, _P]),
    "stout_force_backprop": (_I, [_LAT, _G, _D, _P, _P, _P, _P]),
    "stg_apply_normal": (_I, [_LAT, _G, _I, _I, _D, _D, _P, _P, _P, _P]),
    "stg_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "stg_apply_normal_noalloc": (_I, [_LAT, _G, _I, _I, _D, _D, _P, _P, _P]),
    "stg_dot_workspace_bytes": (_S, []),
    "stg_dot": (_I, [_I, _I, _S, _P, _P, ctypes.POINTER(_D), _P, _S, _P]),
    "stg_cg_default_params": (None, [ctypes.POINTER(StgCgParams)]),
    "stg_workspace_bytes": (_I, [_LAT, _I, _I, _I, ctypes.POINTER(_S)]),
    "cg_solve": (_I, [_LAT, _G, _G, _D, _I, _P, _P, ctypes.POINTER(StgCgParams), _P, _S,
                      ctypes.POINTER(StgCgStats), _P]),
    "multishift_cg_solve": (_I, [_LAT, _G, _G, _D, _I, ctypes.POINTER(_D), _I, _P, _P,
                                 ctypes.POINTER(StgCgParams), _P, _S,
                                 ctypes.POINTER(StgCgStats), _P]),
    "stg_rational_workspace_bytes": (_I, [_LAT, _I, _I, _I, ctypes.POINTER(_S)]),
    "rational_apply": (_I, [_LAT, _G, _G, _D, _I, ctypes.POINTER(_D), ctypes.POINTER(_D), _D,
                            _I, _P, _P, ctypes.POINTER(StgCgParams), _P, _S,
                            ctypes.POINTER(StgCgStats), _P]),
    "stg_batch_workspace_bytes": (_I, [_I, ctypes.POINTER(StgSolveDesc), _I,
                                       ctypes.POINTER(_S)]),
    "cg_solve_batch": (_I, [_I, ctypes.POINTER(StgSolveDesc), ctypes.POINTER(StgCgParams), _P,
                            _S, ctypes.POINTER(StgCgStats), _P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libstagmi.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class StgError(RuntimeError):
    def __init__(self, fn, status):
        lib = load()
        msg = lib.stg_status_string(status).decode()
        last = lib.stg_last_error().decode()
        super().__init__(f"{fn} returned {status} ({msg}){': ' + last if last else ''}")
        self.status = status


def check(fn: str, status: int, ok=(STG_OK,)):
    if status not in ok:
        raise StgError(fn, status)
    return status


def lattice(dims) -> StgLattice:
    lat = StgLattice()
    for i, d in enumerate(dims):
        lat.dims[i] = int(d)
    return lat
