"""ctypes loader for libnbody.so (argument marshalling only).

The library must have been built in-tree with
``python -m paper_cs_0702135_amd.build``; if it is missing, every entry point
raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libnbody.so")

NBODY_OK = 0
NBODY_E_INVAL = -1
NBODY_E_DEVICE = -2
NBODY_E_RANGE = -3
NBODY_E_NONFINITE = -4
NBODY_E_NOMEM = -5

NBODY_ACC_FP32 = 0
NBODY_ACC_DS = 1
NBODY_FIXED_DT = 2
NBODY_ADJ_ACCUMULATE = 4
NBODY_NOALLOC_MAX_NJ = 1048576
NBODY_VALU_KINDS = 5

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
U32 = ctypes.c_uint32
D = ctypes.c_double
INT = ctypes.c_int


class NBodySystem(ctypes.Structure):
    """Mirror of ``nbody_system`` in include/nbody.h."""
    _fields_ = [("n", I64), ("t", P), ("dt", P), ("x", P), ("v", P), ("a", P),
                ("k", P), ("m", P), ("eps2", D), ("eta", D), ("eta_s", D),
                ("dt_max", D), ("dt_min", D), ("flags", U32)]



class NBodyForceConfig(ctypes.Structure):
    """Mirror of ``nbody_force_config`` in include/nbody.h."""
    _fields_ = [("rep", I32), ("i_per_lane", I32), ("waves", I32), ("tile", I32),
                ("min_j_wave", I32), ("target_groups", I32), ("layout", I32)]


class NBodyEnsemble(ctypes.Structure):
    """Mirror of ``nbody_ensemble`` in include/nbody.h."""
    _fields_ = [("n_clusters", I32), ("offsets", P), ("eps2", P), ("t", P), ("dt", P),
                ("x", P), ("v", P), ("a", P), ("k", P), ("m", P), ("eta", D), ("eta_s", D),
                ("dt_max", D), ("dt_min", D), ("flags", U32)]


class NBodyEnsembleConfig(ctypes.Structure):
    """Mirror of ``nbody_ensemble_config`` in include/nbody.h."""
    _fields_ = [("groups_per_cu", I32), ("max_team", I32), ("step_us", D),
                ("barrier_us", D), ("barrier_group_us", D), ("group_rate", D),
                ("steps_coef", D), ("steps_exp", D), ("waves", I32), ("j_tile", I32),
                ("i_per_lane", I32), ("tile_us", D), ("block_coef", D), ("block_exp", D)]


# name -> (restype, argtypes); every symbol include/nbody.h declares
SIGNATURES = {
    "nbody_version": (INT, []),
    "nbody_create": (INT, [ctypes.POINTER(P), INT, P]),
    "nbody_destroy": (INT, [P]),
    "nbody_set_stream": (INT, [P, P]),
    "nbody_last_error": (ctypes.c_char_p, [P]),
    "nbody_sync_status": (INT, [P]),
    "nbody_force": (INT, [P, P, I64, P, P, P, I64, D, P, P, P, U32]),
    "nbody_force_noalloc": (INT, [P, P, I64, P, P, P, I64, D, P, P, P, U32]),
    "nbody_force_sorted": (INT, [P, P, I64, P, P, P, I64, D, P, P, P]),
    "nbody_predict": (INT, [P, I64, D, P, P, P, P, P, P, P]),
    "nbody_schedule": (INT, [P, I64, P, P, P, P, P]),
    "nbody_correct": (INT, [P, I64, I64, P, P, P, P, P, D, D, D, INT, P, P, P, P,
                            P, P]),
    "nbody_initial_dt": (INT, [P, I64, D, P, P, D, D, D, P]),
    "nbody_predict_dev": (INT, [P, I64, P, P, P, P, P, P, P, P]),
    "nbody_force_dev": (INT, [P, P, P, I64, P, P, P, I64, D, P, P, P, U32]),
    "nbody_correct_dev": (INT, [P, I64, P, I64, P, P, P, P, P, D, D, D, INT, P, P, P, P,
                                P, P]),
    "nbody_energy": (INT, [P, I64, P, P, P, D, P]),
    "nbody_init": (INT, [P, ctypes.POINTER(NBodySystem), D]),
    "nbody_blockstep": (INT, [P, ctypes.POINTER(NBodySystem), I64, D,
                              ctypes.POINTER(I64), ctypes.POINTER(I64)]),
    "nbody_ensemble_run": (INT, [P, ctypes.POINTER(NBodyEnsemble), D, P, P]),
    "nbody_ensemble_set": (INT, [P, ctypes.POINTER(NBodyEnsembleConfig)]),
    "nbody_ensemble_get": (INT, [P, ctypes.POINTER(NBodyEnsembleConfig)]),
    "nbody_ensemble_timing": (INT, [P, I32, P, P]),
    "nbody_ensemble_info": (INT, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
    "nbody_ensemble_plan": (INT, [P, I32, I32, P, D, P, P, P, ctypes.POINTER(I32)]),
    "nbody_shared_run": (INT, [P, I64, P, D, D, I64, I64, P, P, P, P, P, P, P, U32]),
    "nbody_shared_run_adjoint": (INT, [P, I64, P, D, D, I64, I64, P, P, P, P, P, P, P, P, P,
                                       P, U32]),
    "nbody_force_adjoint": (INT, [P, I64, P, P, P, D, P, P, P, P, P, P, U32]),
    "nbody_predict_adjoint": (INT, [P, I64, D, P, P, P, P, P, P]),
    "nbody_correct_adjoint": (INT, [P, I64, D, P, P, P, P, P, P, P, P]),
    "nbody_tune_set": (INT, [P, I64, I64, ctypes.POINTER(NBodyForceConfig)]),
    "nbody_tune_clear": (INT, [P]),
    "nbody_profile": (INT, [P, INT, ctypes.POINTER(D), ctypes.POINTER(D),
                            ctypes.POINTER(I64)]),
    "nbody_tune_get": (INT, [P, I64, ctypes.POINTER(NBodyForceConfig)]),
    "nbody_valu_rates": (INT, [P, INT, ctypes.POINTER(D)]),
}

_lib = None


def load():
    """Load libnbody.so and declare its signatures (raises if not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libnbody.so is not built (expected at %s); run "
            "`python -m paper_cs_0702135_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
