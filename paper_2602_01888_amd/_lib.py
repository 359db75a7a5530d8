"""ctypes binding of libtomg (include/tomg.h).  Argument marshalling only:
every step of the solver runs in the HIP kernels of the library.  There is
no CPU fallback: without the built library the import fails."""

from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtomg.so")

TOMG_OK, TOMG_EINVAL, TOMG_ENOMEM, TOMG_EGEOMETRY = 0, -1, -2, -3
TOMG_ENOCONV, TOMG_ENONFINITE, TOMG_EDEVICE, TOMG_ESTATE = -4, -5, -6, -7
STATUS_NAMES = {0: "TOMG_OK", -1: "TOMG_EINVAL", -2: "TOMG_ENOMEM", -3: "TOMG_EGEOMETRY",
                -4: "TOMG_ENOCONV", -5: "TOMG_ENONFINITE", -6: "TOMG_EDEVICE",
                -7: "TOMG_ESTATE"}
TOMG_FP64, TOMG_FP32_IR = 0, 1
TOMG_GS4, TOMG_JACOBI, TOMG_ZEBRA_X, TOMG_ZEBRA_XY = 0, 1, 2, 3
TOMG_NEU_W, TOMG_NEU_E, TOMG_NEU_S, TOMG_NEU_N = 1, 2, 4, 8
TOMG_GALERKIN, TOMG_REDISCRETIZE = 0, 1
FIELD = {"exx": 0, "exy": 1, "eyy": 2, "det": 3, "rhs": 4, "dir": 5, "stencil": 6, "x": 7}

# Every symbol include/tomg.h declares.
EXPORTS = ["tomg_config_default", "tomg_num_levels", "tomg_workspace_bytes", "tomg_create",
           "tomg_destroy", "tomg_last_error", "tomg_set_stream", "setup_coeffs",
           "tomg_setup_coeffs_async", "tomg_setup_check",
           "tomg_update_rhs", "vcycle", "solve", "residual_norm", "tomg_solve_batch",
           "tomg_batch_step", "tomg_batch_launch", "tomg_field", "tomg_laplace_grid",
           "tomg_export", "tomg_level_shape", "tomg_smooth", "tomg_residual", "tomg_profile",
           "tomg_profile_read", "tomg_copy_probe", "tomg_solve_noalloc",
           "tomg_setup_coeffs_desc", "tomg_update_rhs_desc", "tomg_residual_history"]

TOMG_MAP_SINUSOIDAL, TOMG_MAP_PERTURBED_CIRCLE, TOMG_MAP_POLAR = 1, 2, 3
TOMG_MAX_GAUSSIANS = 16
TOMG_SETUP_ASYNC = 1


class MapDesc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("amp", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("r_in", C.c_double),
                ("r_c", C.c_double), ("r_out", C.c_double), ("pert", C.c_double),
                ("coef", C.c_double * 4), ("phase", C.c_double), ("value_in", C.c_double)]


class SourceDesc(C.Structure):
    _fields_ = [("count", C.c_int32), ("reserved", C.c_int32), ("sigma", C.c_double),
                ("amp", C.c_double * TOMG_MAX_GAUSSIANS),
                ("cx", C.c_double * TOMG_MAX_GAUSSIANS),
                ("cy", C.c_double * TOMG_MAX_GAUSSIANS)]


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("xi0", C.c_double), ("eta0", C.c_double),
                ("dx", C.c_double), ("dy", C.c_double), ("precision", C.c_int32),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("smoother", C.c_int32),
                ("jacobi_omega", C.c_double), ("ir_inner_cycles", C.c_int32),
                ("neumann", C.c_int32), ("flux", C.c_int32), ("coarse_op", C.c_int32),
                ("semi_levels", C.c_int32), ("semi_axis", C.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Loads the library (torch must already be imported so that the HIP
    runtime it brought in is the one the library binds to)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libtomg not built: {path} is missing (run __graft_entry__.build())")
    lib = C.CDLL(path)
    P, D, I32, VP = C.c_void_p, C.c_double, C.c_int32, C.c_void_p
    cfgp = C.POINTER(Config)
    sig = {
        "tomg_config_default": (None, [cfgp, I32, I32, D, D]),
        "tomg_num_levels": (I32, [cfgp]),
        "tomg_workspace_bytes": (C.c_size_t, [cfgp]),
        "tomg_create": (C.c_int, [cfgp, VP, C.c_size_t, VP, C.POINTER(P)]),
        "tomg_destroy": (None, [P]),
        "tomg_last_error": (C.c_char_p, [P]),
        "tomg_set_stream": (C.c_int, [P, VP]),
        "setup_coeffs": (C.c_int, [P, VP, VP, VP, VP, VP, VP]),
        "tomg_setup_coeffs_async": (C.c_int, [P, VP, VP, VP, VP, VP, VP]),
        "tomg_setup_check": (C.c_int, [P]),
        "tomg_update_rhs": (C.c_int, [P, VP]),
        "vcycle": (C.c_int, [P, VP]),
        "solve": (C.c_int, [P, VP, D, I32, C.POINTER(I32), C.POINTER(D)]),
        "residual_norm": (C.c_int, [P, VP, C.POINTER(D), C.POINTER(D)]),
        "tomg_solve_batch": (C.c_int, [C.POINTER(P), C.POINTER(VP), I32, D, I32,
                                       C.POINTER(I32), C.POINTER(D), C.POINTER(C.c_int)]),
        "tomg_batch_step": (C.c_int, [C.POINTER(P), C.POINTER(VP), I32, C.POINTER(I32),
                                      C.POINTER(D)]),
        "tomg_batch_launch": (C.c_int, [C.POINTER(P), C.POINTER(VP), I32, C.POINTER(I32), VP]),
        "tomg_field": (C.c_int, [P, VP, VP, VP, VP, VP, VP]),
        "tomg_laplace_grid": (C.c_int, [P, VP, VP, VP, VP, VP, D, I32, C.POINTER(I32)]),
        "tomg_export": (C.c_int, [P, I32, I32, VP]),
        "tomg_level_shape": (C.c_int, [P, I32, C.POINTER(I32), C.POINTER(I32)]),
        "tomg_smooth": (C.c_int, [P, VP, I32]),
        "tomg_residual": (C.c_int, [P, VP, VP]),
        "tomg_profile": (C.c_int, [P, I32]),
        "tomg_profile_read": (C.c_int, [P, C.POINTER(D)]),
        "tomg_copy_probe": (C.c_int, [VP, VP, C.c_size_t, VP]),
        "tomg_setup_coeffs_desc": (C.c_int, [P, C.POINTER(MapDesc), C.POINTER(SourceDesc), VP,
                                             C.c_uint32]),
        "tomg_update_rhs_desc": (C.c_int, [P, C.POINTER(SourceDesc)]),
        "tomg_residual_history": (C.c_int, [P, C.POINTER(D), I32, C.POINTER(I32)]),
        "tomg_solve_noalloc": (C.c_int, [cfgp, VP, VP, VP, VP, VP, VP, VP, D, I32, VP,
                                         C.POINTER(I32), C.POINTER(D), C.c_char_p,
                                         C.c_size_t]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
