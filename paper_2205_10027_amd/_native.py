"""ctypes declarations of the libglasso C ABI (include/glasso.h)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libglasso.so")

c_double_p = ctypes.POINTER(ctypes.c_double)


class GlassoOptions(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("t0", ctypes.c_double),
        ("shrink", ctypes.c_double),
        ("t_floor", ctypes.c_double),
        ("t_min", ctypes.c_double),
        ("warm_start", ctypes.c_int),
        ("tile_policy", ctypes.c_int),
        ("graphs", ctypes.c_int),
        ("w_mixed", ctypes.c_int),
        ("ls_width", ctypes.c_int),
        ("dense_product", ctypes.c_int),
        ("screen", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("method", ctypes.c_int),
    ]


class GlassoInfo(ctypes.Structure):
    _fields_ = [
        ("objective", ctypes.c_double),
        ("kkt_rel1", ctypes.c_double),
        ("kkt_fro", ctypes.c_double),
        ("kkt_max", ctypes.c_double),
        ("nnz", ctypes.c_int64),
        ("iterations", ctypes.c_int),
        ("ls_trials", ctypes.c_int),
        ("status", ctypes.c_int),
        ("fallback_steps", ctypes.c_int),
        ("time_ms", ctypes.c_double * 8),
        ("aza_gemm_products", ctypes.c_int),
        ("aza_sparse_products", ctypes.c_int),
        ("leaf_launches", ctypes.c_int),
        ("leaf_ms", ctypes.c_double),
        ("leaf_flops", ctypes.c_double),
        ("components", ctypes.c_int),
        ("largest_component", ctypes.c_int),
    ]


# name -> (restype, argtypes); mirrors include/glasso.h
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double
_INT = ctypes.c_int
SIGNATURES = {
    "glasso_default_options": (_INT, [ctypes.POINTER(GlassoOptions)]),
    "glasso_create": (_INT, [ctypes.POINTER(_VP), ctypes.POINTER(GlassoOptions)]),
    "glasso_destroy": (_INT, [_VP]),
    "glasso_error_string": (ctypes.c_char_p, [_INT]),
    "glasso_workspace_size": (_INT, [_I64, _INT, ctypes.POINTER(ctypes.c_size_t)]),
    "glasso_autotune": (_INT, [_VP, _I64, _INT, ctypes.POINTER(_INT), _VP]),
    "glasso_solve": (_INT, [_VP, _VP, _I64, _D, _D, _VP, _VP, ctypes.POINTER(GlassoInfo), _VP]),
    "glasso_solve_batched": (_INT, [_VP, _INT, ctypes.POINTER(_VP), ctypes.POINTER(_I64), ctypes.POINTER(_D), _D,
                                     ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(GlassoInfo), _VP]),
    "glasso_solve_small": (_INT, [_VP, _INT, ctypes.POINTER(_VP), ctypes.POINTER(_I64), ctypes.POINTER(_D), _D,
                                   ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(GlassoInfo), _VP]),
    "glasso_solve_small_static": (_INT, [ctypes.POINTER(GlassoOptions), _INT, ctypes.POINTER(_VP),
                                          ctypes.POINTER(_I64), ctypes.POINTER(_D), _D, ctypes.POINTER(_VP),
                                          ctypes.POINTER(_VP), ctypes.POINTER(GlassoInfo), _VP]),
    "glasso_generate": (_INT, [_VP, _INT, _I64, _I64, ctypes.c_uint64, _VP, _VP, _VP, c_double_p, _VP]),
    "glasso_covariance": (_INT, [_VP, _VP, _I64, _I64, _INT, _VP, _VP]),
    "glasso_cholesky": (_INT, [_VP, _VP, _I64, _VP, ctypes.POINTER(_I64), c_double_p, _VP]),
    "glasso_inverse": (_INT, [_VP, _VP, _I64, _VP, _VP]),
    "glasso_gradient_pass": (_INT, [_VP, _VP, _VP, _VP, _I64, _D, _VP, _VP, c_double_p, _VP]),
    "glasso_precond_product": (_INT, [_VP, _VP, _VP, _I64, _INT, _VP, _VP]),
    "glasso_trial_point": (_INT, [_VP, _VP, _VP, _VP, _VP, _I64, _D, _D, _VP, c_double_p, _VP]),
    "glasso_gista_trial_point": (_INT, [_VP, _VP, _VP, _VP, _VP, _I64, _D, _D, _VP, c_double_p, _VP]),
    "glasso_sparse_product": (_INT, [_VP, _VP, _VP, _VP, _I64, _VP, ctypes.POINTER(_INT), _VP]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libglasso.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python paper_2205_10027_amd/build.py` "
            "(the HIP library is required; there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
