"""ctypes binding of libmgfem.so (argument marshalling only).

Every function of include/mgfem.h is declared here with the same name.  The
library is loaded from this package directory; when it is missing the import
raises, so nothing can silently run without the HIP kernels.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgfem.so")

OK, ERR_INVALID_ARG, ERR_OOM, ERR_HIP, ERR_NOT_CONVERGED, ERR_DIVERGED, \
    ERR_SINGULAR_COARSE, ERR_EMPTY_DOMAIN, ERR_UNSUPPORTED = range(9)
STAB_PAPER, STAB_LOCAL_EIG, STAB_FIXED, STAB_GLOBAL = 0, 1, 2, 3
PREC_FP64, PREC_MIXED = 0, 1
CYCLE_V, CYCLE_W, CYCLE_TWO_GRID = 1, 2, 3
COARSE_GALERKIN, COARSE_REDISCRETISED = 0, 1
SOLVE_WARM_START = 1
EXPORT_PSI, EXPORT_CELL_TYPE, EXPORT_CELL_LAMBDA, EXPORT_A, EXPORT_M, EXPORT_G, \
    EXPORT_NODE_FLAGS, EXPORT_RHS, EXPORT_GN = range(9)

EXPORTED = (
    "mgfem_default_params", "mgfem_setup", "mgfem_solve", "mgfem_adjoint", "mgfem_misfit",
    "mgfem_query", "mgfem_export", "mgfem_level_n", "mgfem_smooth", "mgfem_destroy",
    "mgfem_status_string", "mgfem_last_error", "mgfem_setup_batched", "mgfem_solve_batched",
    "mgfem_level_counts", "mgfem_profile", "mgfem_profile_read", "mgfem_batched_tile",
    "mgfem_setup_mixed_bc", "mgfem_solve_mixed_bc", "mgfem_adjoint_neumann", "mgfem_residual_l2",
    "mgfem_misfit_noalloc", "mgfem_step_cycles",
)


class Params(C.Structure):
    _fields_ = [
        ("stab_rule", C.c_int32), ("gamma", C.c_double), ("lambda_fixed", C.c_double),
        ("snap_alpha", C.c_double), ("nu1", C.c_int32), ("nu2", C.c_int32), ("eta", C.c_int32),
        ("coarsest_n", C.c_int32), ("precision", C.c_int32), ("cycle", C.c_int32),
        ("x_lo", C.c_double), ("y_lo", C.c_double), ("x_hi", C.c_double), ("y_hi", C.c_double),
        ("coarse_cycles", C.c_int32), ("coarse_op", C.c_int32), ("inner_cycles", C.c_int32),
    ]


class Info(C.Structure):
    _fields_ = [
        ("N", C.c_int32), ("n_levels", C.c_int32), ("n_active", C.c_int64),
        ("n_cells_by_type", C.c_int64 * 7), ("n_snapped", C.c_int64),
        ("n_cut_vertices", C.c_int64), ("coarse_n", C.c_int32), ("min_theta", C.c_double),
        ("max_lambda", C.c_double), ("setup_ms", C.c_double), ("global_C", C.c_double),
        ("global_iters", C.c_int32),
    ]


_lib = None


def lib():
    """The loaded library (loaded on first use; raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2505_05105_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    P, D, I32, U32, VP = C.c_void_p, C.c_double, C.c_int32, C.c_uint32, C.c_void_p
    DP = C.POINTER(C.c_double)
    sig = {
        "mgfem_default_params": (C.c_int, [C.POINTER(Params)]),
        "mgfem_setup": (C.c_int, [P, I32, C.POINTER(Params), VP, C.POINTER(P)]),
        "mgfem_setup_mixed_bc": (C.c_int, [P, P, I32, C.POINTER(Params), VP, C.POINTER(P)]),
        "mgfem_solve": (C.c_int, [P, P, P, D, I32, U32, P, DP, C.POINTER(I32)]),
        "mgfem_solve_mixed_bc": (C.c_int, [P, P, P, P, D, I32, U32, P, DP, C.POINTER(I32)]),
        "mgfem_adjoint_neumann": (C.c_int, [P, P, P]),
        "mgfem_adjoint": (C.c_int, [P, P, D, I32, P, P, P, DP, C.POINTER(I32)]),
        "mgfem_misfit": (C.c_int, [P, P, P, DP, P]),
        "mgfem_misfit_noalloc": (C.c_int, [P, P, P, DP, P]),
        "mgfem_query": (C.c_int, [P, C.POINTER(Info)]),
        "mgfem_export": (C.c_int, [P, I32, I32, P]),
        "mgfem_level_n": (I32, [P, I32]),
        "mgfem_smooth": (C.c_int, [P, I32, P, P, I32, I32]),
        "mgfem_destroy": (C.c_int, [P]),
        "mgfem_status_string": (C.c_char_p, [C.c_int]),
        "mgfem_last_error": (C.c_char_p, [P]),
        "mgfem_setup_batched": (C.c_int, [I32, C.POINTER(P), C.POINTER(I32), C.POINTER(Params), VP,
                                          C.POINTER(P)]),
        "mgfem_solve_batched": (C.c_int, [P, C.POINTER(P), C.POINTER(P), D, I32, C.POINTER(P), DP,
                                          C.POINTER(I32)]),
        "mgfem_level_counts": (C.c_int, [P, I32, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64)]),
        "mgfem_profile": (C.c_int, [P, I32]),
        "mgfem_profile_read": (C.c_int, [P, I32, C.POINTER(C.c_int64), DP, DP]),
        "mgfem_batched_tile": (C.c_int, [P]),
        "mgfem_residual_l2": (C.c_int, [P, DP, I32, C.POINTER(I32)]),
        "mgfem_step_cycles": (C.c_int, [P, C.POINTER(I32), I32, C.POINTER(I32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class MgfemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mgfem error {code} ({status_string(code)}): {msg}")
        self.code = code


def status_string(code):
    return lib().mgfem_status_string(code).decode()


def last_error(handle=None):
    return lib().mgfem_last_error(handle).decode()


def default_params(**kw) -> Params:
    p = Params()
    lib().mgfem_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def check(code, handle=None, allow=(OK,)):
    if code not in allow:
        raise MgfemError(code, last_error(handle))
    return code
