"""ctypes declarations of the C ABI in include/agca.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("AGCA_LIBRARY") or os.path.join(_PKG, "libagca.so")

AGCA_OK, AGCA_E_INVALID, AGCA_E_OOM, AGCA_E_HIP, AGCA_E_NOCONV, AGCA_E_NUMERIC, AGCA_E_STATE = \
    0, -1, -2, -3, -4, -5, -6
F64, F32, BF16 = 0, 1, 2
SMOOTH_JACOBI, SMOOTH_CHEBYSHEV = 0, 1
STORE_BLOCKS, STORE_MEAN = 0, 1
FLAG_RATIO, FLAG_MACRO, FLAG_NONE, FLAG_ALL = 0, 1, 2, 3
SOLVER_PCG, SOLVER_FCG, SOLVER_IR, SOLVER_STATIONARY = 0, 1, 2, 3
MAX_HISTORY = 1024

STATUS_NAMES = {0: "AGCA_OK", -1: "AGCA_E_INVALID", -2: "AGCA_E_OOM", -3: "AGCA_E_HIP",
                -4: "AGCA_E_NOCONV", -5: "AGCA_E_NUMERIC", -6: "AGCA_E_STATE"}


class Config(C.Structure):
    _fields_ = [("L", C.c_int32), ("ncomp", C.c_int32), ("flag_mode", C.c_int32),
                ("mg_dtype", C.c_int32), ("mg_nu_dtype", C.c_int32), ("pre_sweeps", C.c_int32),
                ("post_sweeps", C.c_int32), ("smoother", C.c_int32), ("flag_ratio", C.c_double),
                ("omega", C.c_double), ("mem_limit_bytes", C.c_uint64),
                ("macro_flags", C.c_uint8 * 48), ("coarse_storage", C.c_int32)]


class LevelInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("nodes", C.c_int64), ("free_nodes", C.c_int64),
                ("elements", C.c_int64), ("flagged", C.c_int64), ("block_bytes", C.c_int64),
                ("level_bytes", C.c_int64), ("lambda_max", C.c_double)]


MAX_MILESTONES = 8


class SolveOpts(C.Structure):
    _fields_ = [("solver", C.c_int32), ("max_iter", C.c_int32), ("tol", C.c_double),
                ("use_x0", C.c_int32), ("record_history", C.c_int32), ("n_milestones", C.c_int32),
                ("milestones", C.c_double * MAX_MILESTONES)]


class StokesOpts(C.Structure):
    _fields_ = [("solver", C.c_int32), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("record_history", C.c_int32), ("tol", C.c_double), ("precond", C.c_int32),
                ("schur", C.c_int32), ("schur_iters", C.c_int32), ("velocity_cycles", C.c_int32),
                ("basis_dtype", C.c_int32)]


STOKES_FGMRES, STOKES_MINRES = 0, 1
STOKES_DIAGONAL, STOKES_TRIANGULAR = 0, 1
SCHUR_MASS, SCHUR_BFBT, SCHUR_BFBT_MG = 0, 1, 2


class SolveStats(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("floor_limited", C.c_int32),
                ("replacements", C.c_int32), ("rel_residual", C.c_double),
                ("recursive_rel_residual", C.c_double), ("floor_estimate", C.c_double),
                ("seconds", C.c_double),
                ("milestone_iterations", C.c_int32 * MAX_MILESTONES),
                ("milestone_seconds", C.c_double * MAX_MILESTONES),
                ("milestone_residuals", C.c_double * MAX_MILESTONES),
                ("history", C.c_double * MAX_HISTORY)]


# name -> (restype, argtypes); every symbol include/agca.h declares
SIGNATURES = {
    "agca_default_config": (None, [C.POINTER(Config)]),
    "agca_validate_config": (C.c_int32, [C.POINTER(Config)]),
    "agca_create": (C.c_int32, [C.POINTER(Config), C.c_void_p, C.POINTER(C.c_void_p), C.c_void_p,
                                C.POINTER(C.c_void_p)]),
    "agca_destroy": (C.c_int32, [C.c_void_p]),
    "agca_macro_gradient": (C.c_int32, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "agca_macro_gradient_noalloc": (C.c_int32, [C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "agca_set_nu": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "agca_set_log_nu": (C.c_int32, [C.c_void_p, C.c_void_p, C.POINTER(C.c_void_p)]),
    "agca_query": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(LevelInfo)]),
    "agca_get_flags": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                                   C.POINTER(C.c_int64)]),
    "agca_get_blocks": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "agca_get_diagonal": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64]),
    "agca_apply": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "agca_residual": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "agca_smooth": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_double,
                                C.c_void_p, C.c_void_p]),
    "agca_restrict": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "agca_prolong_add": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "agca_vcycle": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    "agca_dot": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.POINTER(C.c_double)]),
    "agca_cast": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64]),
    "agca_solve": (C.c_int32, [C.c_void_p, C.POINTER(SolveOpts), C.c_void_p, C.c_void_p,
                               C.POINTER(SolveStats)]),
    "agca_residual_floor": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]),
    "agca_grad_log_nu": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "agca_load_vector": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "agca_stokes_div": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "agca_stokes_grad": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "agca_stokes_mass": (C.c_int32, [C.c_void_p, C.c_void_p]),
    "agca_stokes_solve": (C.c_int32, [C.c_void_p, C.POINTER(StokesOpts), C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.POINTER(SolveStats)]),
    "agca_stokes_schur_apply": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "agca_stokes_z_stencil": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "agca_stokes_z_vcycle": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "agca_device_bytes": (C.c_int64, [C.c_void_p]),
    "agca_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH) -> C.CDLL:
    """Load libagca.so; raise if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2511_13109_amd.build` "
                           "(the AGCA library has no CPU fallback)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class AGCAError(RuntimeError):
    def __init__(self, status: int, func: str, msg: str):
        super().__init__(f"{func} -> {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, func: str) -> int:
    if status != AGCA_OK:
        raise AGCAError(status, func, (load().agca_last_error() or b"").decode())
    return status
