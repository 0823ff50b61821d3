"""ctypes binding of ``include/pdas.h`` (libpdas.so), same names as the C ABI.

Argument marshalling only: every numerical step runs in the HIP kernels of
libpdas.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libpdas.so")
HEADER = os.path.join(ROOT, "include", "pdas.h")

# lp_status
LP_OK = 0
LP_CONVERGED = 1
LP_OPTIMAL_PSI1 = 2
LP_OPTIMAL_ZERO_DIR = 3
LP_MAX_ITER = 4
LP_ERR_INVALID_ARG = -1
LP_ERR_SHAPE = -2
LP_ERR_NOT_INTERIOR = -3
LP_ERR_BREAKDOWN = -4
LP_ERR_NONPOS_PSI = -5
LP_ERR_LOST_INTERIOR = -6
LP_ERR_WORKSPACE = -7
LP_ERR_NO_TAPE = -8
LP_ERR_DEVICE = -9

LP_PREC_FP64 = 0
LP_PREC_MIXED = 1

# lp_method
LP_METHOD_AFFINE = 0
LP_METHOD_PC = 1

# lp_solver
LP_SOLVER_CHOLESKY = 0
LP_SOLVER_WOODBURY = 1


class lp_options(C.Structure):
    _fields_ = [
        ("alpha", C.c_double),
        ("precision", C.c_int32),
        ("tape_capacity", C.c_int32),
        ("mixed_switch_gap", C.c_double),
        ("refine_tol", C.c_double),
        ("refine_max", C.c_int32),
        ("profile", C.c_int32),
        ("syrk_tile", C.c_int32),
        ("syrk_splits", C.c_int32),
        ("syrk32_splits", C.c_int32),
        ("method", C.c_int32),
        ("solver", C.c_int32),
        ("batch_tile", C.c_int32),
        ("batch_graph_iters", C.c_int32),
        ("reserved", C.c_int32),
        ("reserved2", C.c_int32),
    ]


class lp_iter_info(C.Structure):
    _fields_ = [
        ("k", C.c_int32),
        ("status", C.c_int32),
        ("gap_before", C.c_double),
        ("gap_after", C.c_double),
        ("psi", C.c_double),
        ("t", C.c_double),
        ("argmax", C.c_int64),
        ("min_pivot", C.c_double),
        ("precision_used", C.c_int32),
        ("refine_steps", C.c_int32),
        ("refine_resid", C.c_double),
        ("alpha_primal", C.c_double),
        ("alpha_dual", C.c_double),
        ("sigma", C.c_double),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class lp_timings(C.Structure):
    _fields_ = [
        ("normal_kernel_ms", C.c_double),
        ("normal_ms", C.c_double),
        ("potrf_ms", C.c_double),
        ("trsv_ms", C.c_double),
        ("other_ms", C.c_double),
        ("iter_ms", C.c_double),
        ("iterations", C.c_int64),
        ("normal_launches", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class lp_result(C.Structure):
    _fields_ = [
        ("status", C.c_int32),
        ("iters", C.c_int32),
        ("gap", C.c_double),
        ("primal_obj", C.c_double),
        ("dual_obj", C.c_double),
    ]


_vp = C.c_void_p
_i64 = C.c_int64
_st = C.c_int32  # lp_status is an int-sized enum

_lib = None


def _signatures(lib):
    P = _vp
    sig = {
        "lp_options_default": (None, [C.POINTER(lp_options)]),
        "lp_status_string": (C.c_char_p, [C.c_int32]),
        "lp_workspace_size": (_st, [_i64, _i64, C.POINTER(lp_options), C.POINTER(C.c_size_t)]),
        "lp_setup": (_st, [C.POINTER(P), _i64, _i64, P, P, P, P, P, P, C.POINTER(lp_options), P,
                           C.c_size_t, P]),
        "lp_workspace_size_csr": (_st, [_i64, _i64, _i64, C.POINTER(lp_options),
                                        C.POINTER(C.c_size_t)]),
        "lp_setup_csr": (_st, [C.POINTER(P), _i64, _i64, _i64, P, P, P, P, P, P, P, P,
                               C.POINTER(lp_options), P, C.c_size_t, P]),
        "lp_csr_workspace_size": (_st, [_i64, _i64, _i64, C.POINTER(C.c_size_t)]),
        "lp_normal_matrix_csr": (_st, [_i64, _i64, _i64, P, P, P, P, P, _i64, P, C.c_size_t,
                                       P]),
        "lp_iterate": (_st, [P, C.POINTER(lp_iter_info)]),
        "lp_solve": (_st, [P, C.c_double, C.c_int32, C.POINTER(lp_result),
                           C.POINTER(lp_iter_info)]),
        "lp_get_iterate": (_st, [P, P, P, P]),
        "lp_get_direction": (_st, [P, P, P, P]),
        "lp_tape_row": (_st, [P, C.c_int32, P, P, P]),
        "lp_batch_tape_row": (_st, [P, C.c_int32, P, P, P]),
        "lp_destroy": (_st, [P]),
        "lp_get_timings": (_st, [P, C.POINTER(lp_timings)]),
        "lp_blocks_workspace_size": (_st, [_i64, _i64, C.POINTER(C.c_size_t)]),
        "lp_normal_matrix": (_st, [_i64, _i64, P, P, P, _i64, P, C.c_size_t, P]),
        "lp_cholesky": (_st, [_i64, P, _i64, P, C.c_size_t, P, C.POINTER(_i64),
                              C.POINTER(C.c_double)]),
        "lp_chol_solve": (_st, [_i64, P, _i64, P, P, P, C.c_size_t, P]),
        "lp_backward": (_st, [P, P, P, P, P, P, P, P, P, P]),
        "lp_batch_workspace_size": (_st, [C.c_int32, P, P, C.POINTER(lp_options),
                                          C.POINTER(C.c_size_t)]),
        "lp_batch_setup": (_st, [C.POINTER(P), C.c_int32, P, P, P, P, P, P, P, P, P, P, P,
                                 C.POINTER(lp_options), P, C.c_size_t, P]),
        "lp_batch_solve": (_st, [P, C.c_double, C.c_int32, P, P, C.POINTER(C.c_int32)]),
        "lp_batch_iterate": (_st, [P, C.c_double, P, P]),
        "lp_batch_get_iterate": (_st, [P, P, P, P]),
        "lp_batch_backward": (_st, [P, P, P, P, P, P, P, P, P, P]),
        "lp_batch_destroy": (_st, [P]),
        "lp_chol_solve_noalloc": (_st, [_i64, P, _i64, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    return lib


def load():
    """The loaded libpdas (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libpdas.so not found at {LIB_PATH}; build it with "
                "`python -m paper_1502_03543_amd.build` (no CPU fallback exists)")
        _lib = _signatures(C.CDLL(LIB_PATH))
    return _lib


def declared_functions() -> list[str]:
    """Names of the functions declared in include/pdas.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lp_[a-z_0-9]+)\s*\(", text)))


def status_string(code: int) -> str:
    return load().lp_status_string(int(code)).decode()


def check(code: int, what: str = "") -> int:
    """Raise RuntimeError for error statuses; return the status otherwise."""
    if code < 0:
        raise RuntimeError(f"{what}: {status_string(code)}")
    return code


def _fn(name):
    def call(*args):
        return getattr(load(), name)(*args)
    call.__name__ = name
    return call


# C-ABI functions under their own names
lp_options_default = _fn("lp_options_default")
lp_status_string = _fn("lp_status_string")
lp_workspace_size = _fn("lp_workspace_size")
lp_setup = _fn("lp_setup")
lp_workspace_size_csr = _fn("lp_workspace_size_csr")
lp_setup_csr = _fn("lp_setup_csr")
lp_csr_workspace_size = _fn("lp_csr_workspace_size")
lp_normal_matrix_csr = _fn("lp_normal_matrix_csr")
lp_iterate = _fn("lp_iterate")
lp_solve = _fn("lp_solve")
lp_get_iterate = _fn("lp_get_iterate")
lp_get_direction = _fn("lp_get_direction")
lp_tape_row = _fn("lp_tape_row")
lp_batch_tape_row = _fn("lp_batch_tape_row")
lp_destroy = _fn("lp_destroy")
lp_get_timings = _fn("lp_get_timings")
lp_blocks_workspace_size = _fn("lp_blocks_workspace_size")
lp_normal_matrix = _fn("lp_normal_matrix")
lp_cholesky = _fn("lp_cholesky")
lp_chol_solve = _fn("lp_chol_solve")
lp_backward = _fn("lp_backward")
lp_batch_workspace_size = _fn("lp_batch_workspace_size")
lp_batch_setup = _fn("lp_batch_setup")
lp_batch_solve = _fn("lp_batch_solve")
lp_batch_iterate = _fn("lp_batch_iterate")
lp_batch_get_iterate = _fn("lp_batch_get_iterate")
lp_batch_backward = _fn("lp_batch_backward")
lp_batch_destroy = _fn("lp_batch_destroy")
