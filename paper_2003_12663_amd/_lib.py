"""ctypes declarations of the C ABI in include/bem.h (libbem.so, gfx950)."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem.so")

BEM_OK, BEM_ERR_INVALID, BEM_ERR_DEGENERATE, BEM_ERR_OOM, BEM_ERR_HIP, BEM_ERR_NOCONV, BEM_ERR_STATE = range(7)
STATUS_NAMES = {0: "OK", 1: "INVALID", 2: "DEGENERATE", 3: "OOM", 4: "HIP", 5: "NOCONV", 6: "STATE"}

EXPORTS = [
    "bem_create", "bem_destroy", "bem_last_error", "bem_n_unknowns", "bem_assemble", "bem_copy_rows",
    "bem_near_pairs", "bem_rhs", "bem_matvec", "bem_solve_gmres", "bem_eval_field", "bem_trace_lines",
    "bem_streamer_integral", "bem_set_tuning", "bem_set_profiling", "bem_kernel_stats", "bem_reset_stats",
    "bem_get_counter", "bem_streamer_grad", "bem_get_tuning", "bem_autotune", "bem_panel_points",
    "bem_matvec_noalloc", "bem_pair_integrals", "bem_quad_pair_integrals", "bem_compress",
]


class Body(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("eps_plus", ctypes.c_double), ("eps_minus", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("eta", ctypes.c_double), ("restart", ctypes.c_int32),
                ("constraint_form", ctypes.c_int32), ("basis", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("refinements", ctypes.c_int32)]


class CompressInfo(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int64), ("lowrank_blocks", ctypes.c_int64), ("dense_entries", ctypes.c_int64),
                ("factor_entries", ctypes.c_int64), ("max_rank", ctypes.c_int64)]


class TraceParams(ctypes.Structure):
    _fields_ = [("h", ctypes.c_double), ("e_min", ctypes.c_double), ("start_offset", ctypes.c_double),
                ("max_steps", ctypes.c_int32), ("direction", ctypes.c_int32), ("alpha_a", ctypes.c_double),
                ("alpha_e0", ctypes.c_double), ("alpha_p", ctypes.c_double), ("k_str", ctypes.c_double)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libbem.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2003_12663_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "bem_create": (i32, [i64, P, i64, P, P, i32, P, P, P, ctypes.POINTER(P)]),
        "bem_destroy": (None, [P]),
        "bem_last_error": (ctypes.c_char_p, []),
        "bem_n_unknowns": (i64, [P]),
        "bem_near_pairs": (i64, [P]),
        "bem_assemble": (i32, [P]),
        "bem_copy_rows": (i32, [P, i64, i64, P]),
        "bem_rhs": (i32, [P, i32, P, P]),
        "bem_matvec": (i32, [P, i32, P, P, i32]),
        "bem_matvec_noalloc": (i32, [P, i32, P, P, i32]),
        "bem_pair_integrals": (i32, [P, i64, P, P, i32, P, P]),
        "bem_quad_pair_integrals": (i32, [P, i64, P, P, P, P]),
        "bem_compress": (i32, [P, f64, f64, i32, P]),
        "bem_solve_gmres": (i32, [P, i32, P, f64, i32, P, P]),
        "bem_eval_field": (i32, [P, i32, P, i64, P, P, P, P]),
        "bem_trace_lines": (i32, [P, i32, P, i64, P, P, P, P, P, P]),
        "bem_streamer_integral": (i32, [P, i32, P, i64, P, P, P, P, P, P, P]),
        "bem_set_tuning": (i32, [P, ctypes.c_char_p, i64]),
        "bem_set_profiling": (i32, [P, i32]),
        "bem_kernel_stats": (i32, [P, ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(f64)]),
        "bem_reset_stats": (i32, [P]),
        "bem_get_counter": (i32, [P, ctypes.c_char_p, ctypes.POINTER(i64)]),
        "bem_streamer_grad": (i32, [P, i32, P, i64, P, P, P, P, P, P, f64, P, P, P]),
        "bem_get_tuning": (i32, [P, ctypes.c_char_p, ctypes.POINTER(i64)]),
        "bem_autotune": (i32, [P, ctypes.c_char_p, ctypes.POINTER(i32)]),
        "bem_panel_points": (i32, [P, i64, P, P, f64, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
