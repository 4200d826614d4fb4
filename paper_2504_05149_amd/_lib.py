"""ctypes declarations of the se2conv C ABI (include/se2conv.h).

Loads the in-tree libse2conv.so.  There is no fallback: if the library is not
built, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libse2conv.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED_SIZE, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_INTERNAL = range(6)
F32, F64 = 0, 1
PLAN_HOST_ONLY = 0x1
PLAN_GENERIC = 0x2
K_GAUSS_VM, K_SAMPLES, K_RADIAL_PROFILE, K_EXP_GAUSS = 0, 1, 2, 3
KNORM_DISCRETE, KNORM_CONTINUOUS, KNORM_NONE = 0, 1, 2
TABLE_SEPARABLE, TABLE_FULL, TABLE_SHIFT, TABLE_QUARTER = 0, 1, 2, 3
ADJOINT, GRAPH, TIMING = 0x1, 0x2, 0x4
PASS_KINDS = {0: "xt_slab", 1: "y_pencil", 2: "t_pencil", 3: "x_rows"}

EXPORTED = [
    "se2conv_plan", "se2conv_plan_destroy", "se2conv_coeffs", "se2conv_coeffs_sum", "se2conv_table_info",
    "se2conv_table_release", "se2conv_table_quarter", "se2conv_plan_counts", "se2conv_shift_table", "se2conv_apply_shifted", "se2conv_apply", "se2conv_apply_padded", "se2conv_apply_complex", "se2conv_chain", "se2conv_chain_noalloc", "se2conv_pass_times", "se2conv_field_coeffs",
    "se2conv_profile_grad", "se2conv_powers", "se2conv_sample_bumps", "se2conv_autotune", "se2conv_kernel_grad",
    "se2conv_fused_supported", "se2conv_field_spectra", "se2conv_apply_save", "se2conv_backward",
    "se2conv_status_string",
    "se2conv_last_error",
]


class Shape(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("m", ctypes.c_int32)]


class KernelDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("sigma", ctypes.c_double),
        ("kappa", ctypes.c_double),
        ("theta0", ctypes.c_double),
        ("data", ctypes.c_void_p),
        ("n_knots", ctypes.c_int32),
        ("r_max", ctypes.c_double),
    ]


class Shift(ctypes.Structure):
    _fields_ = [("tx", ctypes.c_double), ("ty", ctypes.c_double), ("weight", ctypes.c_double),
                ("roll", ctypes.c_int32)]


class Problem(ctypes.Structure):
    _fields_ = [
        ("shape_idx", ctypes.c_int32),
        ("batch", ctypes.c_int32),
        ("f", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("tables", ctypes.POINTER(ctypes.c_void_p)),
        ("n_tables", ctypes.c_int32),
    ]


class Se2convError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"se2conv status {status}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    lib.se2conv_plan.argtypes = [ctypes.POINTER(Shape), i32, i32, u32, ctypes.POINTER(vp)]
    lib.se2conv_plan_destroy.argtypes = [vp]
    lib.se2conv_coeffs.argtypes = [vp, i32, ctypes.POINTER(KernelDesc), i32, vp, ctypes.POINTER(sz), vp]
    lib.se2conv_coeffs_sum.argtypes = [vp, i32, ctypes.POINTER(KernelDesc), ctypes.POINTER(ctypes.c_double), i32, vp,
                                       ctypes.POINTER(sz), vp]
    lib.se2conv_table_info.argtypes = [vp, vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(sz)]
    lib.se2conv_table_release.argtypes = [vp, vp]
    lib.se2conv_table_quarter.argtypes = [vp, vp, vp, ctypes.POINTER(sz), vp]
    lib.se2conv_shift_table.argtypes = [vp, i32, ctypes.POINTER(Shift), i32, vp, ctypes.POINTER(sz), vp]
    lib.se2conv_apply_shifted.argtypes = [vp, i32, vp, vp, ctypes.POINTER(ctypes.c_void_p), i32, vp, i32, u32, vp]
    lib.se2conv_plan_counts.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.se2conv_apply.argtypes = [vp, i32, vp, vp, vp, i32, u32, vp]
    lib.se2conv_apply_padded.argtypes = [vp, i32, vp, vp, i32, vp, i32, u32, vp]
    lib.se2conv_apply_complex.argtypes = [vp, i32, vp, vp, vp, i32, u32, vp]
    lib.se2conv_chain.argtypes = [vp, ctypes.POINTER(Problem), i32, u32, vp]
    lib.se2conv_chain_noalloc.argtypes = [vp, ctypes.POINTER(Problem), i32, u32, vp]
    lib.se2conv_pass_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(i32), i32,
                                       ctypes.POINTER(i32)]
    lib.se2conv_field_coeffs.argtypes = [vp, i32, vp, i32, vp, sz, vp]
    lib.se2conv_profile_grad.argtypes = [vp, i32, vp, i32, i32, ctypes.c_double, vp, vp]
    lib.se2conv_powers.argtypes = [vp, i32, vp, vp, i32, vp, i32, u32, vp]
    lib.se2conv_sample_bumps.argtypes = [vp, i32, vp, i32, ctypes.c_double, ctypes.c_double, vp, vp]
    lib.se2conv_autotune.argtypes = [vp, i32, i32, vp]
    lib.se2conv_kernel_grad.argtypes = [vp, i32, vp, vp, sz, i32, vp, vp]
    lib.se2conv_fused_supported.argtypes = [vp, i32]
    lib.se2conv_field_spectra.argtypes = [vp, i32, vp, i32, vp, vp]
    lib.se2conv_apply_save.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp]
    lib.se2conv_backward.argtypes = [vp, i32, vp, vp, vp, i32, vp, vp, vp]
    lib.se2conv_status_string.argtypes = [i32]
    lib.se2conv_status_string.restype = ctypes.c_char_p
    lib.se2conv_last_error.argtypes = []
    lib.se2conv_last_error.restype = ctypes.c_char_p
    for name in ["se2conv_plan", "se2conv_plan_destroy", "se2conv_coeffs", "se2conv_coeffs_sum", "se2conv_table_info",
                 "se2conv_table_release", "se2conv_table_quarter", "se2conv_plan_counts", "se2conv_shift_table",
                 "se2conv_apply_shifted",
                 "se2conv_apply", "se2conv_apply_padded", "se2conv_apply_complex", "se2conv_chain",
                 "se2conv_chain_noalloc", "se2conv_pass_times",
                 "se2conv_field_coeffs",
                 "se2conv_profile_grad", "se2conv_powers", "se2conv_sample_bumps", "se2conv_autotune",
                 "se2conv_kernel_grad", "se2conv_fused_supported", "se2conv_field_spectra", "se2conv_apply_save",
                 "se2conv_backward"]:
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != OK:
        lib = load()
        msg = lib.se2conv_last_error().decode() or lib.se2conv_status_string(status).decode()
        raise Se2convError(status, msg)
