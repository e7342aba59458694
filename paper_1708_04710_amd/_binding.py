"""ctypes binding of ``libpms.so`` (the C ABI declared in ``include/pms.h``).

Argument marshalling only: every step of the reduction runs in the HIP
kernels of the library.  Loading fails loudly when the library has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpms.so")

PMS_OK = 0
PMS_ERR_INVALID_ARG = -1
PMS_ERR_NOT_COMPATIBLE = -2
PMS_ERR_OOM = -3
PMS_ERR_HIP = -4
PMS_ERR_NOT_CONVERGED = -5
PMS_ERR_CAPACITY = -6
PMS_ERR_INVARIANT = -7
PMS_ERR_TOO_LARGE = -8
PMS_NOALLOC_BYTES = 128 << 20

STATUS_NAMES = {
    PMS_OK: "PMS_OK", PMS_ERR_INVALID_ARG: "PMS_ERR_INVALID_ARG",
    PMS_ERR_NOT_COMPATIBLE: "PMS_ERR_NOT_COMPATIBLE", PMS_ERR_OOM: "PMS_ERR_OOM",
    PMS_ERR_HIP: "PMS_ERR_HIP", PMS_ERR_NOT_CONVERGED: "PMS_ERR_NOT_CONVERGED",
    PMS_ERR_CAPACITY: "PMS_ERR_CAPACITY", PMS_ERR_INVARIANT: "PMS_ERR_INVARIANT",
    PMS_ERR_TOO_LARGE: "PMS_ERR_TOO_LARGE",
}

# every symbol include/pms.h declares (checked by the CPU test suite)
EXPORTED = [
    "pms_create", "pms_destroy", "pms_last_error", "pms_version", "pms_selftest", "pms_default_options",
    "pms_reduce", "pms_reduce_noalloc", "pms_reduce_batched", "pms_round_stats_read", "pms_essential_estimate", "pms_default_tuning", "pms_set_tuning", "pms_get_tuning", "pms_autotune",
    "pms_profile_enable", "pms_profile_kernels", "pms_profile_kernel_name",
    "pms_profile_read", "pms_profile_read_addition_bytes", "pms_build_lowerstar", "pms_build_vr_i32", "pms_build_vr_f32", "pms_filtration_view_get", "pms_filtration_copy_out",
    "pms_filtration_copy_left_beta", "pms_filtration_free", "pms_gather", "pms_backward_lowerstar", "pms_backward_vr_f32",
]


class PmsBoundary(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("col_ptr", ctypes.c_void_p), ("rows", ctypes.c_void_p),
                ("dim", ctypes.c_void_p), ("left", ctypes.c_void_p), ("beta", ctypes.c_void_p)]


class PmsOptions(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("compression", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("chain", ctypes.c_int32),
                ("tail_active", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("graph_rounds", ctypes.c_int32), ("diagnostics", ctypes.c_int32),
                ("arena_entries", ctypes.c_int64), ("debug_invariants", ctypes.c_int32),
                ("c8", ctypes.c_int32), ("sweep", ctypes.c_int32), ("priority", ctypes.c_int32),
                ("round_budget", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class PmsRoundStats(ctypes.Structure):
    _fields_ = [("round", ctypes.c_int32), ("active", ctypes.c_int32), ("new_pivots", ctypes.c_int64),
                ("additions", ctypes.c_int64), ("xor_entries", ctypes.c_int64), ("low_l1", ctypes.c_int64),
                ("ess_estimate", ctypes.c_int64), ("c8_cleared", ctypes.c_int64)]


class PmsTuning(ctypes.Structure):
    _fields_ = [("lane_blocks", ctypes.c_int32), ("chain_blocks", ctypes.c_int32),
                ("lane_steps", ctypes.c_int32), ("lane_steps_few", ctypes.c_int32),
                ("lane_many", ctypes.c_int32), ("lane_refill", ctypes.c_int32),
                ("lane_flush", ctypes.c_int32), ("wide_blocks", ctypes.c_int32),
                ("lane_cap", ctypes.c_int32), ("solve", ctypes.c_int32)]


class PmsFiltrationView(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("nnz", ctypes.c_int64), ("col_ptr", ctypes.c_void_p),
                ("rows", ctypes.c_void_p), ("dim", ctypes.c_void_p), ("value_f32", ctypes.c_void_p),
                ("value_i64", ctypes.c_void_p), ("crit", ctypes.c_void_p), ("verts", ctypes.c_void_p),
                ("left", ctypes.c_void_p), ("beta", ctypes.c_void_p)]


class PmsResult(ctypes.Structure):
    _fields_ = [("low_star", ctypes.c_void_p), ("pair_birth", ctypes.c_void_p),
                ("pair_death", ctypes.c_void_p), ("cap_pairs", ctypes.c_int64),
                ("essential", ctypes.c_void_p), ("cap_essential", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("n_essential", ctypes.c_int64),
                ("rounds", ctypes.c_int32), ("phase0_pivots", ctypes.c_int32),
                ("additions", ctypes.c_int64), ("xor_entries", ctypes.c_int64),
                ("active_sum", ctypes.c_int64), ("addition_bytes", ctypes.c_int64)]


class PmsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_1708_04710_amd.build")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.pms_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, P]
    lib.pms_create.restype = ctypes.c_int
    lib.pms_destroy.argtypes = [P]
    lib.pms_destroy.restype = None
    lib.pms_last_error.argtypes = [P]
    lib.pms_last_error.restype = ctypes.c_char_p
    lib.pms_version.argtypes = []
    lib.pms_version.restype = ctypes.c_char_p
    lib.pms_selftest.argtypes = [P]
    lib.pms_selftest.restype = ctypes.c_int
    lib.pms_default_options.argtypes = []
    lib.pms_default_options.restype = PmsOptions
    lib.pms_reduce.argtypes = [P, ctypes.POINTER(PmsBoundary), ctypes.POINTER(PmsOptions),
                               ctypes.POINTER(PmsResult)]
    lib.pms_reduce.restype = ctypes.c_int
    lib.pms_reduce_noalloc.argtypes = [P, ctypes.POINTER(PmsBoundary), ctypes.POINTER(PmsOptions),
                                       ctypes.POINTER(PmsResult)]
    lib.pms_reduce_noalloc.restype = ctypes.c_int
    lib.pms_reduce_batched.argtypes = [P, ctypes.c_int32, P, ctypes.POINTER(PmsBoundary), ctypes.POINTER(PmsOptions),
                                       ctypes.POINTER(PmsResult), P, P, P]
    lib.pms_reduce_batched.restype = ctypes.c_int
    lib.pms_round_stats_read.argtypes = [P, ctypes.c_int32, ctypes.POINTER(PmsRoundStats),
                                         ctypes.POINTER(ctypes.c_int32)]
    lib.pms_round_stats_read.restype = ctypes.c_int
    lib.pms_essential_estimate.argtypes = [P, ctypes.c_int64, P]
    lib.pms_essential_estimate.restype = ctypes.c_int
    lib.pms_default_tuning.argtypes = []
    lib.pms_default_tuning.restype = PmsTuning
    lib.pms_set_tuning.argtypes = [P, ctypes.POINTER(PmsTuning)]
    lib.pms_set_tuning.restype = ctypes.c_int
    lib.pms_get_tuning.argtypes = [P, ctypes.POINTER(PmsTuning)]
    lib.pms_get_tuning.restype = ctypes.c_int
    lib.pms_autotune.argtypes = [P, ctypes.POINTER(PmsBoundary), ctypes.c_int32, ctypes.POINTER(PmsOptions),
                                 ctypes.POINTER(PmsTuning), ctypes.c_int32, ctypes.POINTER(PmsResult),
                                 ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    lib.pms_autotune.restype = ctypes.c_int
    lib.pms_profile_enable.argtypes = [P, ctypes.c_int]
    lib.pms_profile_enable.restype = ctypes.c_int
    lib.pms_profile_kernels.argtypes = []
    lib.pms_profile_kernels.restype = ctypes.c_int
    lib.pms_profile_kernel_name.argtypes = [ctypes.c_int]
    lib.pms_profile_kernel_name.restype = ctypes.c_char_p
    lib.pms_profile_read.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    lib.pms_profile_read.restype = ctypes.c_int
    lib.pms_profile_read_addition_bytes.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.pms_profile_read_addition_bytes.restype = ctypes.c_int
    lib.pms_build_lowerstar.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(P)]
    lib.pms_build_lowerstar.restype = ctypes.c_int
    for nm in ("pms_build_vr_i32", "pms_build_vr_f32"):
        fn = getattr(lib, nm)
        fn.argtypes = [P, P, ctypes.c_int32, P, P, P, P, ctypes.c_int32, ctypes.POINTER(P), P]
        fn.restype = ctypes.c_int
    lib.pms_gather.argtypes = [P, P, ctypes.c_int64, P, P, P]
    lib.pms_gather.restype = ctypes.c_int
    lib.pms_backward_lowerstar.argtypes = [P, P, ctypes.c_int64, P, P, P, ctypes.c_int64]
    lib.pms_backward_lowerstar.restype = ctypes.c_int
    lib.pms_backward_vr_f32.argtypes = [P, P, ctypes.c_int64, P, P, P, ctypes.c_int32, ctypes.c_int64, P]
    lib.pms_backward_vr_f32.restype = ctypes.c_int
    lib.pms_filtration_view_get.argtypes = [P, ctypes.POINTER(PmsFiltrationView)]
    lib.pms_filtration_view_get.restype = ctypes.c_int
    lib.pms_filtration_copy_out.argtypes = [P, P, P, P, P, P, P, P]
    lib.pms_filtration_copy_out.restype = ctypes.c_int
    lib.pms_filtration_copy_left_beta.argtypes = [P, P, P, P]
    lib.pms_filtration_copy_left_beta.restype = ctypes.c_int
    lib.pms_filtration_free.argtypes = [P]
    lib.pms_filtration_free.restype = None
    _lib = lib
    return lib


def check(ctx, status: int):
    if status != PMS_OK:
        msg = load().pms_last_error(ctx)
        raise PmsError(status, msg.decode() if msg else "")
