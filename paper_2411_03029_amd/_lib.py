"""ctypes view of libtb.so: the C ABI declared in include/tb.h.

Argument marshalling only.  Every step of the construction and the apply
runs in the library's HIP kernels; there is no Python or CPU fallback, and a
missing library raises immediately.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtb.so")

TB_OK, TB_ERR_INVALID_ARG, TB_ERR_UNSUPPORTED, TB_ERR_OOM, TB_ERR_HIP, \
    TB_ERR_NUMERIC, TB_ERR_IO = range(7)
TB_KERNEL_FOURIER, TB_KERNEL_HELMHOLTZ, TB_KERNEL_RADON, TB_KERNEL_NUDFT, TB_KERNEL_DFT = range(5)
TB_C128, TB_C64, TB_CBF16, TB_C64_OTF, TB_CQ16 = range(5)
TB_STORE_C128, TB_STORE_C64, TB_STORE_CBF16, TB_STORE_OTF, TB_STORE_CQ16 = 1, 2, 4, 8, 16

# every symbol include/tb.h declares
EXPORTS = ("tb_construct", "tb_apply", "tb_apply_adjoint", "tb_apply_noalloc", "tb_apply_batched",
           "tb_batched_reset", "tb_plan_autotune", "tb_plan_set_launch", "tb_plan_info",
           "tb_plan_save", "tb_plan_load", "tb_destroy", "tb_plan_set_timing",
           "tb_plan_stage_times", "tb_last_error", "tb_status_string")

STAGES = ("src_leaf", "src_transfer", "core", "tgt_transfer", "tgt_leaf",
          "tgt_leaf_adj", "tgt_transfer_adj", "core_adj", "src_transfer_adj",
          "src_leaf_adj")


class TbOptions(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int), ("lt_override", ctypes.c_int),
                ("proxy_pair", ctypes.c_int), ("proxy_other", ctypes.c_int),
                ("id_tol_scale", ctypes.c_double), ("store_mask", ctypes.c_uint),
                ("max_rank", ctypes.c_int), ("max_device_bytes", ctypes.c_size_t),
                ("radon_custom", ctypes.c_int), ("radon_a", ctypes.c_double),
                ("radon_b", ctypes.c_double), ("radon_den", ctypes.c_double),
                ("nudft_x", ctypes.POINTER(ctypes.c_double))]


class TbLaunchCfg(ctypes.Structure):
    _fields_ = [("outputs_per_thread", ctypes.c_int), ("rhs_tile", ctypes.c_int),
                ("whole_blocks", ctypes.c_int), ("core_kernel", ctypes.c_int),
                ("fanin_in_turn", ctypes.c_int), ("transfer_mfma", ctypes.c_int),
                ("rhs_per_thread", ctypes.c_int), ("flat_stage", ctypes.c_int)]


class TbPlanInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("d", ctypes.c_int), ("leaf", ctypes.c_int),
                ("n", ctypes.c_longlong), ("L", ctypes.c_int), ("Lt", ctypes.c_int),
                ("Ls", ctypes.c_int), ("r_min", ctypes.c_int), ("r_max", ctypes.c_int),
                ("n_ids", ctypes.c_longlong), ("n_pairs", ctypes.c_longlong),
                ("factor_entries", ctypes.c_longlong), ("core_entries", ctypes.c_longlong),
                ("core_rows", ctypes.c_longlong), ("core_cols", ctypes.c_longlong),
                ("apply_cmacs", ctypes.c_longlong), ("omega", ctypes.c_double),
                ("tol", ctypes.c_double), ("eps_id", ctypes.c_double),
                ("store_mask", ctypes.c_uint), ("device_bytes", ctypes.c_size_t),
                ("construct_ms", ctypes.c_double), ("stage_cmacs", ctypes.c_longlong * 5),
                ("stage_io_entries", ctypes.c_longlong * 5)]


class TBError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libtb.so (built by paper_2411_03029_amd.build); fail loudly."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2411_03029_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.tb_construct.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_longlong,
                                 ctypes.c_double, ctypes.c_double,
                                 ctypes.POINTER(TbOptions), P, ctypes.POINTER(P)]
    lib.tb_apply.argtypes = [P, P, P, ctypes.c_longlong, ctypes.c_int, P]
    lib.tb_apply_adjoint.argtypes = [P, P, P, ctypes.c_longlong, ctypes.c_int, P]
    lib.tb_apply_noalloc.argtypes = [P, P, P, ctypes.c_longlong, ctypes.c_int, ctypes.c_int, P]
    lib.tb_apply_batched.argtypes = [ctypes.c_int, ctypes.POINTER(P), ctypes.POINTER(P),
                                     ctypes.POINTER(P), ctypes.POINTER(ctypes.c_longlong),
                                     ctypes.c_int, ctypes.c_int, P]
    lib.tb_batched_reset.argtypes = []
    lib.tb_plan_set_launch.argtypes = [P, ctypes.c_longlong, ctypes.c_int, ctypes.c_int,
                                       ctypes.POINTER(TbLaunchCfg)]
    lib.tb_plan_autotune.argtypes = [P, ctypes.c_longlong, ctypes.c_int, ctypes.c_char_p, P,
                                     ctypes.POINTER(ctypes.c_int)]
    lib.tb_plan_info.argtypes = [P, ctypes.POINTER(TbPlanInfo)]
    lib.tb_plan_save.argtypes = [P, ctypes.c_char_p]
    lib.tb_plan_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(TbOptions),
                                 ctypes.c_int, P, ctypes.POINTER(P)]
    lib.tb_plan_set_timing.argtypes = [P, ctypes.c_int]
    lib.tb_plan_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_longlong)]
    lib.tb_destroy.argtypes = [P]
    lib.tb_destroy.restype = None
    lib.tb_last_error.restype = ctypes.c_char_p
    lib.tb_status_string.restype = ctypes.c_char_p
    lib.tb_status_string.argtypes = [ctypes.c_int]
    for name in ("tb_construct", "tb_apply", "tb_apply_adjoint", "tb_apply_noalloc",
                 "tb_apply_batched", "tb_batched_reset", "tb_plan_autotune", "tb_plan_set_launch", "tb_plan_info",
                 "tb_plan_save", "tb_plan_load", "tb_plan_set_timing",
                 "tb_plan_stage_times"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def status_name(status: int) -> str:
    return load().tb_status_string(status).decode()


def check(status: int) -> None:
    if status != TB_OK:
        raise TBError(status, load().tb_last_error().decode())
