"""ctypes binding of the C ABI in ``include/sptc.h``: argument marshalling
only.  Every step of the contraction runs in the HIP library ``libsptc.so``;
there is no other code path.  PyTorch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsptc.so")

MAX_ORDER = 16
MAX_OUT_ORDER = 32

OK, ERR_INVALID_ARG, ERR_DIM_MISMATCH, ERR_KEY_OVERFLOW, ERR_OUT_OF_MEMORY, ERR_CAPACITY, ERR_HIP, ERR_INTERNAL = range(8)

# Every symbol the header declares.
EXPORTS = (
    "sptc_default_options", "sptc_plan", "sptc_plan_info", "sptc_execute", "sptc_plan_status", "sptc_free",
    "sptc_status_string", "sptc_last_error", "sptc_plan_y_groups", "sptc_plan_y_grouped", "sptc_plan_x_counts",
    "sptc_plan_set_stage_events", "sptc_plan_x_groups", "sptc_batch_plan", "sptc_batch_sizes", "sptc_batch_info",
    "sptc_batch_execute", "sptc_batch_free", "sptc_pool_trim", "sptc_contract_noalloc",
)

BATCH_MAX = 4096

MODE_GROUPED, MODE_GLOBAL = 0, 1

STAGES = ("y_count", "y_scan", "y_scatter", "x_probe", "p_scan", "out_clear", "expand", "compact", "group_count",
          "group_fill", "direct", "block", "batch_pack", "batch_segments", "x_sort")


class Coo(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("dims", ctypes.POINTER(ctypes.c_int64)), ("nnz", ctypes.c_int64),
                ("idx", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("load_factor", ctypes.c_double), ("validate", ctypes.c_int32), ("max_probe", ctypes.c_int32),
                ("hash_seed", ctypes.c_uint64), ("out_table_slots", ctypes.c_int64),
                ("stage_events", ctypes.POINTER(ctypes.c_void_p)), ("mode", ctypes.c_int32),
                ("block_mfma", ctypes.c_int32), ("tile", ctypes.c_int32), ("lds_max_keys", ctypes.c_int32),
                ("capture_out_cap", ctypes.c_int64), ("operand_order", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("out_order", ctypes.c_int32), ("out_dims", ctypes.c_int64 * MAX_OUT_ORDER),
                ("products", ctypes.c_int64), ("out_nnz_bound", ctypes.c_int64), ("y_groups", ctypes.c_int64),
                ("y_table_slots", ctypes.c_int64), ("out_table_slots", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("key_bits_contract", ctypes.c_int32),
                ("key_bits_x_free", ctypes.c_int32), ("key_bits_y_free", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("x_groups", ctypes.c_int64), ("wave_groups", ctypes.c_int64), ("block_groups", ctypes.c_int64),
                ("global_groups", ctypes.c_int64), ("direct_groups", ctypes.c_int64),
                ("direct_products", ctypes.c_int64), ("block_mfma", ctypes.c_int32),
                ("block_mfma_work", ctypes.c_int64),
                ("block_tiles_scanned", ctypes.c_int32), ("operands_swapped", ctypes.c_int32),
                ("block_dense_rows", ctypes.c_int32)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("ctx", ctypes.c_void_p)]


class SptcError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"sptc error {status} ({status_string(status)}): {detail}")


_lib = None


def load():
    """Load libsptc.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2410_10094_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    st = ctypes.c_int
    lib.sptc_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.sptc_default_options.restype = None
    lib.sptc_plan.argtypes = [ctypes.POINTER(P), ctypes.POINTER(Coo), ctypes.POINTER(Coo), i32, P, P,
                              ctypes.POINTER(Options), ctypes.POINTER(Allocator), P]
    lib.sptc_plan.restype = st
    lib.sptc_plan_info.argtypes = [P, ctypes.POINTER(Info)]
    lib.sptc_plan_info.restype = st
    lib.sptc_execute.argtypes = [P, P, P, i64, P, P]
    lib.sptc_execute.restype = st
    lib.sptc_plan_status.argtypes = [P, P]
    lib.sptc_plan_status.restype = st
    lib.sptc_free.argtypes = [P]
    lib.sptc_free.restype = None
    lib.sptc_status_string.argtypes = [st]
    lib.sptc_status_string.restype = ctypes.c_char_p
    lib.sptc_last_error.argtypes = []
    lib.sptc_last_error.restype = ctypes.c_char_p
    lib.sptc_plan_y_groups.argtypes = [P, P, P, P, i64, ctypes.POINTER(i64), P]
    lib.sptc_plan_y_groups.restype = st
    lib.sptc_plan_y_grouped.argtypes = [P, P, P, P]
    lib.sptc_plan_y_grouped.restype = st
    lib.sptc_plan_x_counts.argtypes = [P, P, P]
    lib.sptc_plan_x_counts.restype = st
    lib.sptc_plan_set_stage_events.argtypes = [P, ctypes.POINTER(ctypes.c_void_p)]
    lib.sptc_plan_set_stage_events.restype = st
    lib.sptc_plan_x_groups.argtypes = [P, P, P, P, i64, ctypes.POINTER(i64), P]
    lib.sptc_plan_x_groups.restype = st
    lib.sptc_batch_plan.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(Coo), ctypes.POINTER(Coo), P, P, P,
                                    ctypes.POINTER(Options), ctypes.POINTER(Allocator), P]
    lib.sptc_batch_plan.restype = st
    lib.sptc_batch_sizes.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.sptc_batch_sizes.restype = st
    lib.sptc_batch_info.argtypes = [P, i32, ctypes.POINTER(Info), ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.sptc_batch_info.restype = st
    lib.sptc_batch_execute.argtypes = [P, P, P, P, P]
    lib.sptc_batch_execute.restype = st
    lib.sptc_batch_free.argtypes = [P]
    lib.sptc_batch_free.restype = None
    lib.sptc_pool_trim.argtypes = [ctypes.c_size_t]
    lib.sptc_pool_trim.restype = st
    lib.sptc_contract_noalloc.argtypes = [ctypes.POINTER(Coo), ctypes.POINTER(Coo), i32, P, P,
                                          ctypes.POINTER(Options), P, P, i64, P, P]
    lib.sptc_contract_noalloc.restype = st
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().sptc_status_string(status).decode()


def last_error() -> str:
    return load().sptc_last_error().decode()


def check(status: int):
    if status != OK:
        raise SptcError(status, last_error())


def default_options() -> Options:
    o = Options()
    load().sptc_default_options(ctypes.byref(o))
    return o


def make_coo(order: int, dims: Sequence[int], nnz: int, idx_ptr: Optional[int], val_ptr: Optional[int]):
    """Build an sptc_coo; returns (struct, keepalive)."""
    dims_arr = (ctypes.c_int64 * max(order, 1))(*[int(d) for d in dims])
    c = Coo(order, ctypes.cast(dims_arr, ctypes.POINTER(ctypes.c_int64)), nnz, idx_ptr or None, val_ptr or None)
    return c, dims_arr


def int_array(values: Sequence[int]):
    return (ctypes.c_int32 * max(len(values), 1))(*[int(v) for v in values])
