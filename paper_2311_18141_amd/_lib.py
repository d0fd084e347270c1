"""ctypes declarations of libspmm.so (include/spmm.h).  Argument marshalling only.

The library is the product: if it is missing this module raises, it never falls
back to another implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspmm.so")

c_i64 = ctypes.c_int64
c_i32 = ctypes.c_int32
c_int = ctypes.c_int
c_uint = ctypes.c_uint
c_vp = ctypes.c_void_p
c_size = ctypes.c_size_t

SPMM_OK = 0
STATUS_NAMES = {0: "SPMM_OK", 1: "SPMM_ERR_INVALID_ARG", 2: "SPMM_ERR_BAD_CSR", 3: "SPMM_ERR_UNSUPPORTED",
                4: "SPMM_ERR_WORKSPACE", 5: "SPMM_ERR_HIP", 6: "SPMM_ERR_ALLOC"}
SPMM_F32 = 0
SPMM_BF16 = 1
SPMM_TILE_VALIDATE = 1
SPMM_TILE_TRANSPOSE = 2
SPMM_BATCH_PERSISTENT = 1
SPMM_BATCH_SINGLE = 2
SPGEMM_BITMAP_ONLY = 16
SPMM_RESERVE_2D = 1
SPMM_RESERVE_3D = 2
SPMM_RESERVE_OWN = 3


class SpmmCsr(ctypes.Structure):
    _fields_ = [("cols", c_i64), ("nnz", c_i64), ("rowptr", c_vp), ("colind", c_vp), ("values", c_vp)]


class SpmmTileOpts(ctypes.Structure):
    _fields_ = [("flags", c_uint), ("long_row", c_i32), ("segment", c_i32), ("bwd_slice", c_i32),
                ("hot_rows", c_i32)]


class SpmmTileStats(ctypes.Structure):
    _fields_ = [("rows", c_i64), ("num_k", c_i64), ("nnz_total", c_i64), ("max_row", c_i64),
                ("empty_rows", c_i64), ("long_rows", c_i64), ("segments", c_i64),
                ("hist_log2", c_i64 * 33), ("nnz_per_k", c_i64 * 16), ("has_transpose", c_i64),
                ("long_rows_t", c_i64), ("segments_t", c_i64), ("long_row", c_i64), ("segment", c_i64),
                ("hot_rows", c_i64), ("hot_nnz", c_i64)]


class SpmmVariant(ctypes.Structure):
    _fields_ = [("kind", c_i32), ("lanes", c_i32), ("vec", c_i32), ("depth", c_i32)]


SPMM_KERNEL_AUTO = 0
SPMM_KERNEL_ROWSPLIT = 1
SPMM_KERNEL_STREAM = 2
SPMM_KERNEL_FUSED = 3


class SpmmError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), message))


EXPORTS = {
    "spmm_tile_create": (c_int, [c_i64, c_int, c_vp, c_vp, c_vp, c_vp]),
    "spmm_tile_destroy": (c_int, [c_vp]),
    "spmm_tile_get_stats": (c_int, [c_vp, c_vp]),
    "spmm_tile_export_transpose": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp]),
    "spmm_tile_set_variant": (c_int, [c_vp, c_i64, c_int, c_vp]),
    "spmm_tile_set_sddmm_variant": (c_int, [c_vp, c_i64, c_int, c_int]),
    "spmm_tile_set_bwd_variant": (c_int, [c_vp, c_i64, c_int, c_vp]),
    "spmm_tile_get_variant": (c_int, [c_vp, c_i64, c_int, c_int, c_vp]),
    "spmm_tile_autotune_bwd": (c_int, [c_vp, c_i64, c_int, c_vp, c_i64, c_vp, c_i64, c_vp, c_vp, c_i64, c_vp,
                                       c_vp]),
    "spmm_tile_autotune": (c_int, [c_vp, c_i64, c_int, c_vp, c_vp, c_vp, c_i64, c_int, c_vp, c_vp]),
    "spmm_fwd_workspace_bytes": (c_int, [c_vp, c_i64, c_vp]),
    "spmm_fwd": (c_int, [c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_i64, c_int, c_i64, c_int, c_vp, c_size, c_vp]),
    "spmm_fwd_noalloc": (c_int, [c_vp, c_int, c_vp, c_vp, c_int, c_vp, c_i64, c_int, c_i64, c_int, c_vp]),
    "spmm_noalloc_scratch_bytes": (c_size, []),
    "spmm_bwd_workspace_bytes": (c_int, [c_vp, c_i64, c_vp]),
    "spmm_bwd": (c_int, [c_vp, c_vp, c_i64, c_vp, c_i64, c_i64, c_int, c_vp, c_vp, c_i64, c_vp, c_size, c_vp]),
    "spgemm_create": (c_int, [c_i64, c_vp, c_vp, c_uint, c_vp, c_vp]),
    "spgemm_destroy": (c_int, [c_vp]),
    "spgemm_info": (c_int, [c_vp, c_vp, c_vp]),
    "spgemm_pattern_entries": (c_int, [c_vp, c_vp]),
    "spgemm_rowptr": (c_int, [c_vp, c_vp, c_vp]),
    "spgemm_compute": (c_int, [c_vp, c_vp, c_vp, c_vp]),
    "spmm_batch_create": (c_int, [c_int, c_vp, c_vp, c_int, c_i64, c_uint, c_vp, c_vp]),
    "spmm_batch_create_grid": (c_int, [c_int, c_vp, c_vp, c_int, c_vp, c_int, c_i64, c_vp, c_vp]),
    "spmm_batch_destroy": (c_int, [c_vp]),
    "spmm_batch_workspace_bytes": (c_int, [c_vp, c_vp]),
    "spmm_batch_get_variant": (c_int, [c_vp, c_int, c_vp]),
    "spmm_batched": (c_int, [c_vp, c_vp, c_vp, c_vp, c_vp, c_int, c_vp, c_size, c_vp]),
    "spmm_tile_accumulate": (c_int, [c_vp, c_i64, c_vp, c_i64, c_i64, c_i64, c_int, c_vp]),
    "spmm_tile_accumulate_n": (c_int, [c_vp, c_i64, c_vp, c_vp, c_int, c_i64, c_i64, c_int, c_vp]),
    "spmm_gather_probe": (c_int, [c_vp, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "spmm_status_string": (ctypes.c_char_p, [c_int]),
    "spmm_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libspmm.so is not built (run `python -m paper_2311_18141_amd.build`); "
                              "there is no fallback implementation")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != SPMM_OK:
        raise SpmmError(status, lib().spmm_last_error().decode(errors="replace"))
