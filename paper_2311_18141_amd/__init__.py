"""Local sparse-times-dense multiply (CSR tile x dense) for MI355X (gfx950).

The kernels live in libspmm.so (C ABI in include/spmm.h); this package is the
thin Python binding over it.  Importing the package does not load the library;
the first call does, and raises if it was not built.
"""
from .ops import (Batch, Tile, spmm_batch_create, spmm_batched, spmm_bwd, spmm_bwd_workspace_bytes, spmm_fwd, spmm_fwd_workspace_bytes,
                  spmm_tile_accumulate, spmm_tile_autotune, spmm_tile_create, spmm_tile_destroy, spmm_tile_export_transpose,
                  spmm_tile_set_variant)

__all__ = ["Batch", "spmm_batch_create", "spmm_batched", "Tile", "spmm_tile_create", "spmm_tile_destroy", "spmm_tile_export_transpose", "spmm_tile_set_variant",
           "spmm_tile_autotune", "spmm_tile_accumulate", "spmm_fwd", "spmm_fwd_workspace_bytes", "spmm_bwd", "spmm_bwd_workspace_bytes"]
