"""torch.autograd.Function for C = A B with A in CSR (one tile), A's values and B differentiable.

Forward runs spmm_fwd; backward runs spmm_bwd: dA on A's pattern (sampled
dense-dense product, FP32 like A's values) and dB = A^T dC through the transposed
structure, in B's dtype (FP32 or BF16).  No gradient flows to the pattern.  The tile handle must have been created with
transpose=True over the same ``values`` tensor that is passed to ``apply``
(values are read live, so in-place updates of that tensor are seen).
"""
from __future__ import annotations

import torch

from .ops import Tile, spmm_bwd, spmm_fwd


class SpMMFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values: torch.Tensor, B: torch.Tensor, tile: Tile) -> torch.Tensor:
        if tile.num_k != 1:
            raise ValueError("SpMMFunction needs a single-tile handle")
        if values.data_ptr() != tile.values[0].data_ptr():
            raise ValueError("values must be the tensor the tile handle was created over")
        C = spmm_fwd(tile, [B.contiguous()])
        ctx.tile = tile
        ctx.save_for_backward(B)
        return C

    @staticmethod
    def backward(ctx, dC: torch.Tensor):
        (B,) = ctx.saved_tensors
        want_dA, want_dB = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (want_dA or want_dB):
            return None, None, None
        # dC arrives in C's dtype (B's): FP32, or BF16 for a BF16 forward (FP32 accumulation)
        dA, dB = spmm_bwd(ctx.tile, dC.contiguous().to(B.dtype), B.contiguous(), want_dA=want_dA, want_dB=want_dB)
        return dA, dB, None


def spmm(values: torch.Tensor, B: torch.Tensor, tile: Tile) -> torch.Tensor:
    return SpMMFunction.apply(values, B, tile)
