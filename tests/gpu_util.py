"""Shared helpers for the GPU parity tests: move seeded inputs to the device, call
the C ABI through the binding, and compare with the FP64 oracle."""
from __future__ import annotations

import sys
from typing import List, Optional, Sequence

import numpy as np
import torch

import oracle
from oracle import compare
import synth
from paper_2311_18141_amd import ops

DEV = "cuda:0"


def note(msg: str) -> None:
    """Name the case before a GPU step, flushed, so a crashed run still says what it ran."""
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def to_dev(csr: synth.CSR):
    return (torch.from_numpy(np.ascontiguousarray(csr.rowptr)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(csr.colind)).to(DEV),
            torch.from_numpy(np.ascontiguousarray(csr.values)).to(DEV), csr.cols)


def make_tile(csrs: Sequence[synth.CSR], validate: bool = True, **kw) -> ops.Tile:
    """Handles in the tests always validate the CSR first (the kernels trust their indices)."""
    return ops.spmm_tile_create(csrs[0].rows, [to_dev(c) for c in csrs], validate=validate, **kw)


def dense_dev(B: np.ndarray, dtype=torch.float32, ld: Optional[int] = None) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(B))
    if dtype == torch.bfloat16:
        t = t.to(torch.bfloat16)       # round to nearest even on the CPU
    if ld is not None and ld > B.shape[1]:
        wide = torch.zeros(B.shape[0], ld, dtype=t.dtype)
        wide[:, : B.shape[1]] = t
        return wide.to(DEV)[:, : B.shape[1]]
    return t.to(DEV)


def host_f32(t: torch.Tensor) -> np.ndarray:
    """Device result -> FP32 NumPy (BF16 widens exactly)."""
    return t.float().cpu().numpy()


def bf16_as_f32(B: np.ndarray) -> np.ndarray:
    """The FP32 value of bf16(B) under round-to-nearest-even, via the oracle's rounding."""
    return oracle.bf16_to_f32(oracle.f32_to_bf16(B))


def row_terms(csrs: Sequence[synth.CSR], rows: Optional[np.ndarray] = None) -> np.ndarray:
    n = sum(c.row_lengths() for c in csrs)
    return n if rows is None else n[rows]


def oracle_fwd(csrs, Bs, k_offset=0, accumulate=False, C0=None, rows=None):
    return oracle.spmm([(c.rowptr, c.colind, c.values) for c in csrs], list(Bs), k_offset=k_offset,
                       accumulate=accumulate, C0=C0, rows=rows)


def assert_fp32_close(got, ref, S, n_terms=None, tol=compare.FP32_TOL, what=""):
    n = None if n_terms is None else np.broadcast_to(np.asarray(n_terms, dtype=np.float64)[:, None], ref.shape)
    st = compare.fp32_stats(got, ref, S, tol=tol, n_terms=n)
    assert compare.fp32_ok(st), (what, st)
    return st


def assert_bf16_close(got, ref, S, what=""):
    st = compare.bf16_stats(got, ref, S)
    assert st["n_over_bound"] == 0, (what, st)
    return st


def fwd(tile, Bs_dev: List[torch.Tensor], **kw) -> torch.Tensor:
    C = ops.spmm_fwd(tile, Bs_dev, **kw)
    torch.cuda.synchronize()
    return C
