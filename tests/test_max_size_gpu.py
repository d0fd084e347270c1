"""The largest operand the library takes: one tile of 2^31 - 2^16 non-zeros (the cap that keeps
int32 positions clear of overflow under the kernels' strides), 16,776,704 rows of 128 entries
over 2^20 columns, built on the device.  Validation, the transposed structure, the forward,
dA and dB run at that size; the oracle checks sampled output rows of C and dB and the dA
entries of sampled rows, exactly (small-integer data: every sum is exact in FP32)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2311_18141_amd import ops

import gpu_util as G

pytestmark = pytest.mark.gpu

L = 128
ROWS = (1 << 24) - 512          # ROWS * L = 2^31 - 2^16
COLS = 1 << 20
N = 4


def _offsets():
    """Row i holds columns [o_i, o_i + L): o_i from a multiplicative hash of i."""
    i = np.arange(ROWS, dtype=np.uint64)
    return ((i * np.uint64(2654435761)) % np.uint64(COLS - L)).astype(np.int64)


def _row_values(i):
    """Values of row(s) i (int64 array): ((i + 3 j) mod 7) - 3, j = 0..L-1."""
    j = np.arange(L, dtype=np.int64)
    return (((np.asarray(i, dtype=np.int64)[..., None] + 3 * j) % 7) - 3).astype(np.float32)


def _sub_csr(rows, off):
    """The listed rows of A as a CSR over all columns (host)."""
    n = len(rows)
    rp = (np.arange(n + 1, dtype=np.int64) * L).astype(np.int32)
    ci = (off[rows][:, None] + np.arange(L)).astype(np.int32).ravel()
    va = _row_values(rows).ravel()
    return rp, ci, va


def test_max_nnz_tile_fwd_bwd():
    nnz = ROWS * L
    assert nnz == (1 << 31) - (1 << 16)
    G.note("max-size tile: %d rows x %d, nnz %d, N %d" % (ROWS, COLS, nnz, N))
    off = _offsets()
    rng = np.random.Generator(np.random.PCG64(31))
    Bh = synth.dense(COLS, N, rng, "int8")
    dCh = synth.dense(ROWS, N, rng, "int8")
    dev = G.DEV
    off_d = torch.from_numpy(off.astype(np.int32)).to(dev)
    rowptr = torch.arange(ROWS + 1, dtype=torch.int64, device=dev).mul_(L).to(torch.int32)
    j = torch.arange(L, dtype=torch.int32, device=dev)
    colind = (off_d[:, None] + j[None, :]).reshape(-1)
    ri = torch.arange(ROWS, dtype=torch.int32, device=dev)
    values = ((ri[:, None] + 3 * j[None, :]) % 7 - 3).to(torch.float32).reshape(-1)
    del ri
    B = torch.from_numpy(Bh).to(dev)
    dC = torch.from_numpy(dCh).to(dev)
    tile = ops.spmm_tile_create(ROWS, [(rowptr, colind, values, COLS)], validate=True, transpose=True)
    C = ops.spmm_fwd(tile, [B])
    dA, dB = ops.spmm_bwd(tile, dC, B)
    torch.cuda.synchronize()
    G.note("max-size tile: checking samples")

    sample = np.unique(np.concatenate([[0, 1, ROWS // 2, ROWS - 2, ROWS - 1],
                                       rng.integers(0, ROWS, size=59)]))
    rp, ci, va = _sub_csr(sample, off)
    ref, _ = oracle.spmm([(rp, ci, va)], [Bh])
    got = C[torch.from_numpy(sample).to(dev)].cpu().numpy().astype(np.float64)
    assert np.array_equal(got, ref)

    dA_ref, _ = oracle.sddmm(rp, ci, dCh[sample], Bh)
    pos = (sample[:, None] * L + np.arange(L)).ravel()
    got = dA[torch.from_numpy(pos).to(dev)].cpu().numpy().astype(np.float64)
    assert np.array_equal(got, dA_ref)

    cols = np.unique(np.concatenate([[0, L - 1, COLS // 2, COLS - 1], rng.integers(0, COLS, size=12)]))
    rows_t = np.nonzero(((off[:, None] <= cols[None, :]) & (cols[None, :] < off[:, None] + L)).any(axis=1))[0]
    rp2, ci2, va2 = _sub_csr(rows_t, off)
    dB_ref, _ = oracle.spmm_t(rp2, ci2, va2, COLS, dCh[rows_t], out_rows=cols)
    got = dB[torch.from_numpy(cols).to(dev)].cpu().numpy().astype(np.float64)
    assert np.array_equal(got, dB_ref)
    del tile, C, dA, dB, colind, values, rowptr
    torch.cuda.empty_cache()
