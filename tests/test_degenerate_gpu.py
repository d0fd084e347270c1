"""Degenerate shapes through every entry point: tiles with no rows, no columns or no non-zeros,
k-tile rows where some k-tiles are empty, batches holding such tiles, SpGEMM with an empty
operand.  Each call succeeds and gives the definition's result (zero sums; C0 kept under
accumulate)."""
import numpy as np
import pytest
import torch

import synth
from paper_2311_18141_amd import ops

import gpu_util as G

pytestmark = pytest.mark.gpu


def _empty(rows, cols):
    return synth.CSR(rows, cols, np.zeros(rows + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


@pytest.mark.parametrize("rows,cols", [(0, 5), (7, 0), (0, 0), (300, 40)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_empty_tile_forward_and_backward(rows, cols, dtype):
    G.note("degenerate tile %dx%d %s" % (rows, cols, dtype))
    A = _empty(rows, cols)
    tile = G.make_tile([A], transpose=True)
    N = 24
    rng = _rng(51)
    B = G.dense_dev(synth.dense(cols, N, rng, "int8"), dtype)
    C0 = synth.dense(rows, N, rng, "int8")
    C = G.fwd(tile, [B])
    assert C.shape == (rows, N) and (rows == 0 or not bool(C.float().abs().sum()))
    Cd = G.dense_dev(C0, dtype)
    G.fwd(tile, [B], C=Cd, accumulate=True)
    assert np.array_equal(G.host_f32(Cd), C0)
    dC = G.dense_dev(synth.dense(rows, N, rng, "int8"), dtype)
    dA, dB = ops.spmm_bwd(tile, dC, B)
    torch.cuda.synchronize()
    assert dA.numel() == 0
    assert dB.shape == (cols, N) and (cols == 0 or not bool(dB.float().abs().sum()))


def test_k_tiles_with_empty_members():
    G.note("degenerate k-tile row")
    rng = _rng(52)
    M, N = 500, 40
    full = synth.random_csr(M, 300, rng.integers(0, 20, size=M), rng, "int8")
    tiles = [_empty(M, 100), full, _empty(M, 0), _empty(M, 50)]
    tile = G.make_tile(tiles)
    Bh = [synth.dense(t.cols, N, rng, "int8") for t in tiles]
    for k_offset in (0, 1, 3):
        C = G.fwd(tile, [G.dense_dev(b) for b in Bh], k_offset=k_offset)
        ref, _ = G.oracle_fwd(tiles, Bh, k_offset=k_offset)
        assert np.array_equal(G.host_f32(C).astype(np.float64), ref)


@pytest.mark.parametrize("persistent,single", [(False, False), (True, False), (False, True), (True, True)])
def test_batch_with_empty_tiles(persistent, single):
    G.note("degenerate batch persistent=%s single=%s" % (persistent, single))
    rng = _rng(53)
    As = [_empty(0, 10), _empty(64, 64), synth.random_csr(200, 150, rng.integers(0, 30, size=200), rng, "int8"),
          _empty(9, 0), synth.random_csr(1, 1, np.array([1]), rng, "int8")]
    Ns = [32, 64, 32, 8, 32]
    handles = [G.make_tile([A]) for A in As]
    batch = ops.spmm_batch_create(handles, Ns, persistent=persistent, single=single)
    Bh = [synth.dense(A.cols, N, rng, "int8") for A, N in zip(As, Ns)]
    C0 = [synth.dense(A.rows, N, rng, "int8") for A, N in zip(As, Ns)]
    Cs = [G.dense_dev(c) for c in C0]
    ops.spmm_batched(batch, [G.dense_dev(b) for b in Bh], Cs, accumulate=True)
    torch.cuda.synchronize()
    for A, b, c0, C in zip(As, Bh, C0, Cs):
        ref, _ = G.oracle_fwd([A], [b], accumulate=True, C0=c0)
        assert np.array_equal(G.host_f32(C).astype(np.float64), ref)


def test_spgemm_empty_operands():
    G.note("degenerate spgemm")
    rng = _rng(54)
    B = synth.random_csr(30, 40, rng.integers(0, 10, size=30), rng, "int8")
    for A, Bm in ((_empty(0, 30), B), (_empty(12, 30), B), (synth.random_csr(12, 30, rng.integers(0, 5, size=12),
                                                                             rng, "int8"), _empty(30, 40)),
                  (synth.random_csr(12, 30, rng.integers(0, 5, size=12), rng, "int8"), _empty(30, 0))):
        plan = ops.spgemm_create(A.rows, G.to_dev(A), G.to_dev(Bm), validate=True)
        assert plan.nnz_c == 0
        rp = ops.spgemm_rowptr(plan)
        ops.spgemm_compute(plan)
        torch.cuda.synchronize()
        assert rp.cpu().tolist() == [0] * (A.rows + 1)
