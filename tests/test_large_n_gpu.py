"""Wide dense operands: a ragged width above 4096 through every kernel family (forward and
backward), and the widest N the library takes, 64 x 65535 = 4,194,240 columns (one grid row
per column window), where a pinned narrow variant that would need more windows than a launch
holds falls back to the library's choice; one column more is refused.  Small-integer data:
FP32 results are exact."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2311_18141_amd import ops
from paper_2311_18141_amd._lib import SpmmError

import gpu_util as G

pytestmark = pytest.mark.gpu

N_MAX = 64 * 65535


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


@pytest.mark.parametrize("variant", [None, ("stream", 0, 1), ("stream", 16, 1), ("rowsplit", 8, 1),
                                     ("rowsplit", 64, 1)])
def test_ragged_wide_n_forward(variant):
    N = 4101
    G.note("wide N=%d variant %s" % (N, variant))
    rng = _rng(41)
    L = rng.integers(0, 40, size=700)
    L[5] = 900
    A = synth.random_csr(700, 900, L, rng, "int8")
    tile = G.make_tile([A], long_row=256, segment=100)
    if variant is not None:
        ops.spmm_tile_set_variant(tile, N, torch.float32, *variant)
    B = synth.dense(A.cols, N, rng, "int8")
    C0 = synth.dense(A.rows, N, rng, "int8")
    Cd = G.dense_dev(C0)
    G.fwd(tile, [G.dense_dev(B)], C=Cd, accumulate=True)
    ref, _ = G.oracle_fwd([A], [B], accumulate=True, C0=C0)
    assert np.array_equal(G.host_f32(Cd).astype(np.float64), ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_ragged_wide_n_backward(dtype):
    N = 4101
    G.note("wide N=%d backward %s" % (N, dtype))
    rng = _rng(42)
    A = synth.random_csr(600, 800, rng.integers(0, 30, size=600), rng, "int8")
    tile = G.make_tile([A], transpose=True)
    B = synth.dense(A.cols, N, rng, "int8")
    dC = synth.dense(A.rows, N, rng, "int8")
    dA, dB = ops.spmm_bwd(tile, G.dense_dev(dC, dtype), G.dense_dev(B, dtype))
    torch.cuda.synchronize()
    dA_ref, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), dA_ref)
    dB_ref, S = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC)
    got = G.host_f32(dB)
    if dtype == torch.float32:
        assert np.array_equal(got.astype(np.float64), dB_ref)
    else:
        G.assert_bf16_close(got, dB_ref, S)


def test_widest_n():
    G.note("widest N=%d" % N_MAX)
    rng = _rng(43)
    A = synth.CSR(5, 3, np.array([0, 2, 2, 5, 6, 7], np.int32), np.array([0, 2, 0, 1, 2, 1, 0], np.int32),
                  np.array([1, -2, 3, 1, -1, 2, 4], np.float32))
    tile = G.make_tile([A], transpose=True)
    B = synth.dense(A.cols, N_MAX, rng, "int8")
    dC = synth.dense(A.rows, N_MAX, rng, "int8")
    Bd = G.dense_dev(B)
    ref, _ = G.oracle_fwd([A], [B])
    for variant in (None, ("rowsplit", 8, 1), ("stream", 4, 4)):
        if variant is not None:
            ops.spmm_tile_set_variant(tile, N_MAX, torch.float32, *variant)
        C = G.fwd(tile, [Bd])
        assert np.array_equal(G.host_f32(C).astype(np.float64), ref), variant
    ops.spmm_tile_set_bwd_variant(tile, N_MAX, torch.float32, "rowsplit", 4, 1)
    dA, dB = ops.spmm_bwd(tile, G.dense_dev(dC), Bd)
    torch.cuda.synchronize()
    dA_ref, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), dA_ref)
    dB_ref, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC)
    assert np.array_equal(G.host_f32(dB).astype(np.float64), dB_ref)
    # one column more is refused before any launch
    wide = torch.zeros(A.cols, N_MAX + 1, device=G.DEV)
    with pytest.raises(SpmmError):
        ops.spmm_fwd(tile, [wide])
    with pytest.raises(SpmmError):
        ops.spmm_bwd(tile, torch.zeros(A.rows, N_MAX + 1, device=G.DEV), wide)
