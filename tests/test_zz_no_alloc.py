"""spmm_fwd_noalloc, the forward that allocates nothing (its scratch is a fixed device array
per GPU): on two calls in a row, the second with a smaller input, it gives the bits of spmm_fwd
with a caller workspace, and both match the FP64 oracle; a forward needing more scratch than
the array holds is refused before any launch."""
import numpy as np
import pytest
import torch

import synth
from paper_2311_18141_amd import ops

import gpu_util as G

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _check(tiles, N, dtype, **kw):
    tile = G.make_tile(tiles, **kw)
    rng = _rng(N + len(tiles))
    Bh = [synth.dense(t.cols, N, rng) for t in tiles]
    Bs = [G.dense_dev(b, dtype) for b in Bh]
    assert ops.spmm_fwd_workspace_bytes(tile, N) <= ops.spmm_noalloc_scratch_bytes()
    C_ws = ops.spmm_fwd(tile, Bs)
    C_na = torch.full_like(C_ws, float("nan"))
    ops.spmm_fwd_noalloc(tile, Bs, C=C_na)
    torch.cuda.synchronize()
    assert torch.equal(C_ws, C_na)
    if dtype == torch.float32:
        rC, SC = G.oracle_fwd(tiles, Bh)
        G.assert_fp32_close(G.host_f32(C_na), rC, SC, G.row_terms(tiles))
    else:
        rC, SC = G.oracle_fwd(tiles, [G.bf16_as_f32(b) for b in Bh])
        G.assert_bf16_close(G.host_f32(C_na), rC, SC)
    return tile


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_noalloc_two_calls_second_smaller(dtype):
    G.note("noalloc forward two calls %s" % dtype)
    rng = _rng(7)
    # first call: two k-tiles, split rows (units write partial rows into the scratch) and
    # staged hot rows (copied into the scratch after the partials)
    M = 6000
    L1 = rng.integers(0, 30, size=M)
    L1[[3, 100, 4000]] = [2500, 900, 1700]
    L2 = rng.integers(0, 10, size=M)
    tiles = [synth.random_csr(M, 3000, L1, rng), synth.random_csr(M, 2000, L2, rng)]
    t1 = _check(tiles, 96, dtype, long_row=64, segment=32, hot_rows=256)
    st = t1.stats()
    assert st["segments"] > 0 and st["hot_rows"] > 0
    # second call, smaller: one tile, fewer rows, fewer split units, narrower N
    L3 = rng.integers(0, 12, size=700)
    L3[5] = 600
    t2 = _check([synth.random_csr(700, 900, L3, rng)], 40, dtype, long_row=64, segment=32)
    assert t2.stats()["segments"] > 0


def test_noalloc_refuses_a_forward_larger_than_its_scratch():
    G.note("noalloc forward too large")
    rng = _rng(8)
    M = 20000
    A = synth.random_csr(M, 4000, np.full(M, 40), rng)
    tile = G.make_tile([A], long_row=8, segment=8)
    N = 1024
    assert ops.spmm_fwd_workspace_bytes(tile, N) > ops.spmm_noalloc_scratch_bytes()
    B = torch.zeros(A.cols, N, device=G.DEV)
    C = torch.zeros(A.rows, N, device=G.DEV)
    with pytest.raises(ops.SpmmError) as e:
        ops.spmm_fwd_noalloc(tile, [B], C=C)
    assert e.value.status == 4   # SPMM_ERR_WORKSPACE
