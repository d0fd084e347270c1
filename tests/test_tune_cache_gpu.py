"""The variant getter and the autotune cache on real handles: a second set of handles for the
same matrices takes every variant from the file without timing, runs the same kernels (bitwise
equal outputs) and feeds them to a batch."""
import numpy as np
import pytest
import torch

import synth
from paper_2311_18141_amd import ops, tune_cache

import gpu_util as G

pytestmark = pytest.mark.gpu


def test_get_variant_reads_back_the_tables():
    G.note("tune cache: get_variant")
    rng = np.random.Generator(np.random.PCG64(1))
    A = synth.random_csr(500, 400, rng.integers(0, 30, size=500), rng)
    t = G.make_tile([A], transpose=True)
    assert ops.spmm_tile_get_variant(t, 64) is None
    ops.spmm_tile_set_variant(t, 64, torch.float32, "rowsplit", 16, 4)
    ops.spmm_tile_set_bwd_variant(t, 64, torch.bfloat16, "stream", 0, 8)
    assert ops.spmm_tile_get_variant(t, 64) == {"kind": "rowsplit", "lanes": 16, "vec": 4}
    assert ops.spmm_tile_get_variant(t, 64, torch.bfloat16) is None
    assert ops.spmm_tile_get_variant(t, 64, torch.bfloat16, bwd=True) == {"kind": "stream", "lanes": 0, "vec": 8}
    ops.spmm_tile_set_variant(t, 64, torch.float32, None)
    assert ops.spmm_tile_get_variant(t, 64) is None


def test_cache_round_trip(tmp_path):
    G.note("tune cache: round trip")
    path = str(tmp_path / "tune.json")
    tiles, Ns = synth.uneven_tiles(6, seed=11, rows_lo=512, rows_hi=4096)
    rng = np.random.Generator(np.random.PCG64(12))
    Bh = [synth.dense(t.cols, N, rng) for t, N in zip(tiles, Ns)]
    Bs = [G.dense_dev(b) for b in Bh]

    def handles():
        return [G.make_tile([t]) for t in tiles]

    h1 = handles()
    C1 = [torch.empty(t.rows, N, device=G.DEV) for t, N in zip(tiles, Ns)]
    assert tune_cache.autotune(path, h1, Bs, C1) == {"from_cache": 0, "tuned": 6}
    h2 = handles()
    C2 = [torch.empty(t.rows, N, device=G.DEV) for t, N in zip(tiles, Ns)]
    assert tune_cache.autotune(path, h2, Bs, C2) == {"from_cache": 6, "tuned": 0}
    for a, b, N in zip(h1, h2, Ns):
        assert ops.spmm_tile_get_variant(a, N) == ops.spmm_tile_get_variant(b, N) is not None
    for a, b, B in zip(h1, h2, Bs):
        x = ops.spmm_fwd(a, [B])
        y = ops.spmm_fwd(b, [B])
        torch.cuda.synchronize()
        assert torch.equal(x, y)
    batch = ops.spmm_batch_create(h2, Ns)
    for i, (h, N) in enumerate(zip(h2, Ns)):
        v = ops.spmm_tile_get_variant(h, N)
        got = batch.variant(i)
        assert got["kind"] == v["kind"]
    ops.spmm_batched(batch, Bs, C2)
    torch.cuda.synchronize()
    for i, (t, b) in enumerate(zip(tiles, Bh)):
        ref, S = G.oracle_fwd([t], [b])
        G.assert_fp32_close(G.host_f32(C2[i]), ref, S, G.row_terms([t]), what="tile %d" % i)
