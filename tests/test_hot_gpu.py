"""Hot-row staging of the forward: the B rows of each k-tile's most used columns are
copied into the workspace on every call and read there.  The staged rows hold the same
values and the summation order is unchanged, so every result must equal the unstaged
forward bit for bit (any values, FP32 and BF16), and the oracle (exactly on integer data,
within the FP32 tolerance otherwise)."""
import numpy as np
import pytest
import torch

import synth
from paper_2311_18141_amd import ops
from paper_2311_18141_amd._lib import SpmmError

import gpu_util as G

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _skewed_tiles(seed=5, kind="pm1"):
    """Row block 0 of a 4 x 4 grid over R-MAT scale 12 (1024 rows, 4 k-tiles of 1024 columns)."""
    g = synth.rmat_row_block(12, 16, 4, 0, seed=seed)
    if kind == "pm1":
        return g.tiles
    rng = _rng(seed)
    return [synth.CSR(t.rows, t.cols, t.rowptr, t.colind, synth.draw_values(rng, t.nnz, kind)) for t in g.tiles]


def _top_cover(t, H):
    cnt = np.bincount(t.colind, minlength=t.cols)
    used = np.sort(cnt[cnt > 0])[::-1]
    return min(H, used.size), int(used[:H].sum())


VARIANTS = [("stream", 64, 1), ("stream", 64, 2), ("stream", 16, 4), ("rowsplit", 8, 4), ("rowsplit", 16, 2),
            ("rowsplit", 64, 1), ("rowsplit", 32, 4)]


@pytest.mark.parametrize("variant,N", [(v, N) for v in VARIANTS for N in (33, 128, 200) if N % v[2] == 0])
def test_staged_equals_unstaged_fp32(variant, N):
    kind, lanes, vec = variant
    G.note("hot fp32 %s N=%d" % (variant, N))
    tiles = _skewed_tiles()
    rng = _rng(N)
    Bs = [synth.dense(t.cols, N, rng) for t in tiles]
    dB = [G.dense_dev(b) for b in Bs]
    off = G.make_tile(tiles, hot_rows=-1, long_row=64, segment=16)
    on = G.make_tile(tiles, hot_rows=100, long_row=64, segment=16)
    st = on.stats()
    assert st["hot_rows"] == sum(_top_cover(t, 100)[0] for t in tiles)
    assert st["hot_nnz"] == sum(_top_cover(t, 100)[1] for t in tiles)
    assert st["long_rows"] > 0
    assert off.stats()["hot_rows"] == 0 and off.stats()["hot_nnz"] == 0
    for t in (off, on):
        ops.spmm_tile_set_variant(t, N, torch.float32, kind, lanes, vec)
    for k_offset, acc in ((0, False), (1, True), (3, False)):
        C0 = torch.from_numpy(synth.dense(tiles[0].rows, N, rng)).to(G.DEV)
        a = G.fwd(off, dB, C=C0.clone(), k_offset=k_offset, accumulate=acc)
        b = G.fwd(on, dB, C=C0.clone(), k_offset=k_offset, accumulate=acc)
        assert torch.equal(a, b), (variant, N, k_offset, acc)
    ref, S = G.oracle_fwd(tiles, Bs)
    got = G.host_f32(G.fwd(on, dB))
    G.assert_fp32_close(got, ref, S, G.row_terms(tiles), what="hot %s N=%d" % (variant, N))


BF16_VARIANTS = [("stream", 64, 2), ("stream", 64, 1), ("rowsplit", 16, 8), ("rowsplit", 32, 4)]


@pytest.mark.parametrize("variant,N", [(v, N) for v in BF16_VARIANTS for N in (37, 128, 256) if N % v[2] == 0])
def test_staged_bf16_integer_exact(variant, N):
    kind, lanes, vec = variant
    G.note("hot bf16 %s N=%d" % (variant, N))
    tiles = _skewed_tiles(seed=6, kind="int4")
    rng = _rng(N + 1)
    Bs = [synth.dense(t.cols, N, rng, "int4") for t in tiles]
    dB = [G.dense_dev(b, torch.bfloat16) for b in Bs]
    off = G.make_tile(tiles, hot_rows=-1)
    on = G.make_tile(tiles, hot_rows=300)
    for t in (off, on):
        ops.spmm_tile_set_variant(t, N, torch.bfloat16, kind, lanes, vec)
    a = G.fwd(off, dB)
    b = G.fwd(on, dB)
    assert torch.equal(a, b)
    # integer sums below 2^24 are exact in FP32; C's BF16 rounding is then the oracle's
    ref, _ = G.oracle_fwd(tiles, Bs)
    assert np.array_equal(G.host_f32(b), G.bf16_as_f32(ref.astype(np.float32)))


def test_staged_integer_exact_vs_oracle_and_ragged_ld():
    """Integer data (exact in any order) with B as a column slice (ld = N + 2; rows of 61
    floats: the staging copy takes its 4-byte path) and every k-tile's columns all staged."""
    G.note("hot integer exact, ragged ld")
    tiles = _skewed_tiles(seed=7, kind="int8")
    rng = _rng(7)
    N = 61
    Bs = [synth.dense(t.cols, N, rng, "int8") for t in tiles]
    dB = [G.dense_dev(b, ld=N + 2) for b in Bs]
    on = G.make_tile(tiles, hot_rows=4096)
    assert on.stats()["hot_rows"] == sum(int((np.bincount(t.colind, minlength=t.cols) > 0).sum()) for t in tiles)
    assert on.stats()["hot_nnz"] == sum(t.nnz for t in tiles)
    ref, _ = G.oracle_fwd(tiles, Bs)
    for kind in ("stream", "rowsplit"):
        ops.spmm_tile_set_variant(on, N, torch.float32, kind)
        assert np.array_equal(G.host_f32(G.fwd(on, dB)).astype(np.float64), ref)


def test_staging_follows_b_between_calls_and_graph_replay():
    """The staged rows are copied on every call: new B values take effect, eagerly and
    in replays of a captured graph."""
    G.note("hot B changes, graph replay")
    tiles = _skewed_tiles(seed=8)
    rng = _rng(8)
    N = 128
    dB = [G.dense_dev(synth.dense(t.cols, N, rng)) for t in tiles]
    off = G.make_tile(tiles, hot_rows=-1)
    on = G.make_tile(tiles, hot_rows=64)
    C = torch.empty(tiles[0].rows, N, device=G.DEV)
    ws = on.workspace(N)
    ops.spmm_fwd(on, dB, C=C, workspace=ws)
    for b in dB:
        b.mul_(-0.5).add_(0.25)
    assert torch.equal(G.fwd(on, dB, C=torch.empty_like(C), workspace=ws), G.fwd(off, dB))
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.spmm_fwd(on, dB, C=C, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.spmm_fwd(on, dB, C=C, workspace=ws)
    for r in range(3):
        for b in dB:
            b.copy_(torch.from_numpy(synth.dense(b.shape[0], N, rng)).to(G.DEV))
        C.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(C, G.fwd(off, dB)), r


def test_workspace_size_and_check():
    G.note("hot workspace")
    tiles = _skewed_tiles(seed=9)
    N = 40
    on = G.make_tile(tiles, hot_rows=50, long_row=64, segment=16)
    off = G.make_tile(tiles, hot_rows=-1, long_row=64, segment=16)
    st = on.stats()
    part = ops.spmm_fwd_workspace_bytes(off, N)
    assert part == 4 * 40 * st["segments"]
    want = (part + 255) // 256 * 256 + 4 * 40 * st["hot_rows"]
    assert ops.spmm_fwd_workspace_bytes(on, N) == want
    dB = [G.dense_dev(synth.dense(t.cols, N, _rng(9))) for t in tiles]
    small = torch.empty(want - 1, dtype=torch.uint8, device=G.DEV)
    with pytest.raises(SpmmError):
        ops.spmm_fwd(on, dB, workspace=small)


def _skewed_large(rows, cols, per_row, hot, p_hot, seed):
    """Rows of about per_row distinct columns: each draw is one of `hot` columns (spread
    over the index range) with probability p_hot, else uniform."""
    rng = _rng(seed)
    n = rows * per_row
    hot_cols = rng.choice(cols, size=hot, replace=False)
    c = np.where(rng.random(n) < p_hot, hot_cols[rng.integers(0, hot, size=n)], rng.integers(0, cols, size=n))
    key = np.unique(np.repeat(np.arange(rows, dtype=np.int64), per_row) * cols + c)
    r, c = key // cols, (key % cols).astype(np.int32)
    lengths = np.bincount(r, minlength=rows)
    return synth.CSR(rows, cols, synth.rowptr_from_lengths(lengths), c, synth.draw_values(rng, c.size, "pm1"))


def test_default_rule():
    """Library rule: on for a large tile whose few hot columns carry most non-zeros, off
    for uniform columns, small tiles, or when switched off."""
    G.note("hot default rule")
    A = _skewed_large(1 << 16, 1 << 20, 24, 3000, 0.6, 10)
    assert A.nnz >= 1 << 20
    t = G.make_tile([A])
    st = t.stats()
    cnt = np.bincount(A.colind, minlength=A.cols)
    used16 = np.sort(cnt[cnt >= 16])[::-1][:16384]
    assert st["hot_rows"] == used16.size > 0
    assert st["hot_nnz"] == int(used16.sum())
    assert G.make_tile([A], hot_rows=-1).stats()["hot_rows"] == 0
    U = synth.uniform_csr(1 << 16, 1 << 20, 24, seed=11)
    assert G.make_tile([U]).stats()["hot_rows"] == 0
    small = _skewed_large(1 << 12, 1 << 20, 24, 300, 0.6, 12)
    assert small.nnz < 1 << 20
    assert G.make_tile([small]).stats()["hot_rows"] == 0
    N = 128
    dB = [G.dense_dev(synth.dense(A.cols, N, _rng(13)))]
    off = G.make_tile([A], hot_rows=-1)
    for kind in ("stream", "rowsplit"):
        ops.spmm_tile_set_variant(t, N, torch.float32, kind)
        ops.spmm_tile_set_variant(off, N, torch.float32, kind)
        assert torch.equal(G.fwd(t, dB), G.fwd(off, dB)), kind


def test_default_rule_scales_with_width():
    """Library rule on a wide tile (2^23 columns): up to one staged row per 128 columns, at most
    65,536 (16,384 for tiles of 2^21 columns or fewer); results bit-identical to no staging."""
    G.note("hot default rule, wide tile")
    A = _skewed_large(1 << 17, 1 << 23, 24, 80000, 0.7, 14)
    t = G.make_tile([A])
    st = t.stats()
    cnt = np.bincount(A.colind, minlength=A.cols)
    used16 = np.sort(cnt[cnt >= 16])[::-1]
    assert used16.size > 65536
    assert st["hot_rows"] == 65536
    assert st["hot_nnz"] == int(used16[:65536].sum())
    N = 64
    dB = [G.dense_dev(synth.dense(A.cols, N, _rng(15)))]
    off = G.make_tile([A], hot_rows=-1)
    assert torch.equal(G.fwd(t, dB), G.fwd(off, dB))


def test_autotune_with_staging_integer_exact():
    G.note("hot autotune")
    tiles = _skewed_tiles(seed=14, kind="int8")
    rng = _rng(14)
    N = 96
    Bs = [synth.dense(t.cols, N, rng, "int8") for t in tiles]
    dB = [G.dense_dev(b) for b in Bs]
    on = G.make_tile(tiles, hot_rows=128)
    C = torch.empty(tiles[0].rows, N, device=G.DEV)
    ops.spmm_tile_autotune(on, dB, C, tune_plan=True)
    ref, _ = G.oracle_fwd(tiles, Bs)
    assert np.array_equal(G.host_f32(G.fwd(on, dB)).astype(np.float64), ref)


def test_backward_of_staged_handle():
    """The backward reads the caller's colind (SDDMM) and the transposed structure (dB):
    staging changes nothing there, and the forward stays bit-identical."""
    G.note("hot backward")
    A = synth.rmat_csr(12, 16, seed=15)
    rng = _rng(15)
    N = 64
    B = torch.from_numpy(synth.dense(A.cols, N, rng)).to(G.DEV)
    dC = torch.from_numpy(synth.dense(A.rows, N, rng)).to(G.DEV)
    out = []
    for hot in (-1, 200):
        tile = G.make_tile([A], transpose=True, hot_rows=hot)
        C = G.fwd(tile, [B])
        dA, dBo = ops.spmm_bwd(tile, dC, B)
        torch.cuda.synchronize()
        out.append((C, dA, dBo))
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1]) and torch.equal(out[0][2], out[1][2])


def test_mixed_staged_and_plain_k_tiles():
    """A k-tile without non-zeros stages nothing (its entries read B directly) while the
    others stage theirs, in one fused launch."""
    G.note("hot mixed k-tiles")
    tiles = _skewed_tiles(seed=16)
    t1 = tiles[1]
    tiles[1] = synth.CSR(t1.rows, t1.cols, np.zeros(t1.rows + 1, np.int32), np.zeros(0, np.int32),
                         np.zeros(0, np.float32))
    rng = _rng(16)
    N = 64
    dB = [G.dense_dev(synth.dense(t.cols, N, rng)) for t in tiles]
    on = G.make_tile(tiles, hot_rows=100)
    assert on.stats()["hot_rows"] == sum(_top_cover(t, 100)[0] for t in tiles)
    off = G.make_tile(tiles, hot_rows=-1)
    for kind in ("stream", "rowsplit"):
        for t in (on, off):
            ops.spmm_tile_set_variant(t, N, torch.float32, kind)
        assert torch.equal(G.fwd(on, dB, k_offset=2), G.fwd(off, dB, k_offset=2)), kind


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("N", [1, 2, 7])
def test_staging_narrow_rows(dtype, N):
    """Rows of 1, 2 and 7 elements: the staging copy's 4- and 2-byte paths (integer data: exact)."""
    G.note("hot narrow N=%d %s" % (N, dtype))
    tiles = _skewed_tiles(seed=17, kind="int4")
    rng = _rng(17 + N)
    Bs = [synth.dense(t.cols, N, rng, "int4") for t in tiles]
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    dB = [G.dense_dev(b, tdt) for b in Bs]
    on = G.make_tile(tiles, hot_rows=200, long_row=32, segment=8)
    off = G.make_tile(tiles, hot_rows=-1, long_row=32, segment=8)
    for kind in ("stream", "rowsplit"):
        for t in (on, off):
            ops.spmm_tile_set_variant(t, N, tdt, kind)
        a, b = G.fwd(on, dB, k_offset=3), G.fwd(off, dB, k_offset=3)
        assert torch.equal(a, b), kind
    ref, _ = G.oracle_fwd(tiles, Bs, k_offset=3)
    got = G.host_f32(G.fwd(on, dB, k_offset=3))
    if dtype == "f32":
        assert np.array_equal(got.astype(np.float64), ref)
    else:
        assert np.array_equal(got, G.bf16_as_f32(ref.astype(np.float32)))


def test_staging_sixteen_k_tiles_and_empty_columns():
    """The most k-tiles a handle takes (16), one of them without columns (its B has no rows)."""
    G.note("hot 16 k-tiles")
    vrng = _rng(118)
    tiles = [synth.CSR(t.rows, t.cols, t.rowptr, t.colind, synth.draw_values(vrng, t.nnz, "int4"))
             for t in synth.rmat_row_block(12, 16, 16, 0, seed=18).tiles]
    t5 = tiles[5]
    tiles[5] = synth.CSR(t5.rows, 0, np.zeros(t5.rows + 1, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    rng = _rng(18)
    N = 48
    Bs = [synth.dense(t.cols, N, rng, "int4") for t in tiles]
    dB = [G.dense_dev(b) for b in Bs]
    on = G.make_tile(tiles, hot_rows=32, long_row=16, segment=4)
    off = G.make_tile(tiles, hot_rows=-1, long_row=16, segment=4)
    assert on.stats()["hot_rows"] == sum(_top_cover(t, 32)[0] for t in tiles if t.nnz)
    for kind in ("stream", "rowsplit"):
        for t in (on, off):
            ops.spmm_tile_set_variant(t, N, torch.float32, kind)
        for k_offset in (0, 7, 15):
            assert torch.equal(G.fwd(on, dB, k_offset=k_offset), G.fwd(off, dB, k_offset=k_offset)), (kind, k_offset)
    ref, _ = G.oracle_fwd(tiles, Bs, k_offset=7)
    assert np.array_equal(G.host_f32(G.fwd(on, dB, k_offset=7)).astype(np.float64), ref)
