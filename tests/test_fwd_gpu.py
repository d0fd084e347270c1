"""Forward parity: libspmm's HIP path against the FP64 oracle on seeded inputs."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2311_18141_amd import ops
from paper_2311_18141_amd._lib import SpmmError

import gpu_util as G

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


KINDS = ["rowsplit", "stream"]


def _pin(tile, N, kind, dtype=torch.float32, lanes=0, vec=0):
    ops.spmm_tile_set_variant(tile, N, dtype, kind, lanes, vec)


def _blockdiag_3x3(value_rng):
    """All 2^9 patterns of a 3x3 block on the diagonal of a 1536 x 1536 tile, small-integer values."""
    rows, cols, vals = [], [], []
    for m in range(512):
        for r in range(3):
            for c in range(3):
                if (m >> (3 * r + c)) & 1:
                    rows.append(3 * m + r)
                    cols.append(3 * m + c)
                    v = int(value_rng.integers(-4, 5)) or 1
                    vals.append(v)
    rows = np.array(rows)
    lengths = np.bincount(rows, minlength=1536)
    return synth.CSR(1536, 1536, synth.rowptr_from_lengths(lengths), np.array(cols, np.int32),
                     np.array(vals, np.float32))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("N", [1, 32, 33, 64, 128, 256])
def test_all_3x3_patterns_exact(N, kind):
    G.note("all_3x3_patterns N=%d %s" % (N, kind))
    rng = _rng(100 + N)
    A = _blockdiag_3x3(rng)
    B = synth.dense(1536, N, rng, "int4")
    tile = G.make_tile([A], validate=True)
    _pin(tile, N, kind)
    got = G.host_f32(G.fwd(tile, [G.dense_dev(B)]))
    ref, _ = G.oracle_fwd([A], [B])
    assert np.array_equal(got.astype(np.float64), ref)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("M", [1, 2, 63, 64, 65, 200])
@pytest.mark.parametrize("N", [1, 32, 33, 64, 128, 256])
def test_small_shapes(M, N, kind):
    G.note("small_shapes M=%d N=%d %s" % (M, N, kind))
    rng = _rng(M * 1000 + N)
    lengths = rng.integers(0, 41, size=M)
    lengths[rng.random(M) < 0.25] = 0
    A = synth.random_csr(M, 97, lengths, rng)
    B = synth.dense(97, N, rng)
    tile = G.make_tile([A], validate=True)
    _pin(tile, N, kind)
    got = G.host_f32(G.fwd(tile, [G.dense_dev(B)]))
    ref, S = G.oracle_fwd([A], [B])
    G.assert_fp32_close(got, ref, S, G.row_terms([A]), what="M=%d N=%d" % (M, N))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("N", [32, 128])
@pytest.mark.parametrize("split", [False, True])
def test_integer_exact_with_long_rows(N, split, kind):
    """Integer values and B in [-8, 8]: every partial sum is an integer below 2^24, so any order is exact."""
    G.note("integer_exact N=%d split=%s %s" % (N, split, kind))
    rng = _rng(7 + N + split)
    M, K = 3001, 60000
    lengths = rng.integers(0, 200, size=M)
    lengths[rng.random(M) < 0.2] = 0
    lengths[[5, 1000, 2999]] = [5000, 50000, 1025]
    A = synth.random_csr(M, K, lengths, rng, "int8")
    B = synth.dense(K, N, rng, "int8")
    kw = dict(long_row=16, segment=8) if split else {}
    tile = G.make_tile([A], validate=True, **kw)
    _pin(tile, N, kind)
    st = tile.stats()
    assert st["max_row"] == 50000 and st["long_rows"] >= 2
    got = G.host_f32(G.fwd(tile, [G.dense_dev(B)]))
    ref, _ = G.oracle_fwd([A], [B])
    assert np.array_equal(got.astype(np.float64), ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_identity_and_permutation_exact(dtype):
    G.note("identity_permutation %s" % dtype)
    rng = _rng(31)
    n, N = 5000, 128
    B = synth.dense(n, N, rng)
    Bd = G.dense_dev(B, dtype)
    eye = synth.CSR(n, n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, np.float32))
    got = G.fwd(G.make_tile([eye]), [Bd])
    assert torch.equal(got, Bd)
    pi = rng.permutation(n).astype(np.int32)
    P = synth.CSR(n, n, np.arange(n + 1, dtype=np.int32), pi, np.ones(n, np.float32))
    got = G.fwd(G.make_tile([P]), [Bd])
    assert torch.equal(got, Bd[torch.from_numpy(pi).long().to(Bd.device)])


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("K", [2, 3, 4, 7])
def test_k_tiles_and_offsets(K, kind):
    """Section 2.1 / Algorithm 2: a tile row of K k-tiles; every k offset gives the untiled product."""
    G.note("k_tiles K=%d %s" % (K, kind))
    rng = _rng(40 + K)
    M, cols, N = 2049, 3001, 64
    lengths = rng.integers(0, 120, size=M)
    lengths[[0, 77]] = [2500, 1800]
    full = synth.random_csr(M, cols, lengths, rng, "int8")
    B = synth.dense(cols, N, rng, "int8")
    ts = -(-cols // K)
    rowid = np.repeat(np.arange(M), full.row_lengths())
    tiles, Bs = [], []
    for k in range(K):
        c0, c1 = k * ts, min(cols, (k + 1) * ts)
        sel = (full.colind >= c0) & (full.colind < c1)
        tiles.append(synth.CSR(M, c1 - c0, synth.rowptr_from_lengths(np.bincount(rowid[sel], minlength=M)),
                               (full.colind[sel] - c0).astype(np.int32), full.values[sel].copy()))
        Bs.append(np.ascontiguousarray(B[c0:c1]))
    tile = G.make_tile(tiles, validate=True, long_row=256, segment=128)
    _pin(tile, N, kind)
    Bd = [G.dense_dev(b) for b in Bs]
    ref, _ = G.oracle_fwd([full], [B])
    outs = []
    for off in range(K + 1):
        got = G.fwd(tile, Bd, k_offset=off)
        assert np.array_equal(G.host_f32(got).astype(np.float64), ref), off
        outs.append(got)
    # real-valued inputs: within tolerance for every offset
    fv = [synth.CSR(t.rows, t.cols, t.rowptr, t.colind, synth.uniform_pm1(rng, t.nnz)) for t in tiles]
    Bf = [synth.dense(b.shape[0], N, rng) for b in Bs]
    tile2 = G.make_tile(fv, long_row=256, segment=128)
    _pin(tile2, N, kind)
    Bfd = [G.dense_dev(b) for b in Bf]
    for off in range(K):
        got = G.host_f32(G.fwd(tile2, Bfd, k_offset=off))
        ref2, S2 = G.oracle_fwd(fv, Bf, k_offset=off)
        G.assert_fp32_close(got, ref2, S2, G.row_terms(fv), what="off=%d" % off)


@pytest.mark.parametrize("kind", KINDS)
def test_accumulate_and_leading_dims(kind):
    G.note("accumulate_and_leading_dims %s" % kind)
    rng = _rng(50)
    M, K, N = 1000, 800, 96
    lengths = rng.integers(0, 50, size=M)
    lengths[3] = 3000 if K >= 3000 else K
    A = synth.random_csr(M, K, lengths, rng)
    B = synth.dense(K, N, rng)
    C0 = synth.dense(M, N, rng)
    tile = G.make_tile([A], long_row=100, segment=64)
    _pin(tile, N, kind)
    Bd = G.dense_dev(B, ld=N + 8)
    Cd = G.dense_dev(C0, ld=N + 4)
    assert Bd.stride(0) == N + 8 and Cd.stride(0) == N + 4
    G.fwd(tile, [Bd], C=Cd, accumulate=True)
    ref, S = G.oracle_fwd([A], [B], accumulate=True, C0=C0)
    G.assert_fp32_close(G.host_f32(Cd), ref, S + np.abs(C0), G.row_terms([A]) + 1)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("N", [32, 128, 256])
def test_bf16_storage(N, kind):
    """B and C in BF16, FP32 products and sums, C rounded once."""
    G.note("bf16 N=%d %s" % (N, kind))
    rng = _rng(60 + N)
    M = K = 4096
    lengths = rng.integers(0, 64, size=M)
    lengths[[1, 2]] = [4000, 1500]
    A = synth.random_csr(M, K, lengths, rng)
    B = synth.dense(K, N, rng)
    tile = G.make_tile([A], long_row=512, segment=256)
    _pin(tile, N, kind, torch.bfloat16)
    got = G.host_f32(G.fwd(tile, [G.dense_dev(B, torch.bfloat16)]))
    Bt = G.bf16_as_f32(B)
    ref, S = G.oracle_fwd([A], [Bt])
    G.assert_bf16_close(got, ref, S)
    # small integers stay exact in BF16 (|C| <= 64, row length <= 4)
    Ai = synth.random_csr(M, K, rng.integers(0, 5, size=M), rng, "int4")
    Bi = synth.dense(K, N, rng, "int4")
    ti = G.make_tile([Ai])
    _pin(ti, N, kind, torch.bfloat16)
    got = G.host_f32(G.fwd(ti, [G.dense_dev(Bi, torch.bfloat16)]))
    ref, _ = G.oracle_fwd([Ai], [Bi])
    assert np.array_equal(got.astype(np.float64), ref)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("empty_share", [0.5, 0.0])
def test_default_rule_every_width_class_exact(empty_share, dtype):
    """No variant entry: the library's own choice at each width class (windows of 64, 128 or 256
    columns, ragged last windows, stream or row-split by the share of empty rows) on small-integer
    inputs, exact in FP32 and in BF16 (|C| <= 64 with at most 4 terms a row)."""
    G.note("default_rule widths empty=%.1f %s" % (empty_share, dtype))
    rng = _rng(90 + int(empty_share * 10))
    M, K = 8192, 4096
    lengths = rng.integers(1, 5, size=M)
    lengths[rng.random(M) < empty_share] = 0
    A = synth.random_csr(M, K, lengths, rng, "int4")
    tile = G.make_tile([A])
    assert (tile.stats()["empty_rows"] * 8 > M) == (empty_share > 0)
    for N in (64, 96, 128, 192, 256, 320, 384):
        B = synth.dense(K, N, rng, "int4")
        got = G.host_f32(G.fwd(tile, [G.dense_dev(B, dtype)]))
        ref, _ = G.oracle_fwd([A], [B])
        assert np.array_equal(got.astype(np.float64), ref), N


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("N", [32, 128])
def test_workload_shapes_scaled(N, kind):
    """Scaled-down versions of the workloads: uniform, R-MAT row block, heavy-tailed rows."""
    G.note("workload_shapes_scaled N=%d %s" % (N, kind))
    cases = []
    er = synth.uniform_csr(4096, 4096, 16, seed=1)
    cases.append(("uniform", [er]))
    g = synth.rmat_row_block(14, 16, 4, 0, seed=2)
    cases.append(("rmat14_rowblock0", g.tiles))
    pl = synth.powerlaw_csr(1 << 15, 1 << 15, 32, 4096, seed=3)
    cases.append(("powerlaw", [pl]))
    rng = _rng(70 + N)
    for name, tiles in cases:
        Bs = [synth.dense(t.cols, N, rng) for t in tiles]
        tile = G.make_tile(tiles, validate=True)
        _pin(tile, N, kind)
        got = G.host_f32(G.fwd(tile, [G.dense_dev(b) for b in Bs]))
        ref, S = G.oracle_fwd(tiles, Bs)
        G.assert_fp32_close(got, ref, S, G.row_terms(tiles), what=name)


@pytest.mark.parametrize("kind", KINDS)
def test_deterministic_and_graph_replay(kind):
    G.note("deterministic_and_graph_replay %s" % kind)
    rng = _rng(80)
    A = synth.powerlaw_csr(1 << 14, 1 << 14, 32, 8192, seed=8)
    B = synth.dense(A.cols, 128, rng, "normal")
    tile = G.make_tile([A], long_row=256, segment=128)
    _pin(tile, 128, kind)
    Bd = G.dense_dev(B)
    C1 = G.fwd(tile, [Bd]).clone()
    C2 = G.fwd(tile, [Bd]).clone()
    assert torch.equal(C1, C2)
    Cg = torch.empty_like(C1)
    ws = tile.workspace(128)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.spmm_fwd(tile, [Bd], C=Cg, workspace=ws)       # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.spmm_fwd(tile, [Bd], C=Cg, workspace=ws)
    for r in range(5):
        Cg.fill_(float("nan"))
        _ = (Bd * 2).sum()                                  # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Cg, C1), r


@pytest.mark.parametrize("case", ["first_not_zero", "decreasing", "last_not_nnz", "col_out_of_range",
                                  "unsorted", "duplicate"])
def test_validation_rejects_bad_csr(case):
    G.note("validation %s" % case)
    rp = np.array([0, 2, 4, 6], np.int32)
    ci = np.array([0, 3, 1, 2, 0, 4], np.int32)
    va = np.ones(6, np.float32)
    if case == "first_not_zero":
        rp = np.array([1, 2, 4, 6], np.int32)
    elif case == "decreasing":
        rp = np.array([0, 4, 2, 6], np.int32)
    elif case == "last_not_nnz":
        rp = np.array([0, 2, 4, 5], np.int32)
    elif case == "col_out_of_range":
        ci = np.array([0, 3, 1, 2, 0, 5], np.int32)
    elif case == "unsorted":
        ci = np.array([3, 0, 1, 2, 0, 4], np.int32)
    elif case == "duplicate":
        ci = np.array([0, 3, 2, 2, 0, 4], np.int32)
    A = synth.CSR(3, 5, rp, ci, va)
    with pytest.raises(SpmmError) as e:
        G.make_tile([A], validate=True)
    assert e.value.status == 2


def test_forward_argument_errors():
    G.note("forward_argument_errors")
    A = synth.uniform_csr(64, 64, 4, seed=9)
    tile = G.make_tile([A], long_row=2, segment=1)
    B = G.dense_dev(synth.dense(64, 32, _rng(1)))
    with pytest.raises(SpmmError) as e:
        ops.spmm_fwd(tile, [B], workspace=torch.empty(4, dtype=torch.uint8, device=G.DEV))
    assert e.value.status == 4
    with pytest.raises(ValueError):
        ops.spmm_fwd(tile, [B, B])


def test_variants_agree_bitwise_on_integers():
    """Every forward variant gives the same integer-valued C (an order-free exact result)."""
    G.note("variants_agree_bitwise")
    rng = _rng(90)
    g = synth.rmat_row_block(13, 16, 4, 0, seed=9)
    tiles = [synth.CSR(t.rows, t.cols, t.rowptr, t.colind, synth.draw_values(rng, t.nnz, "int8")) for t in g.tiles]
    N = 64
    Bs = [synth.dense(t.cols, N, rng, "int8") for t in tiles]
    ref, _ = G.oracle_fwd(tiles, Bs)
    Bd = [G.dense_dev(b) for b in Bs]
    tile = G.make_tile(tiles, long_row=64, segment=32)
    for kind, lanes, vec in [("rowsplit", 4, 1), ("rowsplit", 8, 2), ("rowsplit", 16, 4), ("rowsplit", 32, 2),
                             ("rowsplit", 64, 1), ("stream", 0, 1), ("stream", 0, 2), ("stream", 0, 4),
                             ("stream", 4, 2), ("stream", 16, 1), ("stream", 32, 4), ("stream", 64, 2)]:
        _pin(tile, N, kind, lanes=lanes, vec=vec)
        got = G.host_f32(G.fwd(tile, Bd))
        assert np.array_equal(got.astype(np.float64), ref), (kind, lanes, vec)


def test_autotune_keeps_results():
    G.note("autotune")
    rng = _rng(91)
    A = synth.powerlaw_csr(1 << 15, 1 << 15, 32, 8192, seed=10)
    N = 128
    B = synth.dense(A.cols, N, rng)
    tile = G.make_tile([A])
    Bd = G.dense_dev(B)
    C = torch.empty(A.rows, N, device=G.DEV)
    chosen = ops.spmm_tile_autotune(tile, [Bd], C, tune_plan=True)
    assert chosen["kind"] in ("rowsplit", "stream")
    got = G.host_f32(G.fwd(tile, [Bd]))
    ref, S = G.oracle_fwd([A], [B])
    G.assert_fp32_close(got, ref, S, G.row_terms([A]), what=str(chosen))


def test_variant_argument_errors():
    G.note("variant_argument_errors")
    A = synth.uniform_csr(64, 64, 4, seed=9)
    tile = G.make_tile([A])
    with pytest.raises(SpmmError):
        ops.spmm_tile_set_variant(tile, 32, torch.float32, "rowsplit", lanes=3)
    with pytest.raises(SpmmError):
        ops.spmm_tile_set_variant(tile, 32, torch.float32, "rowsplit", vec=8)
    ops.spmm_tile_set_variant(tile, 32, torch.float32, None)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_stationary_a_partials_and_accumulate(dtype):
    """Section 3.2 / Algorithm 1: the owner of A(i,k) forms the partial A_ik B_kj (overwriting), the
    owner of C(i,j) adds every partial into its tile; the sum equals C0 + sum_k A_ik B_kj."""
    G.note("stationary_a %s" % dtype)
    rng = _rng(93)
    K, M, cols, N = 3, 1500, 900, 64
    tiles = [synth.random_csr(M, cols, rng.integers(0, 30, size=M), rng, "int4") for _ in range(K)]
    Bs = [synth.dense(cols, N, rng, "int4") for _ in range(K)]
    C0 = synth.dense(M, N, rng, "int4")
    Cd = G.dense_dev(C0, dtype)
    for k in range(K):
        h = G.make_tile([tiles[k]])
        part = G.fwd(h, [G.dense_dev(Bs[k], dtype)])            # local_c = local_a * local_b
        ops.spmm_tile_accumulate(Cd, part)                      # C.my_tile() += partial
    torch.cuda.synchronize()
    ref, S = G.oracle_fwd(tiles, Bs, accumulate=True, C0=C0)
    got = G.host_f32(Cd)
    if dtype == torch.float32:
        assert np.array_equal(got.astype(np.float64), ref)      # small integers: exact in any order
    else:
        # every partial and every running sum is rounded to BF16 once per step
        assert np.all(np.abs(got - ref) <= (K + 1) * 2.0 ** -8 * (np.abs(C0) + S) + 1e-6)
