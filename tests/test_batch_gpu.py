"""Batched launch (flat and persistent hand-out, one launch per class or a single launch for every
class): every tile of the batch against the FP64 oracle, the modes against each other, graph replays."""
import numpy as np
import pytest
import torch

import synth
from paper_2311_18141_amd import ops

import gpu_util as G

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _tiles(count, seed, rows_hi=4096, value_kind="pm1", long_rows=False):
    tiles, Ns = synth.uneven_tiles(count, seed, rows_lo=64, rows_hi=rows_hi, per_row_lo=0, per_row_hi=64)
    rng = _rng(seed + 1)
    out = []
    for t in tiles:
        L = t.row_lengths()
        if long_rows and t.rows > 200:
            L = L.copy()
            L[rng.integers(0, t.rows, size=3)] = min(t.cols, 1500)
        A = synth.random_csr(t.rows, t.cols, L, rng, value_kind)
        out.append(A)
    return out, Ns


MODES = {"flat": (False, False), "persistent": (True, False), "single": (False, True),
         "single_persistent": (True, True)}


def _run(As, Ns, dtype=torch.float32, kw=None, variants=None, accumulate=False, value_kind="pm1", seed=0,
         mode="flat", item_nnz=0):
    rng = _rng(seed)
    handles = [G.make_tile([A], **(kw or {})) for A in As]
    if variants is not None:
        for h, N, v in zip(handles, Ns, variants):
            ops.spmm_tile_set_variant(h, N, dtype, *v)
    Bh = [synth.dense(A.cols, N, rng, value_kind) for A, N in zip(As, Ns)]
    C0 = [synth.dense(A.rows, N, rng, value_kind) for A, N in zip(As, Ns)]
    Bs = [G.dense_dev(b, dtype) for b in Bh]
    Cs = [G.dense_dev(c, dtype) for c in C0]
    persistent, single = MODES[mode]
    batch = ops.spmm_batch_create(handles, Ns, dtype, item_nnz=item_nnz, persistent=persistent, single=single)
    ops.spmm_batched(batch, Bs, Cs, accumulate=accumulate)
    torch.cuda.synchronize()
    return handles, batch, Bh, C0, Bs, Cs


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("long_rows", [False, True])
def test_batch_matches_oracle(dtype, long_rows, mode):
    G.note("batch dtype=%s long_rows=%s mode=%s" % (dtype, long_rows, mode))
    As, Ns = _tiles(24, 3, long_rows=long_rows)
    kw = dict(long_row=256, segment=128) if long_rows else {}
    handles, batch, Bh, C0, Bs, Cs = _run(As, Ns, dtype, kw, seed=4, mode=mode)
    for t, (A, N) in enumerate(zip(As, Ns)):
        got = G.host_f32(Cs[t])
        if dtype == torch.float32:
            ref, S = G.oracle_fwd([A], [Bh[t]])
            G.assert_fp32_close(got, ref, S, G.row_terms([A]), what="tile %d %s" % (t, batch.variant(t)))
        else:
            ref, S = G.oracle_fwd([A], [G.bf16_as_f32(Bh[t])])
            G.assert_bf16_close(got, ref, S, what="tile %d" % t)


@pytest.mark.parametrize("mode", sorted(MODES))
@pytest.mark.parametrize("variant", [("stream", 0, 1), ("stream", 0, 2), ("stream", 0, 4),
                                     ("rowsplit", 8, 0), ("rowsplit", 16, 0), ("rowsplit", 32, 0),
                                     ("rowsplit", 64, 0)])
def test_batch_variants_integer_exact(variant, mode):
    G.note("batch variant %s mode=%s" % (variant, mode))
    As, Ns = _tiles(12, 5, value_kind="int8", long_rows=True)
    Ns = [128] * len(As)
    handles, batch, Bh, C0, Bs, Cs = _run(As, Ns, kw=dict(long_row=256, segment=100), value_kind="int8",
                                          variants=[variant] * len(As), accumulate=True, seed=6, mode=mode)
    for t, A in enumerate(As):
        ref, _ = G.oracle_fwd([A], [Bh[t]], accumulate=True, C0=C0[t])
        assert np.array_equal(G.host_f32(Cs[t]).astype(np.float64), ref), (t, variant, batch.variant(t))


@pytest.mark.parametrize("mode", sorted(MODES))
def test_batch_graph_replay_deterministic(mode):
    G.note("batch graph replay mode=%s" % mode)
    As, Ns = _tiles(40, 7, long_rows=True)
    handles, batch, Bh, C0, Bs, Cs = _run(As, Ns, kw=dict(long_row=256, segment=128), seed=8, mode=mode)
    eager = [c.clone() for c in Cs]
    ws = batch.workspace()
    ops.spmm_batched(batch, Bs, Cs, workspace=ws)
    torch.cuda.synchronize()
    for c, e in zip(Cs, eager):
        assert torch.equal(c, e)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.spmm_batched(batch, Bs, Cs, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.spmm_batched(batch, Bs, Cs, workspace=ws)
    for r in range(10):
        for c in Cs:
            c.fill_(float("nan"))
        _ = (Bs[0] * 3).sum()
        g.replay()
        torch.cuda.synchronize()
        for t, (c, e) in enumerate(zip(Cs, eager)):
            assert torch.equal(c, e), (r, t)


def test_batch_autotuned_tiles():
    """Per-tile variants chosen by the autotuner, then one batched launch."""
    G.note("batch autotuned")
    As, Ns = _tiles(16, 9, rows_hi=8192)
    rng = _rng(10)
    handles = [G.make_tile([A]) for A in As]
    Bh = [synth.dense(A.cols, N, rng) for A, N in zip(As, Ns)]
    Bs = [G.dense_dev(b) for b in Bh]
    Cs = [torch.empty(A.rows, N, device=G.DEV) for A, N in zip(As, Ns)]
    for h, B, C in zip(handles, Bs, Cs):
        ops.spmm_tile_autotune(h, [B], C, tune_plan=False)
    batch = ops.spmm_batch_create(handles, Ns)
    ops.spmm_batched(batch, Bs, Cs)
    torch.cuda.synchronize()
    for t, A in enumerate(As):
        ref, S = G.oracle_fwd([A], [Bh[t]])
        G.assert_fp32_close(G.host_f32(Cs[t]), ref, S, G.row_terms([A]), what="tile %d %s" % (t, batch.variant(t)))


@pytest.mark.parametrize("item_nnz", [64, 1024, 1 << 20])
def test_batch_modes_and_item_sizes_agree(item_nnz):
    """Every hand-out and launch form, any item size: bitwise the same output (each row is summed
    in CSR order by one wave whatever the item boundaries, split rows in unit order)."""
    G.note("batch modes item_nnz=%d" % item_nnz)
    As, Ns = _tiles(30, 11, long_rows=True)
    kw = dict(long_row=256, segment=128)
    _, _, _, _, _, C_ref = _run(As, Ns, kw=kw, seed=12)
    for mode in sorted(MODES):
        _, batch, _, _, _, Cs = _run(As, Ns, kw=kw, seed=12, mode=mode, item_nnz=item_nnz)
        for t, (c, r) in enumerate(zip(Cs, C_ref)):
            assert torch.equal(c, r), (t, mode, batch.variant(t))


@pytest.mark.parametrize("mode", ["single", "single_persistent"])
def test_single_launch_repeated_calls(mode):
    """The single-launch form's counters are never reset: many calls in a row (eager, varying
    accumulate) keep giving the first call's bits."""
    G.note("batch single launch repeated mode=%s" % mode)
    As, Ns = _tiles(20, 13, long_rows=True)
    kw = dict(long_row=128, segment=64)
    handles, batch, Bh, C0, Bs, Cs = _run(As, Ns, kw=kw, seed=14, mode=mode)
    first = [c.clone() for c in Cs]
    ws = batch.workspace()
    for r in range(25):
        for c in Cs:
            c.fill_(float("nan"))
        ops.spmm_batched(batch, Bs, Cs, workspace=ws)
        if r % 5 == 4:
            torch.cuda.synchronize()
            for t, (c, e) in enumerate(zip(Cs, first)):
                assert torch.equal(c, e), (r, t)
    torch.cuda.synchronize()
    for t, (c, e) in enumerate(zip(Cs, first)):
        assert torch.equal(c, e), t
