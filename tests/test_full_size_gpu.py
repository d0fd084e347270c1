"""Parity at the full workload sizes, in the launch configuration bench.py times (its pinned
kernel variant and split plan per workload), on sampled outputs the oracle computes one by
one, plus properties that hold at any size (bit-exact transposed structure, finite
differences)."""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import compare
from paper_2311_18141_amd import ops

import gpu_util as G

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402  (the pinned launch configuration of each workload)

pytestmark = pytest.mark.gpu


def _bench_tile(workload, tiles, N, dtypes=(torch.float32,), transpose=False, dev_tiles=None):
    """A handle built and pinned the way bench.py builds it for `workload`."""
    pin = bench.PINNED[workload]
    dt = dev_tiles or [G.to_dev(t) for t in tiles]
    tile = ops.spmm_tile_create(tiles[0].rows, dt, validate=True, transpose=transpose,
                                long_row=pin["long_row"], segment=pin["segment"])
    for d in dtypes:
        kind, lanes, vec = pin["variant"]
        ops.spmm_tile_set_variant(tile, N, d, kind, lanes, vec)
        if "bwd_variant" in pin:                      # the backward's dB pass
            ops.spmm_tile_set_bwd_variant(tile, N, d, *pin["bwd_variant"])
    if "sddmm" in pin:
        ops.spmm_tile_set_sddmm_variant(tile, N, pin["sddmm"][0], pin["sddmm"][1])
    return tile


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _sample_rows(lens, rng, n=2000):
    rows = len(lens)
    pick = [rng.choice(rows, size=min(n, rows), replace=False), np.argsort(lens)[-50:]]
    empty = np.flatnonzero(lens == 0)
    if empty.size:
        pick.append(empty[:20])
    return np.unique(np.concatenate(pick)).astype(np.int64)


def test_uniform_4096_n32_full():
    G.note("full uniform 4096 N=32")
    A = synth.uniform_csr(4096, 4096, 16, seed=1)
    B = synth.dense(4096, 32, synth.streams(1)[2])
    tile = G.make_tile([A])
    got = G.host_f32(G.fwd(tile, [G.dense_dev(B)]))
    ref, S = G.oracle_fwd([A], [B])
    st = G.assert_fp32_close(got, ref, S, G.row_terms([A]))
    print("uniform4096 N=32:", st)


def test_rmat22_rowblock0_kloop_n128():
    """One GPU's share of a 4x4 stationary-C SpMM: row block 0, 4 k-tiles, N = 128."""
    t0 = time.time()
    g = synth.rmat_row_block(22, 16, 4, 0, seed=2)
    G.note("full rmat22 row block 0 (generated in %.0f s)" % (time.time() - t0))
    rs = synth.streams(2)
    Bs = [synth.dense(t.cols, 128, rs[2]) for t in g.tiles]
    tile = _bench_tile("rmat22_rowblock0_4x4_n128", g.tiles, 128)
    st = tile.stats()
    assert st["nnz_total"] == sum(t.nnz for t in g.tiles)
    Bd = [G.dense_dev(b) for b in Bs]
    C = G.fwd(tile, Bd)
    lens = G.row_terms(g.tiles)
    rows = _sample_rows(lens, _rng(21))
    got = C[torch.from_numpy(rows).to(C.device)].cpu().numpy()
    ref, S = G.oracle_fwd(g.tiles, Bs, rows=rows)
    res = G.assert_fp32_close(got, ref, S, lens[rows], what="rmat22")
    print("rmat22 k-loop:", res, "sampled rows", rows.size, "imbalance", g.imbalance)
    # Algorithm 2's k offset: another order gives a result within the same bound.
    C2 = G.fwd(tile, Bd, k_offset=3)[torch.from_numpy(rows).to(C.device)].cpu().numpy()
    ref2, S2 = G.oracle_fwd(g.tiles, Bs, k_offset=3, rows=rows)
    G.assert_fp32_close(C2, ref2, S2, lens[rows], what="rmat22 offset 3")


@pytest.fixture(scope="module")
def powerlaw2m():
    t0 = time.time()
    A = synth.powerlaw_csr(1 << 21, 1 << 21, 32, 65536, seed=3)
    rs = synth.streams(3)
    B = synth.dense(A.cols, 128, rs[2], "normal")
    dC = synth.dense(A.rows, 128, rs[3], "normal")
    G.note("full powerlaw 2M generated in %.0f s" % (time.time() - t0))
    rp, ci, va, _ = G.to_dev(A)
    tile = _bench_tile("powerlaw2m_n128_fwdbwd", [A], 128, transpose=True, dev_tiles=[(rp, ci, va, A.cols)])
    return A, B, dC, tile, va


def test_powerlaw2m_transpose_bit_exact(powerlaw2m):
    A, B, dC, tile, va = powerlaw2m
    G.note("full powerlaw 2M transpose")
    rpT, ciT, perm = ops.spmm_tile_export_transpose(tile)
    torch.cuda.synchronize()
    r = oracle.transpose(A.rowptr, A.colind, A.cols)
    assert np.array_equal(rpT.cpu().numpy(), r[0])
    assert np.array_equal(ciT.cpu().numpy(), r[1])
    assert np.array_equal(perm.cpu().numpy(), r[2])


def test_powerlaw2m_fwd_bwd_sampled(powerlaw2m):
    A, B, dC, tile, va = powerlaw2m
    G.note("full powerlaw 2M fwd+bwd sampled")
    Bd, dCd = G.dense_dev(B), G.dense_dev(dC)
    C = G.fwd(tile, [Bd])
    dA, dB = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    rng = _rng(31)
    lens = A.row_lengths()
    rows = _sample_rows(lens, rng)
    ref, S = G.oracle_fwd([A], [B], rows=rows)
    G.assert_fp32_close(C[torch.from_numpy(rows).to(C.device)].cpu().numpy(), ref, S, lens[rows], what="C")
    ents = np.unique(np.concatenate([rng.choice(A.nnz, 1000, replace=False),
                                     np.arange(A.rowptr[np.argmax(lens)], A.rowptr[np.argmax(lens)] + 50)]))
    rA, SA = oracle.sddmm(A.rowptr, A.colind, dC, B, entries=ents.astype(np.int64))
    gotA = dA[torch.from_numpy(ents).to(dA.device)].cpu().numpy()
    st = compare.fp32_stats(gotA, rA, SA, n_terms=np.full(ents.size, 128))
    assert compare.fp32_ok(st), st
    cnt = np.bincount(A.colind, minlength=A.cols)
    cols = np.unique(np.concatenate([rng.choice(A.cols, 1000, replace=False), np.argsort(cnt)[-20:]]))
    rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC, out_rows=cols.astype(np.int64))
    gotB = dB[torch.from_numpy(cols).to(dB.device)].cpu().numpy()
    G.assert_fp32_close(gotB, rB, SB, cnt[cols], what="dB")


def test_powerlaw2m_n512_windowed_backward_sampled(powerlaw2m):
    """The heavy-tailed matrix at N = 512 with the library's default shapes, as the bench's
    N = 512 workload runs it: the fused backward in two 256-column windows (partial dot
    products summed by a second kernel) and the row-split forward; sampled C, dA and dB
    against the FP64 oracle."""
    A, _, _, tile, _ = powerlaw2m
    G.note("full powerlaw 2M N=512 windowed backward sampled")
    N = 512
    rs = synth.streams(5)
    B = synth.dense(A.cols, N, rs[2], "normal")
    dC = synth.dense(A.rows, N, rs[3], "normal")
    Bd, dCd = G.dense_dev(B), G.dense_dev(dC)
    C = G.fwd(tile, [Bd])
    dA, dB = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    rng = _rng(37)
    lens = A.row_lengths()
    rows = _sample_rows(lens, rng)
    ref, S = G.oracle_fwd([A], [B], rows=rows)
    G.assert_fp32_close(C[torch.from_numpy(rows).to(C.device)].cpu().numpy(), ref, S, lens[rows], what="C")
    ents = np.unique(np.concatenate([rng.choice(A.nnz, 1000, replace=False),
                                     np.arange(A.rowptr[np.argmax(lens)], A.rowptr[np.argmax(lens)] + 50)]))
    rA, SA = oracle.sddmm(A.rowptr, A.colind, dC, B, entries=ents.astype(np.int64))
    gotA = dA[torch.from_numpy(ents).to(dA.device)].cpu().numpy()
    st = compare.fp32_stats(gotA, rA, SA, n_terms=np.full(ents.size, N))
    assert compare.fp32_ok(st), st
    cnt = np.bincount(A.colind, minlength=A.cols)
    cols = np.unique(np.concatenate([rng.choice(A.cols, 1000, replace=False), np.argsort(cnt)[-20:]]))
    rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC, out_rows=cols.astype(np.int64))
    gotB = dB[torch.from_numpy(cols).to(dB.device)].cpu().numpy()
    G.assert_fp32_close(gotB, rB, SB, cnt[cols], what="dB")


def test_powerlaw2m_fwd_bwd_bf16_sampled(powerlaw2m):
    """The BF16 forward + backward workload (B, C, dC, dB in BF16; dA FP32) at full size with its
    pinned shapes: C and dB within the BF16 bound, dA within the FP32 bound, on bf16(B), bf16(dC)."""
    A, B, dC, _, _ = powerlaw2m
    G.note("full powerlaw 2M fwd+bwd bf16 sampled")
    tile = _bench_tile("powerlaw2m_n128_fwdbwd_bf16", [A], 128, dtypes=(torch.bfloat16,), transpose=True)
    Bd, dCd = G.dense_dev(B, torch.bfloat16), G.dense_dev(dC, torch.bfloat16)
    C = G.fwd(tile, [Bd])
    dA, dB = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    Bt, dCt = G.bf16_as_f32(B), G.bf16_as_f32(dC)
    rng = _rng(33)
    lens = A.row_lengths()
    rows = _sample_rows(lens, rng)
    ref, S = G.oracle_fwd([A], [Bt], rows=rows)
    G.assert_bf16_close(C[torch.from_numpy(rows).to(C.device)].float().cpu().numpy(), ref, S, what="C bf16")
    ents = np.unique(np.concatenate([rng.choice(A.nnz, 1000, replace=False),
                                     np.arange(A.rowptr[np.argmax(lens)], A.rowptr[np.argmax(lens)] + 50)]))
    rA, SA = oracle.sddmm(A.rowptr, A.colind, dCt, Bt, entries=ents.astype(np.int64))
    st = compare.fp32_stats(dA[torch.from_numpy(ents).to(dA.device)].cpu().numpy(), rA, SA,
                            n_terms=np.full(ents.size, 128))
    assert compare.fp32_ok(st), st
    cnt = np.bincount(A.colind, minlength=A.cols)
    cols = np.unique(np.concatenate([rng.choice(A.cols, 1000, replace=False), np.argsort(cnt)[-20:]]))
    rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dCt, out_rows=cols.astype(np.int64))
    G.assert_bf16_close(dB[torch.from_numpy(cols).to(dB.device)].float().cpu().numpy(), rB, SB, what="dB bf16")
    del tile


def test_powerlaw2m_finite_differences(powerlaw2m):
    """1,000 sampled entries of dA and 1,000 of dB against central differences (h = 1, exact for a
    linear map up to the forward's rounding)."""
    A, B, dC, tile, va = powerlaw2m
    G.note("full powerlaw 2M finite differences")
    Bd, dCd = G.dense_dev(B), G.dense_dev(dC)
    dA, dB = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    rng = _rng(32)
    lens = A.row_lengths()
    top = int(np.argmax(lens))
    ps = rng.choice(A.nnz, size=1000, replace=False)
    ps[:10] = A.rowptr[top] + np.arange(10)
    rowid = np.repeat(np.arange(A.rows), lens)
    rows = rowid[ps]
    _, SC = G.oracle_fwd([A], [B], rows=np.unique(rows).astype(np.int64))
    SC = dict(zip(np.unique(rows).tolist(), SC))
    _, SA = oracle.sddmm(A.rowptr, A.colind, dC, B, entries=ps.astype(np.int64))
    dAh = dA[torch.from_numpy(ps).to(dA.device)].double().cpu().numpy()
    C = torch.empty(A.rows, 128, device=Bd.device)
    worst = 0.0
    for t, p in enumerate(ps):
        i = int(rows[t])
        v0 = va[p].item()
        va[p] = v0 + 1.0
        Cp = ops.spmm_fwd(tile, [Bd], C=C)[i].double().cpu().numpy()
        va[p] = v0 - 1.0
        Cm = ops.spmm_fwd(tile, [Bd], C=C)[i].double().cpu().numpy()
        va[p] = v0
        fd = float(np.dot(dC[i].astype(np.float64), (Cp - Cm) / 2.0))
        bound = 1e-5 * (float(np.dot(np.abs(dC[i]), SC[i])) + SA[t])
        worst = max(worst, abs(fd - dAh[t]) / bound)
        assert abs(fd - dAh[t]) <= bound, (p, fd, dAh[t], bound)
    cnt = np.bincount(A.colind, minlength=A.cols)
    js = rng.choice(A.cols, size=1000, replace=True)
    js[:5] = np.argsort(cnt)[-5:]
    ns = rng.integers(0, 128, size=1000)
    _, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC, out_rows=np.unique(js).astype(np.int64))
    SB = dict(zip(np.unique(js).tolist(), SB))
    order = np.argsort(A.colind, kind="stable")
    starts = np.concatenate([[0], np.cumsum(cnt)])
    worst_b = 0.0
    for j, n in zip(js, ns):
        j, n = int(j), int(n)
        b0 = Bd[j, n].item()
        Bd[j, n] = b0 + 1.0
        Cp = ops.spmm_fwd(tile, [Bd], C=C)[:, n].double()
        Bd[j, n] = b0 - 1.0
        Cm = ops.spmm_fwd(tile, [Bd], C=C)[:, n].double()
        Bd[j, n] = b0
        fd = float((dCd[:, n].double() * (Cp - Cm)).sum().item() / 2.0)
        rows_j = rowid[order[starts[j]:starts[j + 1]]].astype(np.int64)
        _, Sx = G.oracle_fwd([A], [B], rows=rows_j)
        bound = 1e-5 * (float(np.dot(np.abs(dC[rows_j, n]), Sx[:, n])) + SB[j][n])
        got = dB[j, n].item()
        worst_b = max(worst_b, abs(fd - got) / max(bound, 1e-300))
        assert abs(fd - got) <= bound + 1e-30, (j, n, fd, got, bound)
    print("finite differences: worst |fd - dA|/bound %.3g, worst |fd - dB|/bound %.3g" % (worst, worst_b))


def test_rmat23_n256_bf16_and_f32():
    """BF16 B and C with FP32 accumulation next to the FP32 path on the same inputs."""
    t0 = time.time()
    A = synth.rmat_csr(23, 32, seed=5)
    B = synth.dense(A.cols, 256, synth.streams(5)[2])
    G.note("full rmat23 N=256 generated in %.0f s (nnz %d)" % (time.time() - t0, A.nnz))
    tile = _bench_tile("rmat23_n256_f32", [A], 256)
    kind, lanes, vec = bench.PINNED["rmat23_n256_bf16"]["variant"]
    ops.spmm_tile_set_variant(tile, 256, torch.bfloat16, kind, lanes, vec)
    assert bench.PINNED["rmat23_n256_bf16"]["long_row"] == bench.PINNED["rmat23_n256_f32"]["long_row"]
    lens = A.row_lengths()
    rows = _sample_rows(lens, _rng(51), n=1000)
    ridx = None
    Bd = G.dense_dev(B)
    C32 = G.fwd(tile, [Bd])
    ridx = torch.from_numpy(rows).to(C32.device)
    got32 = C32[ridx].cpu().numpy()
    del C32
    ref, S = G.oracle_fwd([A], [B], rows=rows)
    st32 = G.assert_fp32_close(got32, ref, S, lens[rows], what="fp32")
    del Bd
    Bh = G.dense_dev(B, torch.bfloat16)
    C16 = G.fwd(tile, [Bh])
    got16 = C16[ridx].float().cpu().numpy()
    Bt = G.bf16_as_f32(B)
    reft, St = G.oracle_fwd([A], [Bt], rows=rows)
    st16 = G.assert_bf16_close(got16, reft, St, what="bf16 kernel-only")
    total = compare.relative_stats(got16, ref, S)
    print("rmat23 fp32:", st32)
    print("rmat23 bf16 vs oracle(bf16(B)):", st16)
    print("rmat23 bf16 vs oracle(B) [total error]:", total)


def test_uneven512_batched_sampled():
    """512 uneven tiles in one batched launch with autotuned per-tile variants; sampled rows of every
    tile against the oracle; the persistent hand-out gives the same bits."""
    t0 = time.time()
    tiles, Ns = synth.uneven_tiles(512, seed=4)
    G.note("full uneven512 generated in %.0f s (nnz %d)" % (time.time() - t0, sum(t.nnz for t in tiles)))
    rng = synth.streams(4)[3]
    handles, Bh, Bs, Cs = [], [], [], []
    for t, N in zip(tiles, Ns):
        b = synth.dense(t.cols, N, rng)
        Bh.append(b)
        Bs.append(G.dense_dev(b))
        Cs.append(torch.empty(t.rows, N, device=G.DEV))
        handles.append(G.make_tile([t]))
    for h, B, C in zip(handles, Bs, Cs):
        ops.spmm_tile_autotune(h, [B], C, tune_plan=False)
    batch = ops.spmm_batch_create(handles, Ns)
    ops.spmm_batched(batch, Bs, Cs)
    torch.cuda.synchronize()
    sel = _rng(41)
    worst = 0.0
    for t, (A, N) in enumerate(zip(tiles, Ns)):
        rows = np.unique(np.concatenate([sel.choice(A.rows, size=8, replace=False), [0, A.rows - 1]])).astype(np.int64)
        got = Cs[t][torch.from_numpy(rows).to(G.DEV)].cpu().numpy()
        ref, S = G.oracle_fwd([A], [Bh[t]], rows=rows)
        st = G.assert_fp32_close(got, ref, S, A.row_lengths()[rows], what="tile %d %s" % (t, batch.variant(t)))
        worst = max(worst, st["max_rel_to_scale"])
    print("uneven512 batched: worst |err|/S over sampled rows %.3g" % worst)
    flat = [c.clone() for c in Cs]
    for kw in (dict(persistent=True), dict(single=True), dict(single=True, persistent=True)):
        G.note("uneven512 batched %s" % kw)
        pb = ops.spmm_batch_create(handles, Ns, **kw)
        for c in Cs:
            c.fill_(float("nan"))
        ops.spmm_batched(pb, Bs, Cs, workspace=pb.workspace())
        torch.cuda.synchronize()
        for t, (c, f) in enumerate(zip(Cs, flat)):
            assert torch.equal(c, f), (t, kw)
        del pb
