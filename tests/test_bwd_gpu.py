"""Backward parity: transposed structure (bit-exact), SDDMM dA and dB = A^T dC against
the FP64 oracle, the autograd Function, and finite differences."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import compare
from paper_2311_18141_amd import ops
from paper_2311_18141_amd.autograd import SpMMFunction

import gpu_util as G

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _case(name):
    rng = _rng(hash(name) % 1000)
    if name == "empty":
        return synth.CSR(7, 5, np.zeros(8, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    if name == "one_col":
        L = rng.integers(0, 2, size=300)
        return synth.random_csr(300, 1, L, rng)
    if name == "one_row":
        return synth.random_csr(1, 5000, np.array([4000]), rng)
    if name == "hot_column":
        L = rng.integers(0, 30, size=20000)
        A = synth.random_csr(20000, 700, L, rng)
        return A
    if name == "powerlaw":
        return synth.powerlaw_csr(1 << 15, 1 << 15, 32, 8192, seed=5)
    if name == "wide":
        L = rng.integers(0, 12, size=4000)
        return synth.random_csr(4000, 1 << 20, L, rng)
    if name == "rmat":
        return synth.rmat_row_block(13, 16, 2, 0, seed=6).tiles[0]
    raise KeyError(name)


CASES = ["empty", "one_col", "one_row", "hot_column", "powerlaw", "wide", "rmat"]


@pytest.mark.parametrize("name", CASES)
def test_transpose_bit_exact(name):
    G.note("transpose %s" % name)
    A = _case(name)
    tile = G.make_tile([A], transpose=True)
    rpT, ciT, perm = ops.spmm_tile_export_transpose(tile)
    torch.cuda.synchronize()
    r_rpT, r_ciT, r_perm = oracle.transpose(A.rowptr, A.colind, A.cols)
    assert np.array_equal(rpT.cpu().numpy(), r_rpT)
    assert np.array_equal(ciT.cpu().numpy(), r_ciT)
    assert np.array_equal(perm.cpu().numpy(), r_perm)


@pytest.mark.parametrize("name", CASES)
@pytest.mark.parametrize("N", [32, 128])
def test_backward_vs_oracle(name, N):
    G.note("backward %s N=%d" % (name, N))
    A = _case(name)
    rng = _rng(N + len(name))
    B = synth.dense(A.cols, N, rng, "normal")
    dC = synth.dense(A.rows, N, rng, "normal")
    tile = G.make_tile([A], transpose=True, long_row=512, segment=256)
    dA, dB = ops.spmm_bwd(tile, G.dense_dev(dC), G.dense_dev(B))
    torch.cuda.synchronize()
    rA, SA = oracle.sddmm(A.rowptr, A.colind, dC, B)
    st = compare.fp32_stats(dA.cpu().numpy(), rA, SA, n_terms=np.full(A.nnz, N))
    assert compare.fp32_ok(st), st
    rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC)
    cnt = np.bincount(A.colind, minlength=A.cols)
    G.assert_fp32_close(G.host_f32(dB), rB, SB, cnt, what="dB")


@pytest.mark.parametrize("bwd_slice", [0, 16, 32])
@pytest.mark.parametrize("split", [False, True])
def test_backward_integer_exact(split, bwd_slice):
    G.note("backward_integer_exact split=%s slice=%d" % (split, bwd_slice))
    rng = _rng(90 + split)
    M, K, N = 5000, 3000, 64
    L = rng.integers(0, 40, size=M)
    L[[10, 20]] = [2900, 1500]
    A = synth.random_csr(M, K, L, rng, "int8")
    B = synth.dense(K, N, rng, "int8")
    dC = synth.dense(M, N, rng, "int8")
    kw = dict(long_row=8, segment=4) if split else {}
    tile = G.make_tile([A], transpose=True, bwd_slice=bwd_slice, **kw)
    dA, dB = ops.spmm_bwd(tile, G.dense_dev(dC), G.dense_dev(B))
    torch.cuda.synchronize()
    rA, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    rB, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, K, dC)
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), rA)
    assert np.array_equal(dB.cpu().numpy().astype(np.float64), rB)


def test_autograd_function():
    G.note("autograd_function")
    rng = _rng(95)
    A = synth.powerlaw_csr(4096, 3000, 16, 1024, seed=11)
    B = synth.dense(A.cols, 64, rng, "normal")
    dC = synth.dense(A.rows, 64, rng, "normal")
    rp, ci, va, _ = G.to_dev(A)
    tile = ops.spmm_tile_create(A.rows, [(rp, ci, va, A.cols)], validate=True, transpose=True)
    values = va.requires_grad_(True)
    Bt = G.dense_dev(B).requires_grad_(True)
    C = SpMMFunction.apply(values, Bt, tile)
    C.backward(G.dense_dev(dC))
    rC, SC = G.oracle_fwd([A], [B])
    G.assert_fp32_close(G.host_f32(C.detach()), rC, SC, G.row_terms([A]))
    rA, SA = oracle.sddmm(A.rowptr, A.colind, dC, B)
    assert compare.fp32_ok(compare.fp32_stats(values.grad.cpu().numpy(), rA, SA))
    rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC)
    G.assert_fp32_close(G.host_f32(Bt.grad), rB, SB)
    # needs_input_grad: only B
    Bt.grad = None
    values.grad = None
    v2 = va.detach()
    C2 = SpMMFunction.apply(v2, Bt, tile)
    C2.backward(G.dense_dev(dC))
    assert values.grad is None and Bt.grad is not None


def test_finite_differences_scaled():
    """C is linear in the values and in B, so central differences with h = 1 have no truncation error."""
    G.note("finite_differences_scaled")
    rng = _rng(96)
    A = synth.powerlaw_csr(8192, 8192, 32, 2048, seed=12)
    N = 128
    B = synth.dense(A.cols, N, rng, "normal")
    dC = synth.dense(A.rows, N, rng, "normal")
    rp, ci, va, _ = G.to_dev(A)
    tile = ops.spmm_tile_create(A.rows, [(rp, ci, va, A.cols)], validate=True, transpose=True)
    Bd, dCd = G.dense_dev(B), G.dense_dev(dC)
    dA, dB = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    dA = dA.cpu().numpy().astype(np.float64)
    dB = dB.cpu().numpy().astype(np.float64)
    _, SC = G.oracle_fwd([A], [B])
    _, SA = oracle.sddmm(A.rowptr, A.colind, dC, B)
    rowid = np.repeat(np.arange(A.rows), A.row_lengths())
    ps = rng.choice(A.nnz, size=100, replace=False)
    ps[0] = A.rowptr[np.argmax(A.row_lengths())]
    for p in ps:
        i = rowid[p]
        v0 = va[p].item()
        va[p] = v0 + 1.0
        Cp = ops.spmm_fwd(tile, [Bd])[i].double().cpu().numpy()
        va[p] = v0 - 1.0
        Cm = ops.spmm_fwd(tile, [Bd])[i].double().cpu().numpy()
        va[p] = v0
        fd = float(np.dot(dC[i].astype(np.float64), (Cp - Cm) / 2.0))
        bound = 1e-5 * (float(np.dot(np.abs(dC[i]), SC[i])) + SA[p])
        assert abs(fd - dA[p]) <= bound, (p, fd, dA[p], bound)
    cnt = np.bincount(A.colind, minlength=A.cols)
    js = rng.choice(A.cols, size=40, replace=False)
    js[0] = int(np.argmax(cnt))
    _, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC, out_rows=js.astype(np.int64))
    for t, j in enumerate(js):
        n = int(rng.integers(0, N))
        b0 = Bd[j, n].item()
        Bd[j, n] = b0 + 1.0
        Cp = ops.spmm_fwd(tile, [Bd])[:, n].double()
        Bd[j, n] = b0 - 1.0
        Cm = ops.spmm_fwd(tile, [Bd])[:, n].double()
        Bd[j, n] = b0
        fd = float((dCd[:, n].double() * (Cp - Cm)).sum().item() / 2.0)
        rows_j = rowid[A.colind == j]
        bound = 1e-5 * (float(np.dot(np.abs(dC[rows_j, n]), SC[rows_j, n])) + SB[t, n])
        assert abs(fd - dB[j, n]) <= bound + 1e-30, (j, n, fd, dB[j, n], bound)


@pytest.mark.parametrize("N", [1, 12, 64, 136])
@pytest.mark.parametrize("lanes,per_group", [(4, 1), (4, 4), (8, 8), (16, 2), (32, 4), (64, 8)])
def test_sddmm_variants_integer_exact(lanes, per_group, N):
    """Every SDDMM shape gives the exact dA on integer data, ragged nnz and columns included."""
    G.note("sddmm_variant lanes=%d per_group=%d N=%d" % (lanes, per_group, N))
    rng = _rng(300 + N)
    M, K = 777, 901
    L = rng.integers(0, 23, size=M)
    L[5] = 900
    A = synth.random_csr(M, K, L, rng, "int8")
    B = synth.dense(K, N, rng, "int8")
    dC = synth.dense(M, N, rng, "int8")
    tile = G.make_tile([A], transpose=True)
    ops.spmm_tile_set_sddmm_variant(tile, N, lanes, per_group)
    dA, _ = ops.spmm_bwd(tile, G.dense_dev(dC), G.dense_dev(B), want_dB=False)
    torch.cuda.synchronize()
    rA, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), rA)


def test_sddmm_variant_argument_errors():
    G.note("sddmm_variant_argument_errors")
    A = synth.random_csr(10, 10, np.full(10, 3), _rng(1))
    tile = G.make_tile([A], transpose=True)
    for lanes, per_group in [(3, 1), (128, 1), (8, 3), (8, 16), (4, 8)]:
        with pytest.raises(ops.SpmmError):
            ops.spmm_tile_set_sddmm_variant(tile, 32, lanes, per_group)
    with pytest.raises(ops.SpmmError):
        ops.spmm_tile_set_sddmm_variant(tile, 0, 8, 4)
    ops.spmm_tile_set_sddmm_variant(tile, 32, 0)   # clearing an absent entry is fine


@pytest.mark.parametrize("name", ["powerlaw", "hot_column", "rmat"])
def test_backward_bf16_vs_oracle(name):
    """BF16 dC and B (the backward of a BF16 forward): dA in FP32 within the FP32 bound of the
    oracle on bf16(dC), bf16(B); dB rounded once to BF16, within the BF16 bound."""
    G.note("backward bf16 %s" % name)
    A = _case(name)
    rng = _rng(41 + len(name))
    N = 128
    B = synth.dense(A.cols, N, rng, "normal")
    dC = synth.dense(A.rows, N, rng, "normal")
    tile = G.make_tile([A], transpose=True)
    dA, dB = ops.spmm_bwd(tile, G.dense_dev(dC, torch.bfloat16), G.dense_dev(B, torch.bfloat16))
    torch.cuda.synchronize()
    assert dA.dtype == torch.float32 and dB.dtype == torch.bfloat16
    Bt, dCt = G.bf16_as_f32(B), G.bf16_as_f32(dC)
    rA, SA = oracle.sddmm(A.rowptr, A.colind, dCt, Bt)
    st = compare.fp32_stats(dA.cpu().numpy(), rA, SA, n_terms=np.full(A.nnz, N))
    assert compare.fp32_ok(st), st
    rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dCt)
    G.assert_bf16_close(dB.float().cpu().numpy(), rB, SB, what="dB bf16")


def test_backward_bf16_integer_exact():
    """Integer data: dA exact; dB equals the exact sum rounded once to BF16 (round to nearest even)."""
    G.note("backward bf16 integer exact")
    rng = _rng(43)
    M, K, N = 3000, 2500, 64
    L = rng.integers(0, 30, size=M)
    L[7] = 2400
    A = synth.random_csr(M, K, L, rng, "int8")
    B = synth.dense(K, N, rng, "int8")
    dC = synth.dense(M, N, rng, "int8")
    tile = G.make_tile([A], transpose=True, long_row=64, segment=16)
    dA, dB = ops.spmm_bwd(tile, G.dense_dev(dC, torch.bfloat16), G.dense_dev(B, torch.bfloat16))
    torch.cuda.synchronize()
    rA, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), rA)
    rB, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, K, dC)
    assert np.abs(rB).max() < 2 ** 24          # exact in FP32 before the one rounding
    want = oracle.f32_to_bf16(rB.astype(np.float32))
    got = dB.cpu().view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(got, want)


def test_autograd_bf16():
    G.note("autograd bf16")
    rng = _rng(44)
    A = synth.powerlaw_csr(4096, 3000, 16, 1024, seed=21)
    B = synth.dense(A.cols, 64, rng, "normal")
    dC = synth.dense(A.rows, 64, rng, "normal")
    rp, ci, va, _ = G.to_dev(A)
    tile = ops.spmm_tile_create(A.rows, [(rp, ci, va, A.cols)], validate=True, transpose=True)
    values = va.requires_grad_(True)
    Bt = G.dense_dev(B, torch.bfloat16).requires_grad_(True)
    C = SpMMFunction.apply(values, Bt, tile)
    assert C.dtype == torch.bfloat16
    C.backward(G.dense_dev(dC, torch.bfloat16))
    assert values.grad.dtype == torch.float32 and Bt.grad.dtype == torch.bfloat16
    Btf, dCt = G.bf16_as_f32(B), G.bf16_as_f32(dC)
    rA, SA = oracle.sddmm(A.rowptr, A.colind, dCt, Btf)
    assert compare.fp32_ok(compare.fp32_stats(values.grad.cpu().numpy(), rA, SA))
    rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dCt)
    G.assert_bf16_close(Bt.grad.float().cpu().numpy(), rB, SB, what="dB")


BWD_VARIANTS = [("stream", 64, 1), ("stream", 64, 2), ("stream", 16, 4), ("rowsplit", 8, 4), ("rowsplit", 16, 4),
                ("rowsplit", 32, 2), ("rowsplit", 64, 2), ("rowsplit", 64, 1)]


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("variant", BWD_VARIANTS)
def test_dB_variants_integer_exact(variant, dtype):
    """Every kernel variant of the dB pass (forward kernels over the transpose, split rows
    included) gives the exact integer sum (rounded once to BF16 for a BF16 dB)."""
    kind, lanes, vec = variant
    G.note("dB variant %s %s" % (variant, dtype))
    rng = _rng(95)
    M, K, N = 4000, 2000, 64
    L = rng.integers(0, 24, size=M)
    A = synth.random_csr(M, K, L, rng, "int8")
    hub = rng.choice(M, size=300, replace=False)          # column 5 is used by 300 rows: split in A^T
    cols = [np.union1d(A.colind[A.rowptr[i]:A.rowptr[i + 1]], [5]) if i in set(hub) else
            A.colind[A.rowptr[i]:A.rowptr[i + 1]] for i in range(M)]
    lengths = np.array([len(c) for c in cols])
    A = synth.CSR(M, K, synth.rowptr_from_lengths(lengths), np.concatenate(cols).astype(np.int32),
                  rng.integers(-8, 9, size=int(lengths.sum())).astype(np.float32))
    B = synth.dense(K, N, rng, "int8")
    dC = synth.dense(M, N, rng, "int8")
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    tile = G.make_tile([A], transpose=True, long_row=128, segment=32)
    assert tile.stats()["long_rows_t"] > 0
    ops.spmm_tile_set_bwd_variant(tile, N, tdt, kind, lanes, vec)
    _, dB = ops.spmm_bwd(tile, G.dense_dev(dC, tdt), G.dense_dev(B, tdt), want_dA=False)
    torch.cuda.synchronize()
    rB, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, K, dC)
    if dtype == "f32":
        assert np.array_equal(dB.cpu().numpy().astype(np.float64), rB)
    else:
        assert np.abs(rB).max() < 2 ** 24
        got = dB.cpu().view(torch.int16).numpy().view(np.uint16)
        assert np.array_equal(got, oracle.f32_to_bf16(rB.astype(np.float32)))


@pytest.mark.parametrize("N", [128, 384])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_autotune_bwd(dtype, N):
    """The dB-pass autotuner keeps a variant; the backward then still matches the oracle (at
    N = 384 the fused candidates include column windows)."""
    G.note("autotune dB %s N=%d" % (dtype, N))
    rng = _rng(96)
    A = synth.powerlaw_csr(1 << 14, 1 << 14, 16, 4096, seed=9)
    A = synth.CSR(A.rows, A.cols, A.rowptr, A.colind, rng.integers(-8, 9, size=A.nnz).astype(np.float32))
    B = synth.dense(A.cols, N, rng, "int8")
    dC = synth.dense(A.rows, N, rng, "int8")
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    tile = G.make_tile([A], transpose=True)
    dCd, Bd = G.dense_dev(dC, tdt), G.dense_dev(B, tdt)
    chosen = ops.spmm_tile_autotune_bwd(tile, dCd)
    assert chosen["kind"] in ("stream", "rowsplit") and chosen["vec"] >= 1
    # with B the whole backward is timed, fused shapes included
    chosen_full = ops.spmm_tile_autotune_bwd(tile, dCd, B=Bd)
    assert chosen_full["kind"] in ("stream", "rowsplit", "fused") and chosen_full["vec"] >= 1
    assert ops.spmm_tile_get_variant(tile, N, tdt, bwd=True) == chosen_full
    dA, dB = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    rA, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    rB, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC)
    assert np.array_equal(dA.cpu().numpy().astype(np.float64), rA)
    if dtype == "f32":
        assert np.array_equal(dB.cpu().numpy().astype(np.float64), rB)
    else:
        got = dB.cpu().view(torch.int16).numpy().view(np.uint16)
        assert np.array_equal(got, oracle.f32_to_bf16(rB.astype(np.float32)))
    ops.spmm_tile_set_bwd_variant(tile, N, tdt, None)          # cleared: the library rule again
    dA2, dB2 = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    assert torch.equal(dA, dA2) and torch.equal(dB, dB2)


FUSED_SHAPES = {"f32": [(4, 1), (8, 2), (16, 4), (32, 2), (64, 1), (64, 4)],
                "bf16": [(8, 1), (4, 2), (8, 8), (16, 4), (32, 2), (32, 4), (64, 2), (64, 4), (64, 8)]}


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("N", [1, 3, 36, 64, 100, 300, 520])
def test_fused_backward_integer_exact(N, dtype):
    """The fused backward (one pass over A^T for dA and dB) at every group shape that covers N or
    needs at most ceil(N / 256) column windows, split rows of A^T included: dA and dB exact on
    integer data (dB rounded once for BF16), as the two-pass form's."""
    rng = _rng(500 + N)
    M, K = 3000, 1200
    L = rng.integers(0, 20, size=M)
    A = synth.random_csr(M, K, L, rng, "int8")
    hub = rng.choice(M, size=400, replace=False)          # column 7 is used by >= 400 rows: split in A^T
    cols = [np.union1d(A.colind[A.rowptr[i]:A.rowptr[i + 1]], [7]) if i in set(hub) else
            A.colind[A.rowptr[i]:A.rowptr[i + 1]] for i in range(M)]
    lengths = np.array([len(c) for c in cols])
    A = synth.CSR(M, K, synth.rowptr_from_lengths(lengths), np.concatenate(cols).astype(np.int32),
                  rng.integers(-8, 9, size=int(lengths.sum())).astype(np.float32))
    small = dtype == "bf16"      # BF16: |dC|, |B| <= 4 keeps every dot product exact
    B = synth.dense(K, N, rng, "int8")
    dC = synth.dense(M, N, rng, "int8")
    if small:
        B, dC = np.clip(B, -4, 4), np.clip(dC, -4, 4)
    tdt = torch.float32 if dtype == "f32" else torch.bfloat16
    tile = G.make_tile([A], transpose=True, long_row=128, segment=32)
    assert tile.stats()["long_rows_t"] > 0
    rA, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    rB, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, K, dC)
    assert np.abs(rB).max() < 2 ** 24 and np.abs(rA).max() < 2 ** 24
    want_B = (rB if dtype == "f32" else oracle.f32_to_bf16(rB.astype(np.float32)))
    Bd, dCd = G.dense_dev(B, tdt), G.dense_dev(dC, tdt)
    ops.spmm_tile_set_bwd_variant(tile, N, tdt, "rowsplit", 0, 0)
    _, dB_two = ops.spmm_bwd(tile, dCd, Bd)
    ran = 0
    for lanes, vec in FUSED_SHAPES[dtype]:
        if N % vec or -(-N // (lanes * vec)) > min(8, max(1, -(-N // 256))):
            continue
        for depth in (1, 2, 4, 8):
            if depth > lanes:
                continue
            G.note("fused backward N=%d %s lanes=%d vec=%d depth=%d" % (N, dtype, lanes, vec, depth))
            ops.spmm_tile_set_bwd_variant(tile, N, tdt, "fused", lanes, vec, depth)
            dA, dB = ops.spmm_bwd(tile, dCd, Bd)
            torch.cuda.synchronize()
            ran += 1
            what = (lanes, vec, depth)
            assert np.array_equal(dA.cpu().numpy().astype(np.float64), rA), what
            if dtype == "f32":
                assert np.array_equal(dB.cpu().numpy().astype(np.float64), want_B), what
            else:
                assert np.array_equal(dB.cpu().view(torch.int16).numpy().view(np.uint16), want_B), what
            assert torch.equal(dB, dB_two), what
    assert ran > 0


def test_fused_variant_argument_errors():
    """depth belongs to the fused kind only: 1, 2, 4 or 8, at most the group's lanes."""
    G.note("fused variant argument errors")
    A = synth.random_csr(10, 10, np.full(10, 3), _rng(2))
    tile = G.make_tile([A], transpose=True)
    for kind, lanes, vec, depth in [("rowsplit", 16, 4, 2), ("stream", 64, 2, 4), ("fused", 16, 4, 3),
                                    ("fused", 4, 4, 8), ("fused", 16, 4, 16)]:
        with pytest.raises(ops.SpmmError):
            ops.spmm_tile_set_bwd_variant(tile, 64, torch.float32, kind, lanes, vec, depth)
    with pytest.raises(ops.SpmmError):   # the forward's table takes no fused kind
        ops.spmm_tile_set_variant(tile, 64, torch.float32, "fused", 16, 4)
    ops.spmm_tile_set_bwd_variant(tile, 64, torch.float32, "fused", 16, 4, 8)
    assert ops.spmm_tile_get_variant(tile, 64, torch.float32, bwd=True) == {"kind": "fused", "lanes": 16, "vec": 4,
                                                                             "depth": 8}


def test_fused_backward_choice():
    """Without an entry both gradients come from the fused pass, in column windows when one
    group does not cover N (260, 600); with a column slice set, or an N whose vector width
    would need windows narrower than 256 columns (258: two-element vectors), the two-pass
    form runs; every form matches the oracle."""
    G.note("fused backward choice")
    rng = _rng(510)
    A = synth.powerlaw_csr(1 << 13, 1 << 13, 16, 2048, seed=13)
    for N, slice_ in [(128, 0), (128, 32), (260, 0), (258, 0), (600, 0)]:
        B = synth.dense(A.cols, N, rng, "normal")
        dC = synth.dense(A.rows, N, rng, "normal")
        tile = G.make_tile([A], transpose=True, bwd_slice=slice_)
        Bd, dCd = G.dense_dev(B), G.dense_dev(dC)
        dA, dB = ops.spmm_bwd(tile, dCd, Bd)
        torch.cuda.synchronize()
        rA, SA = oracle.sddmm(A.rowptr, A.colind, dC, B)
        st = compare.fp32_stats(dA.cpu().numpy(), rA, SA, n_terms=np.full(A.nnz, N))
        assert compare.fp32_ok(st), (N, slice_, st)
        rB, SB = oracle.spmm_t(A.rowptr, A.colind, A.values, A.cols, dC)
        G.assert_fp32_close(G.host_f32(dB), rB, SB, np.bincount(A.colind, minlength=A.cols), what="dB")


@pytest.mark.parametrize("form", ["fused", "fused_windows", "two_pass"])
def test_backward_deterministic_and_graph_replay(form):
    """spmm_bwd (split rows of A^T included) gives the same bits on every call, and a captured
    HIP graph of it, replayed with unrelated eager work between replays and its outputs poisoned
    before each, reproduces the eager result every time (the fused form in column windows too:
    its partial dot products summed by a second kernel)."""
    G.note("backward graph replay %s" % form)
    rng = _rng(520)
    M, K = 6000, 900
    N = 384 if form == "fused_windows" else 128
    A = synth.random_csr(M, K, rng.integers(0, 40, size=M), rng, "normal")
    tile = G.make_tile([A], transpose=True, long_row=128, segment=64)
    assert tile.stats()["long_rows_t"] > 0
    if form == "fused":
        ops.spmm_tile_set_bwd_variant(tile, N, torch.float32, "fused", 32, 4, 4)
    elif form == "fused_windows":
        ops.spmm_tile_set_bwd_variant(tile, N, torch.float32, "fused", 64, 4, 4)   # 2 windows of 256
    else:
        ops.spmm_tile_set_bwd_variant(tile, N, torch.float32, "rowsplit", 0, 0)
    Bd = G.dense_dev(synth.dense(K, N, rng, "normal"))
    dCd = G.dense_dev(synth.dense(M, N, rng, "normal"))
    dA1, dB1 = ops.spmm_bwd(tile, dCd, Bd)
    dA1, dB1 = dA1.clone(), dB1.clone()
    dA2, dB2 = ops.spmm_bwd(tile, dCd, Bd)
    torch.cuda.synchronize()
    assert torch.equal(dA1, dA2) and torch.equal(dB1, dB2)
    dA = torch.empty_like(dA1)
    dB = torch.empty_like(dB1)
    ws = tile.workspace(N, "bwd")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.spmm_bwd(tile, dCd, Bd, dA=dA, dB=dB, workspace=ws)      # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.spmm_bwd(tile, dCd, Bd, dA=dA, dB=dB, workspace=ws)
    for r in range(5):
        dA.fill_(float("nan"))
        dB.fill_(float("nan"))
        _ = (dCd * 2).sum()                                           # unrelated eager work
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(dA, dA1) and torch.equal(dB, dB1), r
