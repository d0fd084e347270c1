"""Pins of the FP64 oracle against things other than itself.

Each check compares the oracle with a library routine that uses a different
algorithm (NumPy dense products, SciPy sparse products and transposition, torch's
BF16 conversion), a hand-worked fixture, a closed form or an invariant of the
mathematics (identity, permutation, linearity, adjoint, k-tile decomposition).
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def dense_of(rowptr, colind, values, cols):
    """Densify a CSR tile (test-side construction, no summation involved)."""
    rows = len(rowptr) - 1
    A = np.zeros((rows, cols), dtype=np.float64)
    r = np.repeat(np.arange(rows), np.diff(np.asarray(rowptr, dtype=np.int64)))
    A[r, np.asarray(colind)] = np.asarray(values, dtype=np.float64)
    return A


def small_csr(rng, rows, cols, value_kind="pm1", max_len=None, empty_frac=0.2):
    max_len = cols if max_len is None else min(max_len, cols)
    lengths = rng.integers(0, max_len + 1, size=rows)
    lengths[rng.random(rows) < empty_frac] = 0
    return synth.random_csr(rows, cols, lengths, rng, value_kind)


# ---------------------------------------------------------------------------
# Hand-worked fixture
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(GOLDEN, "spmm_worked_example.json")) as f:
        return json.load(f)


def _tile(d):
    return (np.array(d["rowptr"], np.int32), np.array(d["colind"], np.int32), np.array(d["values"], np.float32))


def test_golden_forward(golden):
    A = _tile(golden["A"])
    B = np.array(golden["B"], np.float32)
    C, S = oracle.spmm([A], [B])
    assert np.array_equal(C, np.array(golden["C"], np.float64))
    C0 = np.array(golden["C0"], np.float32)
    Ca, _ = oracle.spmm([A], [B], accumulate=True, C0=C0)
    assert np.array_equal(Ca, np.array(golden["C_accumulate"], np.float64))
    # S is the same sum over absolute values: row 0 = 2*|[3,4]| + 1*|[7,8]|
    assert np.array_equal(S[0], np.array([13.0, 16.0]))
    assert np.array_equal(S[1], np.zeros(2))


def test_golden_k_tiles(golden):
    kt = golden["k_tiles"]
    tiles = [_tile(t) for t in kt["tiles"]]
    Bs = [np.array(b, np.float32) for b in kt["B"]]
    for off in range(4):
        C, _ = oracle.spmm(tiles, Bs, k_offset=off)
        assert np.array_equal(C, np.array(golden["C"], np.float64)), off


def test_golden_backward(golden):
    rp, ci, va = _tile(golden["A"])
    B = np.array(golden["B"], np.float32)
    dC = np.array(golden["dC"], np.float32)
    dA, _ = oracle.sddmm(rp, ci, dC, B)
    assert np.array_equal(dA, np.array(golden["dA"], np.float64))
    dB, _ = oracle.spmm_t(rp, ci, va, 4, dC)
    assert np.array_equal(dB, np.array(golden["dB"], np.float64))
    rpT, ciT, perm = oracle.transpose(rp, ci, 4)
    t = golden["transpose"]
    assert rpT.tolist() == t["rowptrT"] and ciT.tolist() == t["colindT"] and perm.tolist() == t["perm"]
    C, _ = oracle.spmm([(rp, ci, va)], [B])
    assert float((C * dC).sum()) == golden["adjoint_value"]
    assert float((va.astype(np.float64) * dA).sum()) == golden["adjoint_value"]
    assert float((dB * B).sum()) == golden["adjoint_value"]


def test_golden_bf16(golden):
    cases = golden["bf16_rne"]["cases"]
    x = np.array([int(a, 16) for a, _ in cases], dtype=np.uint32).view(np.float32)
    want = np.array([int(b, 16) for _, b in cases], dtype=np.uint16)
    assert np.array_equal(oracle.f32_to_bf16(x), want)


# ---------------------------------------------------------------------------
# Dense and sparse library cross-checks
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rows,cols,N,seed", [(1, 1, 1, 0), (7, 5, 3, 1), (64, 64, 64, 2), (33, 17, 1, 3),
                                              (50, 40, 32, 4), (3, 64, 65, 5)])
def test_spmm_vs_dense(rows, cols, N, seed):
    rng = _rng(seed)
    A = small_csr(rng, rows, cols)
    B = synth.dense(cols, N, rng)
    C, S = oracle.spmm([(A.rowptr, A.colind, A.values)], [B])
    ref = dense_of(A.rowptr, A.colind, A.values, cols) @ B.astype(np.float64)
    Sref = np.abs(dense_of(A.rowptr, A.colind, A.values, cols)) @ np.abs(B.astype(np.float64))
    assert np.all(np.abs(C - ref) <= 1e-12 * Sref)
    assert np.allclose(S, Sref, rtol=1e-12, atol=0)


def test_spmm_brute_force_3x3():
    """All 2^9 patterns of a 3x3 tile with small-integer values: exact against dense products."""
    rng = _rng(7)
    B = rng.integers(-4, 5, size=(3, 3)).astype(np.float32)
    for mask in range(512):
        pat = np.array([(mask >> b) & 1 for b in range(9)], dtype=bool).reshape(3, 3)
        vals = rng.integers(-4, 5, size=9).astype(np.float32).reshape(3, 3)
        vals[vals == 0] = 1
        r, c = np.nonzero(pat)
        rowptr = np.concatenate([[0], np.cumsum(pat.sum(1))]).astype(np.int32)
        C, _ = oracle.spmm([(rowptr, c.astype(np.int32), vals[r, c])], [B])
        ref = np.where(pat, vals, 0).astype(np.float64) @ B.astype(np.float64)
        assert np.array_equal(C, ref), mask


@pytest.mark.parametrize("seed", [11, 12])
def test_spmm_vs_scipy(seed):
    rng = _rng(seed)
    A = small_csr(rng, 3000, 2500, max_len=40)
    B = synth.dense(2500, 48, rng, "normal")
    C, S = oracle.spmm([(A.rowptr, A.colind, A.values)], [B])
    M = sp.csr_matrix((A.values.astype(np.float64), A.colind, A.rowptr), shape=(A.rows, A.cols))
    ref = M @ B.astype(np.float64)
    assert np.all(np.abs(C - ref) <= 1e-12 * S + 1e-300)


def test_spmm_row_subset_and_leading_dims():
    rng = _rng(13)
    A = small_csr(rng, 400, 300, max_len=30)
    Bfull = synth.dense(300, 80, rng)
    B = Bfull[:, 5:69]                     # leading dimension 80, N = 64
    C, S = oracle.spmm([(A.rowptr, A.colind, A.values)], [B])
    rows = np.array([399, 0, 17, 17, 250], dtype=np.int64)
    Cs, Ss = oracle.spmm([(A.rowptr, A.colind, A.values)], [B], rows=rows)
    assert np.array_equal(Cs, C[rows]) and np.array_equal(Ss, S[rows])
    ref = dense_of(A.rowptr, A.colind, A.values, 300) @ np.ascontiguousarray(B).astype(np.float64)
    assert np.all(np.abs(C - ref) <= 1e-12 * S)


def test_spmm_accumulate():
    rng = _rng(14)
    A = small_csr(rng, 100, 90, max_len=20)
    B = synth.dense(90, 16, rng)
    C0 = synth.dense(100, 16, rng)
    C, S = oracle.spmm([(A.rowptr, A.colind, A.values)], [B], accumulate=True, C0=C0)
    ref = C0.astype(np.float64) + dense_of(A.rowptr, A.colind, A.values, 90) @ B.astype(np.float64)
    assert np.all(np.abs(C - ref) <= 1e-12 * (S + np.abs(C0)))
    empty = np.diff(A.rowptr) == 0
    assert np.array_equal(C[empty], C0[empty].astype(np.float64))


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
def test_identity_and_permutation_exact():
    rng = _rng(15)
    n, N = 257, 33
    B = synth.dense(n, N, rng)
    eye = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n, np.float32))
    C, _ = oracle.spmm([eye], [B])
    assert np.array_equal(C, B.astype(np.float64))
    pi = rng.permutation(n).astype(np.int32)
    P = (np.arange(n + 1, dtype=np.int32), pi, np.ones(n, np.float32))
    C, _ = oracle.spmm([P], [B])
    assert np.array_equal(C, B[pi].astype(np.float64))
    # transpose of a permutation is its inverse
    rpT, ciT, perm = oracle.transpose(*P[:2], n)
    inv = np.empty(n, np.int64)
    inv[pi] = np.arange(n)
    assert np.array_equal(ciT, inv) and np.array_equal(perm, inv) and np.array_equal(rpT, np.arange(n + 1))
    # dB = P^T dC is an exact row permutation
    dC = synth.dense(n, N, rng)
    dB, _ = oracle.spmm_t(P[0], P[1], P[2], n, dC)
    assert np.array_equal(dB[pi], dC.astype(np.float64))
    # signed powers of two stay exact
    s = synth.draw_values(rng, n, "pow2")
    C, _ = oracle.spmm([(P[0], P[1], s)], [B])
    assert np.array_equal(C, s[:, None].astype(np.float64) * B[pi].astype(np.float64))


def test_linearity():
    rng = _rng(16)
    A = small_csr(rng, 300, 200, max_len=25)
    B1 = synth.dense(200, 24, rng)
    B2 = synth.dense(200, 24, rng)
    alpha, beta = np.float32(0.75), np.float32(-1.25)
    Bc = alpha * B1 + beta * B2                      # exact in FP32? not necessarily: compare in FP64 scale
    t = (A.rowptr, A.colind, A.values)
    C1, S1 = oracle.spmm([t], [B1])
    C2, S2 = oracle.spmm([t], [B2])
    Cc, Sc = oracle.spmm([t], [Bc])
    ref = dense_of(*t, 200) @ Bc.astype(np.float64)
    assert np.all(np.abs(Cc - ref) <= 1e-13 * Sc + 1e-300)
    lin = float(alpha) * C1 + float(beta) * C2
    # Bc carries one FP32 rounding per entry; bound its effect by u32 * (|a|S1 + |b|S2).
    assert np.all(np.abs(Cc - lin) <= 2 ** -23 * (abs(alpha) * S1 + abs(beta) * S2) + 1e-12 * Sc)
    # (A1 + A2) B = A1 B + A2 B for disjoint patterns: split A's entries by parity of position.
    keep = (np.arange(A.nnz) % 2 == 0)
    v1 = np.where(keep, A.values, 0).astype(np.float32)
    v2 = np.where(~keep, A.values, 0).astype(np.float32)
    D1, _ = oracle.spmm([(A.rowptr, A.colind, v1)], [B1])
    D2, _ = oracle.spmm([(A.rowptr, A.colind, v2)], [B1])
    assert np.all(np.abs(D1 + D2 - C1) <= 1e-13 * S1 + 1e-300)


def test_integer_exact():
    rng = _rng(17)
    A = small_csr(rng, 500, 400, value_kind="int8", max_len=60)
    B = synth.dense(400, 40, rng, "int8")
    C, _ = oracle.spmm([(A.rowptr, A.colind, A.values)], [B])
    ref = dense_of(A.rowptr, A.colind, A.values, 400).astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(C, ref.astype(np.float64))


@pytest.mark.parametrize("grid", [2, 3, 4])
def test_k_tile_decomposition(grid):
    """Section 2.1: C_i = sum_k A_ik B_k over column tiles equals the untiled product, for every k offset."""
    rng = _rng(18 + grid)
    cols = 301
    A = small_csr(rng, 120, cols, max_len=50)
    B = synth.dense(cols, 20, rng, "int8")
    Aint = synth.CSR(A.rows, A.cols, A.rowptr, A.colind, synth.draw_values(rng, A.nnz, "int8"))
    ts = -(-cols // grid)
    tiles, Bs = [], []
    for k in range(grid):
        c0, c1 = k * ts, min(cols, (k + 1) * ts)
        rows = np.repeat(np.arange(A.rows), np.diff(A.rowptr))
        sel = (A.colind >= c0) & (A.colind < c1)
        lens = np.bincount(rows[sel], minlength=A.rows)
        tiles.append((synth.rowptr_from_lengths(lens), (A.colind[sel] - c0).astype(np.int32), Aint.values[sel]))
        Bs.append(B[c0:c1])
    full, S = oracle.spmm([(A.rowptr, A.colind, Aint.values)], [B])
    for off in range(grid + 2):
        C, Sk = oracle.spmm(tiles, Bs, k_offset=off)
        assert np.array_equal(C, full)          # integer inputs: exact in any order
        assert np.array_equal(Sk, S)


def test_sddmm_vs_dense():
    rng = _rng(19)
    A = small_csr(rng, 60, 50, max_len=20)
    B = synth.dense(50, 37, rng)
    dC = synth.dense(60, 37, rng)
    dA, S = oracle.sddmm(A.rowptr, A.colind, dC, B)
    full = dC.astype(np.float64) @ B.astype(np.float64).T
    Sfull = np.abs(dC.astype(np.float64)) @ np.abs(B.astype(np.float64)).T
    r = np.repeat(np.arange(60), np.diff(A.rowptr))
    assert np.all(np.abs(dA - full[r, A.colind]) <= 1e-12 * Sfull[r, A.colind])
    ent = np.array([A.nnz - 1, 0, 3, 3], dtype=np.int64)
    dAe, _ = oracle.sddmm(A.rowptr, A.colind, dC, B, entries=ent)
    assert np.array_equal(dAe, dA[ent])


def test_spmm_t_vs_dense_and_scipy():
    rng = _rng(20)
    A = small_csr(rng, 700, 500, max_len=30)
    dC = synth.dense(700, 19, rng, "normal")
    dB, S = oracle.spmm_t(A.rowptr, A.colind, A.values, 500, dC)
    ref = dense_of(A.rowptr, A.colind, A.values, 500).T @ dC.astype(np.float64)
    assert np.all(np.abs(dB - ref) <= 1e-12 * S + 1e-300)
    M = sp.csr_matrix((A.values.astype(np.float64), A.colind, A.rowptr), shape=(700, 500))
    assert np.all(np.abs(dB - M.T @ dC.astype(np.float64)) <= 1e-12 * S + 1e-300)
    rows = np.array([499, 3, 0], dtype=np.int64)
    dBs, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, 500, dC, out_rows=rows)
    assert np.array_equal(dBs, dB[rows])


def test_adjoint_identity():
    """<dC, A B> = sum_p val[p] dA[p] = <A^T dC, B>."""
    rng = _rng(21)
    A = small_csr(rng, 400, 350, max_len=40)
    B = synth.dense(350, 32, rng, "normal")
    dC = synth.dense(400, 32, rng, "normal")
    C, _ = oracle.spmm([(A.rowptr, A.colind, A.values)], [B])
    dA, _ = oracle.sddmm(A.rowptr, A.colind, dC, B)
    dB, _ = oracle.spmm_t(A.rowptr, A.colind, A.values, 350, dC)
    a = float((C * dC).sum())
    b = float((A.values.astype(np.float64) * dA).sum())
    c = float((dB * B).sum())
    scale = float(np.abs(C * dC).sum())
    assert abs(a - b) <= 1e-12 * scale and abs(a - c) <= 1e-12 * scale


# ---------------------------------------------------------------------------
# Transposed structure
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("rows,cols,seed", [(1, 1, 0), (300, 200, 1), (1000, 3000, 2), (2000, 17, 3)])
def test_transpose_vs_scipy(rows, cols, seed):
    rng = _rng(30 + seed)
    A = small_csr(rng, rows, cols, max_len=min(cols, 50))
    rpT, ciT, perm = oracle.transpose(A.rowptr, A.colind, cols)
    # SciPy's transpose carries the original positions as data (exact in FP64).
    M = sp.csr_matrix((np.arange(A.nnz, dtype=np.float64) + 1.0, A.colind, A.rowptr), shape=(rows, cols))
    T = M.T.tocsr()
    T.sort_indices()
    assert np.array_equal(rpT, T.indptr)
    assert np.array_equal(ciT, T.indices)
    assert np.array_equal(perm, (T.data - 1.0).astype(np.int64))
    # involution and permutation properties
    rp2, ci2, perm2 = oracle.transpose(rpT, ciT, rows)
    assert np.array_equal(rp2, A.rowptr) and np.array_equal(ci2, A.colind)
    assert np.array_equal(perm[perm2], np.arange(A.nnz))
    assert rpT[-1] == A.nnz and np.array_equal(np.sort(perm), np.arange(A.nnz))


# ---------------------------------------------------------------------------
# BF16 rounding
# ---------------------------------------------------------------------------
def test_bf16_vs_torch_stratified():
    """Every upper half with lower halves covering both sides of every tie."""
    import torch
    hi = np.arange(1 << 16, dtype=np.uint32) << 16
    lows = np.array([0x0000, 0x0001, 0x3FFF, 0x7FFF, 0x8000, 0x8001, 0xBFFF, 0xFFFF], dtype=np.uint32)
    bits = (hi[:, None] | lows[None, :]).ravel()
    x = bits.view(np.float32)
    ours = oracle.f32_to_bf16(x)
    theirs = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    nan = np.isnan(x)
    assert np.array_equal(ours[~nan], theirs[~nan])
    assert np.all(ours[nan] == 0x7FC0)


@pytest.mark.slow
def test_bf16_vs_torch_exhaustive():
    """All 2^32 FP32 bit patterns, in chunks small enough that their buffers are reused."""
    import torch
    step = 1 << 22
    base = np.arange(step, dtype=np.uint32)
    bits = np.empty(step, dtype=np.uint32)
    for start in range(0, 1 << 32, step):
        np.add(base, np.uint32(start), out=bits)
        x = bits.view(np.float32)
        ours = oracle.f32_to_bf16(x)
        theirs = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
        nan = np.isnan(x)
        assert np.array_equal(ours[~nan], theirs[~nan]), hex(start)
