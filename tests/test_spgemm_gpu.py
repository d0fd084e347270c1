"""Local SpGEMM C = A B on the GPU against the FP64 oracle: exact structure (row pointer and
sorted column indices), FP32 values within the tolerance of the sum's scale (integer data:
exact), every row class (wave hash sets and tables, workgroup bitmap and table, dense rows,
the global bitmap for wide B) at and around its boundaries, live values, graph replay."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import compare
from paper_2311_18141_amd import ops
from paper_2311_18141_amd._lib import SpmmError

import gpu_util as G

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _plan(A, B, validate=True, keep_pattern=True):
    dA = G.to_dev(A)
    dB = G.to_dev(B)
    return ops.spgemm_create(A.rows, dA, dB, validate=validate, keep_pattern=keep_pattern), dA, dB


def _products_per_row(A, B):
    lb = B.row_lengths()
    rowid = np.repeat(np.arange(A.rows), A.row_lengths())
    return np.bincount(rowid, weights=lb[A.colind], minlength=A.rows).astype(np.int64)


def _oracle(A, B, compress_cols=False):
    if not compress_cols:
        return oracle.spgemm((A.rowptr, A.colind, A.values), (B.rowptr, B.colind, B.values), B.cols)
    # B's used columns, in order, renumbered 0..u-1: an order-preserving bijection, so the
    # oracle on the compressed problem gives C's entries in the same order
    used = np.unique(B.colind)
    cB = np.searchsorted(used, B.colind).astype(np.int32)
    rp, ci, va, S = oracle.spgemm((A.rowptr, A.colind, A.values), (B.rowptr, cB, B.values), max(len(used), 1))
    return rp, used[ci].astype(np.int64), va, S


def _check(A, B, exact=False, plan=None, compress_cols=False, keep_pattern=True):
    if plan is None:
        plan, dA, dB = _plan(A, B, keep_pattern=keep_pattern)
        if not keep_pattern:
            assert plan.pattern_entries == 0
    rp = ops.spgemm_rowptr(plan)
    ci, va = ops.spgemm_compute(plan)
    calls = [(ci, va)]
    if plan.pattern_entries:
        # the first call found C's columns and kept them; the next one runs the kept-pattern kernels
        calls.append(ops.spgemm_compute(plan))
        ci, va = calls[-1]
    torch.cuda.synchronize()
    r_rp, r_ci, r_va, S = _oracle(A, B, compress_cols)
    assert plan.nnz_c == int(r_rp[-1])
    assert plan.products == int(_products_per_row(A, B).sum())
    assert np.array_equal(rp.cpu().numpy().astype(np.int64), r_rp)
    n_terms = np.repeat(_products_per_row(A, B) + 1, np.diff(r_rp))
    for ci, va in calls:
        assert np.array_equal(ci.cpu().numpy().astype(np.int64), r_ci)
        got = va.cpu().numpy().astype(np.float64)
        if exact:
            assert np.array_equal(got, r_va)
        else:
            st = compare.fp32_stats(got, r_va, S, n_terms=n_terms)
            assert compare.fp32_ok(st), st
    return plan


def _b_rows_of_lengths(lengths, cols, rng, kind="pm1"):
    return synth.random_csr(len(lengths), cols, np.asarray(lengths), rng, kind)


def _select_rows(K, picks, rng, kind="pm1"):
    """A with row r holding the (sorted, distinct) B rows picks[r]."""
    M = len(picks)
    L = np.array([len(p) for p in picks])
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int32)
    ci = np.concatenate([np.sort(np.asarray(p, dtype=np.int32)) for p in picks]) if L.sum() else np.zeros(0, np.int32)
    A = synth.random_csr(M, K, L, rng, kind)
    return synth.CSR(M, K, rp, ci.astype(np.int32), A.values)


@pytest.mark.parametrize("M,K,N,d", [(1, 1, 1, 1.0), (5, 7, 3, 0.5), (200, 150, 300, 0.02), (1000, 1000, 1000, 0.01)])
def test_spgemm_small_vs_oracle(M, K, N, d):
    G.note("spgemm small M=%d K=%d N=%d" % (M, K, N))
    rng = _rng(M + N)
    A = synth.random_csr(M, K, rng.binomial(K, d, size=M), rng, "normal")
    B = synth.random_csr(K, N, rng.binomial(N, d, size=K), rng, "normal")
    _check(A, B)


@pytest.mark.parametrize("keep_pattern", [True, False])
def test_spgemm_class_boundaries_integer_exact(keep_pattern):
    """Rows whose product and output counts sit on each side of every class boundary
    (128, 256, 512 for the wave classes; the workgroup table's half size; dense rows);
    the long rows with the kept column pattern and with the bitmap found on every call."""
    G.note("spgemm class boundaries keep_pattern=%s" % keep_pattern)
    rng = _rng(11)
    N = 30000
    lengths = [0, 1, 127, 128, 129, 255, 256, 257, 511, 512, 513, 1000, 4095, 4096, 4097, 8191, 8192, 8193,
               12000, 20000]
    B = _b_rows_of_lengths(lengths, N, rng, "int8")
    K = B.rows
    picks = [[k] for k in range(K)]                       # one B row each: products = output = length
    picks += [list(range(K))]                             # everything: dense, high compression
    picks += [[2, 3, 4], [9, 10], [13, 14, 15], [16, 17], [], [0], [18, 19]]
    A = _select_rows(K, picks, rng, "int8")
    plan = _check(A, B, exact=True, keep_pattern=keep_pattern)
    if keep_pattern:
        # the columns of every row (wave and workgroup tables, windows through a split table)
        assert plan.pattern_entries == plan.nnz_c > 0


def test_spgemm_wide_b_global_bitmap():
    """B wide enough that a bitmap over its columns does not fit in LDS: the symbolic
    pass uses the global per-workgroup bitmaps."""
    G.note("spgemm wide B")
    rng = _rng(12)
    N = 3_000_000
    B = _b_rows_of_lengths([600, 700, 2000, 40, 9000], N, rng, "int8")
    A = _select_rows(B.rows, [[0], [1, 2], [0, 1, 2, 3, 4], [3], [4], []], rng, "int8")
    _check(A, B, exact=True, compress_cols=True)


@pytest.mark.parametrize("keep_pattern", [True, False])
def test_spgemm_rmat_aa(keep_pattern):
    """C = A A on a skewed R-MAT matrix: all classes at once."""
    G.note("spgemm rmat14 A*A keep_pattern=%s" % keep_pattern)
    A = synth.rmat_csr(14, 8, seed=13)
    _check(A, A, keep_pattern=keep_pattern)


@pytest.mark.parametrize("keep_pattern", [True, False])
def test_spgemm_rmat_aa_integer_exact(keep_pattern):
    G.note("spgemm rmat13 A*A int keep_pattern=%s" % keep_pattern)
    rng = _rng(14)
    A0 = synth.rmat_csr(13, 8, seed=14)
    A = synth.CSR(A0.rows, A0.cols, A0.rowptr, A0.colind, rng.integers(-3, 4, size=A0.nnz).astype(np.float32))
    _check(A, A, exact=True, keep_pattern=keep_pattern)


def test_spgemm_cancellation_and_empty():
    G.note("spgemm cancellation and empty")
    A = synth.CSR(3, 2, np.array([0, 2, 2, 3], np.int32), np.array([0, 1, 1], np.int32),
                  np.array([1, 1, 2], np.float32))
    B = synth.CSR(2, 4, np.array([0, 2, 4], np.int32), np.array([1, 3, 1, 2], np.int32),
                  np.array([1, 5, -1, 7], np.float32))
    plan = _check(A, B, exact=True)
    assert plan.nnz_c == 3 + 2  # row 0: cols 1 (1 - 1 = 0, kept), 2, 3; row 2: cols 1, 2
    Z = synth.CSR(4, 2, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    plan, _, _ = _plan(Z, B)
    assert plan.nnz_c == 0 and plan.products == 0
    assert ops.spgemm_rowptr(plan).cpu().tolist() == [0] * 5
    ops.spgemm_compute(plan)
    torch.cuda.synchronize()


def test_spgemm_values_read_live_and_repeat():
    """The plan caches structure only: new values of A take effect; integer data repeats exactly."""
    G.note("spgemm live values")
    rng = _rng(15)
    A = synth.random_csr(500, 400, rng.integers(0, 30, size=500), rng, "int8")
    B = synth.random_csr(400, 600, rng.integers(0, 30, size=400), rng, "int8")
    plan, dA, dB = _plan(A, B)
    ci1, va1 = ops.spgemm_compute(plan)
    ci1, va1 = ci1.clone(), va1.clone()
    ci2, va2 = ops.spgemm_compute(plan)
    torch.cuda.synchronize()
    assert torch.equal(ci1, ci2) and torch.equal(va1, va2)
    dA[2].mul_(-2.0)
    A2 = synth.CSR(A.rows, A.cols, A.rowptr, A.colind, (A.values * -2.0).astype(np.float32))
    _check(A2, B, exact=True, plan=plan)


def test_spgemm_graph_replay():
    G.note("spgemm graph replay")
    rng = _rng(16)
    A = synth.random_csr(3000, 2000, rng.integers(0, 40, size=3000), rng, "int8")
    B = synth.random_csr(2000, 5000, rng.integers(0, 40, size=2000), rng, "int8")
    plan, dA, dB = _plan(A, B)
    ci = torch.empty(plan.nnz_c, dtype=torch.int32, device=G.DEV)
    va = torch.empty(plan.nnz_c, dtype=torch.float32, device=G.DEV)
    ops.spgemm_compute(plan, ci, va)
    torch.cuda.synchronize()
    ref_ci, ref_va = ci.clone(), va.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.spgemm_compute(plan, ci, va)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.spgemm_compute(plan, ci, va)
    for r in range(4):
        ci.fill_(-1)
        va.fill_(float("nan"))
        _ = (dA[2] * 3).sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ci, ref_ci) and torch.equal(va, ref_va), r


def test_spgemm_rejects_bad_csr():
    G.note("spgemm bad csr")
    rng = _rng(17)
    A = synth.random_csr(10, 10, np.full(10, 3), rng)
    bad = synth.CSR(A.rows, A.cols, A.rowptr, A.colind.copy(), A.values)
    bad.colind[4] = 99
    with pytest.raises(SpmmError):
        _plan(bad, A)
    with pytest.raises(SpmmError):
        _plan(A, bad)


def test_spgemm_very_wide_b_dense_slots():
    """B so wide (about 201M columns) that long rows cannot be cut into column windows:
    they accumulate in dense global rows (values + bitmap) instead."""
    G.note("spgemm very wide B (dense slots)")
    rng = _rng(18)
    N = (1 << 27) + (1 << 26)
    B = _b_rows_of_lengths([5000, 6000, 700, 20], N, rng, "int8")
    A = _select_rows(B.rows, [[0, 1], [2], [0, 1, 2, 3], [3], []], rng, "int8")
    _check(A, B, exact=True, compress_cols=True)


def test_spgemm_long_rows_without_split_table():
    """B with so many rows that its window split table would exceed its budget (800K rows x
    93 windows): long rows find each window's B-row range by binary search instead."""
    G.note("spgemm long rows, binary-searched windows")
    rng = _rng(19)
    K, N = 800_000, 3_000_000
    L = np.zeros(K, dtype=np.int64)
    hot = rng.choice(K, size=6, replace=False)
    L[hot] = [9000, 7000, 3000, 600, 40, 5]
    B = synth.random_csr(K, N, L, rng, "int8")
    A = _select_rows(K, [list(hot[:2]), list(hot), [hot[2]], list(hot[3:]), []], rng, "int8")
    _check(A, B, exact=True, compress_cols=True)


@pytest.mark.parametrize("keep_pattern", [True, False])
def test_spgemm_medium_rows_to_windows(keep_pattern):
    """C with 300K columns: rows of 4K-8K entries cannot keep a column bitmap beside their
    16K-slot table, and there are few windows, so they take the window path."""
    G.note("spgemm medium rows through windows keep_pattern=%s" % keep_pattern)
    rng = _rng(20)
    N = 300_000
    B = _b_rows_of_lengths([4500, 6000, 8100, 600, 3000, 20000], N, rng, "int8")
    A = _select_rows(B.rows, [[0], [1], [2], [3, 4], [0, 3], [5], [1, 2, 3]], rng, "int8")
    _check(A, B, exact=True, keep_pattern=keep_pattern)


@pytest.mark.parametrize("keep_pattern", [True, False])
def test_spgemm_long_rows_negative_zero_products(keep_pattern):
    """Long rows (column windows) with -0.0 products (an A or a B value stored as -0.0 times
    a positive value): a column reached only by such products is still a structural entry,
    so a kernel that told presence from its sum would miss it; the structure stays exact.
    Both long-row paths (at most and more than 1,024 A entries) are covered, as are rows
    with no such column, a row whose every product is -0.0, and +0.0 products."""
    G.note("spgemm long rows, -0.0 products keep_pattern=%s" % keep_pattern)
    rng = _rng(21)
    N = 70000
    cols0 = rng.choice(N, 9000, replace=False)
    rest = np.setdiff1d(np.arange(N), cols0)
    cols1 = rng.choice(rest, 8, replace=False)
    cols2 = rng.choice(np.setdiff1d(rest, cols1), 6, replace=False)
    brows = [cols0, cols1, cols2] + [rng.choice(N, 12, replace=False) for _ in range(1100)]
    bvals = ([rng.integers(1, 4, 9000), rng.integers(1, 4, 8), np.full(6, -0.0)]
             + [rng.integers(-3, 4, 12) for _ in range(1100)])
    order = [np.argsort(c) for c in brows]
    B = synth.CSR(len(brows), N, np.concatenate([[0], np.cumsum([len(c) for c in brows])]).astype(np.int32),
                  np.concatenate([c[o] for c, o in zip(brows, order)]).astype(np.int32),
                  np.concatenate([v[o] for v, o in zip(bvals, order)]).astype(np.float32))
    assert np.signbit(B.values[B.rowptr[2]:B.rowptr[3]]).all()
    many = list(range(3, 1103))
    arows = [([0, 1], [1.0, -0.0]),            # B row 1's columns: only -0.0 products
             ([0, 2], [1.0, 2.0]),             # B row 2's columns: 2 x -0.0
             ([0, 1, 2], [1.0, -0.0, 5.0]),
             ([0, 1], [1.0, 2.0]),             # no -0.0 product
             (many + [1], None),               # more than 1,024 A entries, one -0.0 product row
             (many, None),
             ([1], [-0.0]),                    # a short row (hash path)
             ([0], [-0.0]),                    # every product -0.0: every window redone
             ([0, 1], [-1.0, 0.0])]            # +0.0 products
    rp, ci, va = [0], [], []
    for ks, vs in arows:
        ks = np.asarray(ks)
        if vs is None:
            vs = rng.integers(-3, 4, len(ks)).astype(np.float32)
            vs[ks == 1] = -0.0
            vs[(ks != 1) & (vs == 0)] = 1.0
        vs = np.asarray(vs, np.float32)
        o = np.argsort(ks)
        ci.append(ks[o])
        va.append(vs[o])
        rp.append(rp[-1] + len(ks))
    A = synth.CSR(len(arows), B.rows, np.asarray(rp, np.int32), np.concatenate(ci).astype(np.int32),
                  np.concatenate(va))
    plan = _check(A, B, exact=True, keep_pattern=keep_pattern)
    assert (plan.pattern_entries > 0) == keep_pattern


def _long_rows_case(rng):
    """Integer data with rows of C longer than 4,096 entries (three 32K-column windows),
    one of them from more than 1,024 A entries, beside short and medium rows."""
    N = 70000
    lengths = [9000, 5000, 700, 40] + [12] * 1100
    B = _b_rows_of_lengths(lengths, N, rng, "int8")
    A = _select_rows(B.rows, [[0], [0, 1], [2, 3], list(range(4, 1104)), [1], list(range(1104)), []], rng, "int8")
    return A, B


def test_spgemm_long_rows_live_values_and_repeat():
    """With the kept pattern the plan still caches structure only: calls repeat exactly on
    integer data, new values of A and of B take effect, and the results equal those of a
    plan that finds the long rows' columns on every call."""
    G.note("spgemm long rows, live values with the kept pattern")
    rng = _rng(22)
    A, B = _long_rows_case(rng)
    plan, dA, dB = _plan(A, B)
    assert plan.pattern_entries > 0
    ci1, va1 = ops.spgemm_compute(plan)
    ci1, va1 = ci1.clone(), va1.clone()
    ci2, va2 = ops.spgemm_compute(plan)
    plain, _, _ = _plan(A, B, keep_pattern=False)
    ci3, va3 = ops.spgemm_compute(plain)
    torch.cuda.synchronize()
    assert torch.equal(ci1, ci2) and torch.equal(va1, va2)
    assert torch.equal(ci1, ci3) and torch.equal(va1, va3)
    dA[2].mul_(-2.0)
    dB[2].mul_(3.0)
    A2 = synth.CSR(A.rows, A.cols, A.rowptr, A.colind, (A.values * -2.0).astype(np.float32))
    B2 = synth.CSR(B.rows, B.cols, B.rowptr, B.colind, (B.values * 3.0).astype(np.float32))
    _check(A2, B2, exact=True, plan=plan)


def test_spgemm_graph_capture_as_first_call():
    """A plan's first compute call made under graph capture keeps no columns (its copy would only
    run at replay): replays and the eager calls after it, the first of which keeps the columns and
    the next of which uses them, all give the eager result."""
    G.note("spgemm graph capture as the first call")
    rng = _rng(24)
    A, B = _long_rows_case(rng)
    plan, dA, dB = _plan(A, B)
    ref, _, _ = _plan(A, B, keep_pattern=False)
    ref_ci, ref_va = ops.spgemm_compute(ref)
    ci = torch.empty(plan.nnz_c, dtype=torch.int32, device=G.DEV)
    va = torch.empty(plan.nnz_c, dtype=torch.float32, device=G.DEV)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ops.spgemm_compute(plan, ci, va)
    for r in range(3):
        ci.fill_(-1)
        va.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ci, ref_ci) and torch.equal(va, ref_va), r
    for r in range(3):   # finds and keeps the columns, then uses them
        ci.fill_(-1)
        va.fill_(float("nan"))
        ops.spgemm_compute(plan, ci, va)
        torch.cuda.synchronize()
        assert torch.equal(ci, ref_ci) and torch.equal(va, ref_va), r
    g.replay()           # the captured (column-finding) form still agrees
    torch.cuda.synchronize()
    assert torch.equal(ci, ref_ci) and torch.equal(va, ref_va)


def test_spgemm_long_rows_graph_replay():
    """The kept-pattern long-row kernel replayed from a graph: every replay equals the eager call."""
    G.note("spgemm long rows, graph replay")
    rng = _rng(23)
    A, B = _long_rows_case(rng)
    plan, dA, dB = _plan(A, B)
    assert plan.pattern_entries > 0
    ci = torch.empty(plan.nnz_c, dtype=torch.int32, device=G.DEV)
    va = torch.empty(plan.nnz_c, dtype=torch.float32, device=G.DEV)
    ops.spgemm_compute(plan, ci, va)
    torch.cuda.synchronize()
    ref_ci, ref_va = ci.clone(), va.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        ops.spgemm_compute(plan, ci, va)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ops.spgemm_compute(plan, ci, va)
    for r in range(4):
        ci.fill_(-1)
        va.fill_(float("nan"))
        _ = (dA[2] * 3).sum()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(ci, ref_ci) and torch.equal(va, ref_va), r
