"""Pins of the oracle's sparse-times-sparse product C = A B (CPU only).

The oracle's SpGEMM is checked against what fixes it independently: dense NumPy
products of the dense forms (values) and of the 0/1 indicator matrices (the
structural pattern), SciPy's sparse product, exhaustive 2x2 patterns, identity and
permutation matrices, integer-exact data, a cancellation that must keep its entry,
row subsets, the |A||B| scale, and associativity.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import synth



def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _csr_from_dense(D):
    M = sp.csr_matrix(D)
    M.sort_indices()
    return M


def _csr_pattern(rows, cols, density, rng, values="pm1"):
    L = rng.binomial(cols, density, size=rows)
    return synth.random_csr(rows, cols, L, rng, values)


def _dense_of(rp, ci, va, rows, cols):
    D = np.zeros((rows, cols), dtype=np.float64)
    for i in range(rows):
        for p in range(rp[i], rp[i + 1]):
            D[i, ci[p]] += va[p]
    return D


def _run(A, B):
    return oracle.spgemm((A.rowptr, A.colind, A.values), (B.rowptr, B.colind, B.values), B.cols)


def _indicator(X):
    D = np.zeros((X.rows, X.cols), dtype=np.int64)
    for i in range(X.rows):
        D[i, X.colind[X.rowptr[i]:X.rowptr[i + 1]]] = 1
    return D


def _check_against_dense(A, B, exact=False):
    rp, ci, va, S = _run(A, B)
    M, N = A.rows, B.cols
    # pattern: structural product of the indicator matrices
    P = (_indicator(A) @ _indicator(B)) > 0
    got_pattern = np.zeros((M, N), dtype=bool)
    for i in range(M):
        cols = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cols) > 0), "row %d columns not strictly increasing" % i
        got_pattern[i, cols] = True
    assert np.array_equal(got_pattern, P)
    Ad = _dense_of(A.rowptr, A.colind, A.values.astype(np.float64), A.rows, A.cols)
    Bd = _dense_of(B.rowptr, B.colind, B.values.astype(np.float64), B.rows, B.cols)
    Cd = Ad @ Bd
    Sd = np.abs(Ad) @ np.abs(Bd)
    got = _dense_of(rp, ci, va, M, N)
    gotS = _dense_of(rp, ci, S, M, N)
    if exact:
        assert np.array_equal(got, Cd)
        assert np.array_equal(gotS, Sd)
    else:
        assert np.allclose(got, Cd, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(Sd).max()))
        assert np.allclose(gotS, Sd, rtol=1e-12, atol=0)
    return rp, ci, va, S


@pytest.mark.parametrize("M,K,N,d", [(1, 1, 1, 1.0), (7, 5, 9, 0.3), (40, 30, 50, 0.1), (64, 64, 64, 0.05)])
def test_spgemm_vs_dense(M, K, N, d):
    rng = _rng(M * 1000 + N)
    A = _csr_pattern(M, K, d, rng, "normal")
    B = _csr_pattern(K, N, d, rng, "normal")
    _check_against_dense(A, B)


def test_spgemm_integer_exact():
    rng = _rng(3)
    A = _csr_pattern(60, 70, 0.2, rng, "int8")
    B = _csr_pattern(70, 80, 0.2, rng, "int8")
    _check_against_dense(A, B, exact=True)


def test_spgemm_exhaustive_2x2_patterns():
    """All 16 x 16 pattern pairs of 2x2 matrices with distinct integer values."""
    for pa, pb in itertools.product(range(16), range(16)):
        def mk(pat, base):
            rows, cols, vals = [], [], []
            for i in range(2):
                for j in range(2):
                    if pat >> (2 * i + j) & 1:
                        rows.append(i)
                        cols.append(j)
                        vals.append(base + 2 * i + j)
            L = np.bincount(np.array(rows, dtype=np.int64), minlength=2)
            rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int32)
            return synth.CSR(2, 2, rp, np.array(cols, dtype=np.int32), np.array(vals, dtype=np.float32))
        _check_against_dense(mk(pa, 1), mk(pb, 5), exact=True)


def test_spgemm_vs_scipy():
    rng = _rng(4)
    A = _csr_pattern(300, 200, 0.03, rng, "normal")
    B = _csr_pattern(200, 250, 0.03, rng, "normal")
    rp, ci, va, _ = _run(A, B)
    a = sp.csr_matrix((A.values.astype(np.float64), A.colind, A.rowptr), shape=(A.rows, A.cols))
    b = sp.csr_matrix((B.values.astype(np.float64), B.colind, B.rowptr), shape=(B.rows, B.cols))
    c = (a @ b).tocsr()
    c.sort_indices()
    # normal values: no product sum cancels to exactly zero, so SciPy's pruning changes nothing
    assert np.array_equal(rp, c.indptr)
    assert np.array_equal(ci, c.indices)
    assert np.allclose(va, c.data, rtol=1e-13, atol=1e-13)


def test_spgemm_cancellation_keeps_entry():
    """[1 1] times [1; -1] is a structural 1x1 entry whose value is exactly zero."""
    A = synth.CSR(1, 2, np.array([0, 2], np.int32), np.array([0, 1], np.int32), np.array([1, 1], np.float32))
    B = synth.CSR(2, 1, np.array([0, 1, 2], np.int32), np.array([0, 0], np.int32), np.array([1, -1], np.float32))
    rp, ci, va, S = _run(A, B)
    assert rp.tolist() == [0, 1] and ci.tolist() == [0] and va.tolist() == [0.0] and S.tolist() == [2.0]


def test_spgemm_identity_and_permutation():
    rng = _rng(5)
    A = _csr_pattern(50, 50, 0.1, rng, "normal")
    I = synth.CSR(50, 50, np.arange(51, dtype=np.int32), np.arange(50, dtype=np.int32), np.ones(50, np.float32))
    for X, Y in ((I, A), (A, I)):
        rp, ci, va, _ = _run(X, Y)
        assert np.array_equal(rp, A.rowptr) and np.array_equal(ci, A.colind)
        assert np.array_equal(va, A.values.astype(np.float64))
    perm = rng.permutation(50)
    P = synth.CSR(50, 50, np.arange(51, dtype=np.int32), perm.astype(np.int32), np.ones(50, np.float32))
    rp, ci, va, _ = _run(P, A)   # row i of P A is row perm[i] of A
    for i in range(50):
        j = perm[i]
        assert np.array_equal(ci[rp[i]:rp[i + 1]], A.colind[A.rowptr[j]:A.rowptr[j + 1]])
        assert np.array_equal(va[rp[i]:rp[i + 1]], A.values[A.rowptr[j]:A.rowptr[j + 1]].astype(np.float64))


def test_spgemm_rows_subset_and_empty():
    rng = _rng(6)
    L = rng.integers(0, 6, size=80)
    L[[3, 9]] = 0
    A = synth.random_csr(80, 90, L, rng, "normal")
    B = synth.random_csr(90, 70, rng.integers(0, 6, size=90), rng, "normal")
    rp, ci, va, S = _run(A, B)
    rows = np.array([79, 3, 0, 9, 41], dtype=np.int64)
    rp2, ci2, va2, S2 = oracle.spgemm((A.rowptr, A.colind, A.values), (B.rowptr, B.colind, B.values), B.cols,
                                      rows=rows)
    for r, i in enumerate(rows):
        assert np.array_equal(ci2[rp2[r]:rp2[r + 1]], ci[rp[i]:rp[i + 1]])
        assert np.array_equal(va2[rp2[r]:rp2[r + 1]], va[rp[i]:rp[i + 1]])
        assert np.array_equal(S2[rp2[r]:rp2[r + 1]], S[rp[i]:rp[i + 1]])
    assert rp[4] - rp[3] == 0 and rp[10] - rp[9] == 0
    Z = synth.CSR(5, 90, np.zeros(6, np.int32), np.zeros(0, np.int32), np.zeros(0, np.float32))
    rp, ci, va, S = _run(Z, B)
    assert rp.tolist() == [0] * 6 and ci.size == 0


def test_spgemm_associative_pattern():
    """(A B) C and A (B C) have the same pattern and agree to rounding (integer data: exactly)."""
    rng = _rng(7)
    A = _csr_pattern(30, 25, 0.15, rng, "int4")
    B = _csr_pattern(25, 35, 0.15, rng, "int4")
    C = _csr_pattern(35, 20, 0.15, rng, "int4")
    def prod(X, Y):
        rp, ci, va, _ = _run(X, Y)
        return synth.CSR(X.rows, Y.cols, rp.astype(np.int32), ci.astype(np.int32), va.astype(np.float32))
    L = prod(prod(A, B), C)
    R = prod(A, prod(B, C))
    assert np.array_equal(L.rowptr, R.rowptr) and np.array_equal(L.colind, R.colind)
    assert np.array_equal(L.values, R.values)
