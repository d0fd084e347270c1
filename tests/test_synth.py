"""The seeded input generators: determinism per seed, canonical CSR, and the distribution
each workload's recipe states (R-MAT quadrant shares, the heavy-tailed degree law, uniform
rows, the uneven batch's ranges)."""
import numpy as np
import pytest

import synth


def _canonical(A):
    rp, ci = A.rowptr, A.colind
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and A.values.dtype == np.float32
    assert rp[0] == 0 and rp[-1] == A.nnz == ci.size == A.values.size
    assert np.all(np.diff(rp.astype(np.int64)) >= 0)
    if A.nnz:
        assert ci.min() >= 0 and ci.max() < A.cols
        rowid = np.repeat(np.arange(A.rows), np.diff(rp))
        same = rowid[1:] == rowid[:-1]
        assert np.all(ci[1:][same] > ci[:-1][same]), "columns must be strictly increasing within a row"


def _same(A, B):
    return (A.rows, A.cols) == (B.rows, B.cols) and all(
        np.array_equal(x, y) for x, y in ((A.rowptr, B.rowptr), (A.colind, B.colind), (A.values, B.values)))


@pytest.mark.parametrize("make", [
    lambda s: synth.uniform_csr(3000, 5000, 17, seed=s),
    lambda s: synth.rmat_csr(12, 8, seed=s),
    lambda s: synth.powerlaw_csr(1 << 12, 1 << 12, 16, 1024, seed=s),
    lambda s: synth.rmat_row_block(12, 8, 4, 1, seed=s).tiles[2],
])
def test_deterministic_per_seed_and_canonical(make):
    A, B, C = make(5), make(5), make(6)
    _canonical(A)
    _canonical(C)
    assert _same(A, B)
    assert not _same(A, C)


def test_uniform_rows_hold_exactly_their_count():
    A = synth.uniform_csr(2000, 300, 40, seed=1)
    assert np.all(np.diff(A.rowptr) == 40)
    _canonical(A)
    full = synth.uniform_csr(50, 64, 64, seed=2)   # a row as long as the tile is wide
    assert np.array_equal(full.colind.reshape(50, 64), np.tile(np.arange(64, dtype=np.int32), (50, 1)))


def test_rmat_quadrant_shares():
    """Top-level quadrant shares of R-MAT scale 16 (edge factor 4) match (0.57, 0.19, 0.19,
    0.05) within the shift that merging repeated edges causes (they repeat most in a)."""
    s = 16
    A = synth.rmat_csr(s, 4, seed=3)
    half = 1 << (s - 1)
    rowid = np.repeat(np.arange(A.rows), np.diff(A.rowptr))
    rb, cb = rowid >= half, A.colind >= half
    shares = np.array([np.mean(~rb & ~cb), np.mean(~rb & cb), np.mean(rb & ~cb), np.mean(rb & cb)])
    assert np.allclose(shares, synth.RMAT_GRAPH500, atol=0.03), shares
    assert A.nnz > 0.9 * (4 << s)          # few repeated edges at this density
    # no vertex permutation: the hub is vertex 0 (all bits in quadrant a)
    assert np.argmax(np.diff(A.rowptr)) < 16


def test_rmat_row_block_is_the_matrix_cut_into_tiles():
    g = synth.rmat_row_block(12, 8, 4, 1, seed=9)
    A = synth.rmat_csr(12, 8, seed=9)
    ts = A.rows // 4
    for k, t in enumerate(g.tiles):
        assert (t.rows, t.cols) == (ts, ts)
        for i in (0, 7, ts - 1):
            r = ts + i
            full = A.colind[A.rowptr[r]:A.rowptr[r + 1]]
            want = full[(full >= k * ts) & (full < (k + 1) * ts)] - k * ts
            assert np.array_equal(t.colind[t.rowptr[i]:t.rowptr[i + 1]], want)
    assert g.grid_nnz.sum() == A.nnz
    assert g.imbalance >= 1.0


def test_pareto_degrees_recipe():
    """Sum exactly mean * rows, the largest row exactly dmax, every row at least 1, and a tail
    P(d >= x) ~ x^-(alpha - 1): the log-log slope between 32 and 512 is near -1.1."""
    rows, mean, dmax = 1 << 18, 32, 65536
    d = synth.pareto_degrees(rows, mean, dmax, 2.1, np.random.Generator(np.random.PCG64(4)))
    assert d.sum() == mean * rows and d.max() == dmax and d.min() >= 1
    p32, p512 = np.mean(d >= 32), np.mean(d >= 512)
    slope = np.log(p512 / p32) / np.log(512 / 32)
    assert -1.35 < slope < -0.85, slope


def test_uneven_tiles_recipe():
    tiles, widths = synth.uneven_tiles(40, seed=4, rows_hi=4096)
    assert len(tiles) == len(widths) == 40
    assert set(widths) <= {32, 64, 128, 256}
    for t in tiles:
        _canonical(t)
        assert t.rows == t.cols and 1024 <= t.rows <= 4096
        lens = np.diff(t.rowptr)
        assert np.all(lens == lens[0]) and 4 <= lens[0] <= 256


def test_dense_kinds():
    rng = np.random.Generator(np.random.PCG64(7))
    x = synth.dense(300, 40, rng)
    assert x.shape == (300, 40) and x.dtype == np.float32 and x.min() >= -1 and x.max() < 1
    i = synth.dense(300, 40, rng, "int8")
    assert np.array_equal(i, np.rint(i)) and np.abs(i).max() <= 8
    n = synth.dense(1000, 40, rng, "normal")
    assert abs(float(n.mean())) < 0.02 and abs(float(n.std()) - 1.0) < 0.02
