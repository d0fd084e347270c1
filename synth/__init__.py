"""Seeded synthetic inputs for the local sparse-times-dense multiply.

This module serves both the CPU oracle and the GPU path; it holds none of the
method's arithmetic (no products, no sums over non-zeros, no transposition).
It draws random patterns and values and assembles them into canonical CSR:
row pointer, strictly increasing column indices per row, FP32 values
(Section 3.1 describes the three-array CSR tile; Section 6 fixes FP32 values
with 32-bit indices).

The paper evaluates on public matrices (Table 1) that are not available here;
the generators below stand in for them with the same kinds of structure:
uniform sparsity, R-MAT power-law graphs, heavy-tailed row degrees, and many
uneven tiles.  Every generator is deterministic in its integer seed: the seed
feeds ``numpy.random.SeedSequence(seed).spawn(4)`` and the four children drive
PCG64 streams for (pattern, values, first dense operand, second dense operand).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np

# Graph500 R-MAT quadrant probabilities (a, b, c, d).
RMAT_GRAPH500 = (0.57, 0.19, 0.19, 0.05)


@dataclasses.dataclass
class CSR:
    """A CSR tile: ``rowptr`` int32[rows+1], ``colind`` int32[nnz], ``values`` float32[nnz].

    Column indices are tile-local, strictly increasing within each row.
    """

    rows: int
    cols: int
    rowptr: np.ndarray
    colind: np.ndarray
    values: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.colind.shape[0])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))


def streams(seed: int, n: int = 4) -> List[np.random.Generator]:
    """``n`` independent PCG64 generators spawned from ``SeedSequence(seed)``."""
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


def uniform_pm1(rng: np.random.Generator, shape) -> np.ndarray:
    """FP32 values uniform on [-1, 1)."""
    x = rng.random(shape, dtype=np.float32)
    x *= np.float32(2.0)
    x -= np.float32(1.0)
    return x


def normal_f32(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape, dtype=np.float32)


def rowptr_from_lengths(lengths: np.ndarray) -> np.ndarray:
    rp = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=rp[1:])
    if rp[-1] >= 2**31:
        raise ValueError("tile has 2^31 or more non-zeros; 32-bit indices cannot address it")
    return rp.astype(np.int32)


def distinct_sorted_columns(rng: np.random.Generator, lengths: np.ndarray, ncols: int) -> np.ndarray:
    """For each row r draw ``lengths[r]`` distinct columns uniformly from [0, ncols), sorted.

    Rejection sampling: draw with replacement, sort per row, redraw the later copy
    of every repeated column, repeat until no row holds a repeat.  The result is a
    uniformly random subset per row.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    if lengths.size and int(lengths.max()) > ncols:
        raise ValueError("a row cannot hold more distinct columns than the tile has")
    nnz = int(lengths.sum())
    if nnz == 0:
        return np.zeros(0, dtype=np.int32)
    row = np.repeat(np.arange(lengths.shape[0], dtype=np.int64), lengths)
    key = row * ncols + rng.integers(0, ncols, size=nnz, dtype=np.int64)
    key.sort()
    starts = np.zeros(lengths.shape[0] + 1, dtype=np.int64)
    np.cumsum(lengths, out=starts[1:])
    while True:
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if dup.size == 0:
            break
        # Rows that hold a repeat get the repeat redrawn, then only those rows are
        # re-sorted: keys are row * ncols + col, so one sort of the gathered rows keeps
        # every row inside its own segment.
        bad_rows = np.unique(key[dup] // ncols)
        key[dup] = (key[dup] // ncols) * ncols + rng.integers(0, ncols, size=dup.size, dtype=np.int64)
        seg_len = lengths[bad_rows]
        seg_start = starts[bad_rows]
        first = np.zeros(seg_len.shape[0], dtype=np.int64)
        np.cumsum(seg_len[:-1], out=first[1:])
        idx = np.repeat(seg_start - first, seg_len) + np.arange(int(seg_len.sum()), dtype=np.int64)
        sub = key[idx]
        sub.sort()
        key[idx] = sub
    return (key - row * ncols).astype(np.int32)


def _csr_from_sorted_keys(key: np.ndarray, rows: int, cols: int, values: np.ndarray) -> CSR:
    r = key // cols
    c = (key - r * cols).astype(np.int32)
    lengths = np.bincount(r, minlength=rows)
    return CSR(rows, cols, rowptr_from_lengths(lengths), c, values)


# ---------------------------------------------------------------------------
# Uniform (Erdos-Renyi style) tile with a fixed number of non-zeros per row.
# ---------------------------------------------------------------------------
def uniform_csr(rows: int, cols: int, per_row: int, seed: int, values: str = "pm1") -> CSR:
    """Every row holds exactly ``per_row`` distinct uniform columns; values U[-1,1) FP32."""
    rs = streams(seed)
    lengths = np.full(rows, per_row, dtype=np.int64)
    col = distinct_sorted_columns(rs[0], lengths, cols)
    vals = uniform_pm1(rs[1], col.shape[0]) if values == "pm1" else normal_f32(rs[1], col.shape[0])
    return CSR(rows, cols, rowptr_from_lengths(lengths), col, vals)


def random_csr(rows: int, cols: int, lengths: np.ndarray, rng: np.random.Generator,
               value_kind: str = "pm1") -> CSR:
    """CSR with the given row lengths, distinct uniform sorted columns.

    ``value_kind``: "pm1" (U[-1,1)), "normal", "int8" (integers in [-8, 8]),
    "int4" (integers in [-4, 4]), "ones", "pow2" (+-2^e, e in [-3, 3]).
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    col = distinct_sorted_columns(rng, lengths, cols)
    return CSR(rows, cols, rowptr_from_lengths(lengths), col, draw_values(rng, col.shape[0], value_kind))


def draw_values(rng: np.random.Generator, n, value_kind: str) -> np.ndarray:
    if value_kind == "pm1":
        return uniform_pm1(rng, n)
    if value_kind == "normal":
        return normal_f32(rng, n)
    if value_kind == "int8":
        return rng.integers(-8, 9, size=n).astype(np.float32)
    if value_kind == "int4":
        return rng.integers(-4, 5, size=n).astype(np.float32)
    if value_kind == "ones":
        return np.ones(n, dtype=np.float32)
    if value_kind == "pow2":
        e = rng.integers(-3, 4, size=n)
        s = rng.choice(np.array([-1.0, 1.0]), size=n)
        return (s * np.ldexp(1.0, e)).astype(np.float32)
    raise ValueError(value_kind)


# ---------------------------------------------------------------------------
# R-MAT graphs (recursive quadrant choice per edge, MSB first, no noise, no
# vertex permutation; directed; self loops kept; repeated edges merged on the
# pattern, then one value drawn per unique entry in CSR order).
# ---------------------------------------------------------------------------
def rmat_keys(scale: int, edge_factor: int, rng: np.random.Generator,
              probs: Sequence[float] = RMAT_GRAPH500, chunk: int = 1 << 24) -> np.ndarray:
    """Sorted unique edge keys ``row << scale | col`` of an R-MAT graph."""
    a, b, c, _ = probs
    t_ab = np.float32(a + b)            # below: row bit 0
    t_a = np.float32(a)
    t_abc = np.float32(a + b + c)
    n_edges = edge_factor << scale
    out = []
    for start in range(0, n_edges, chunk):
        m = min(chunk, n_edges - start)
        row = np.zeros(m, dtype=np.int64)
        col = np.zeros(m, dtype=np.int64)
        for _ in range(scale):
            u = rng.random(m, dtype=np.float32)
            rbit = u >= t_ab                                   # quadrants c, d
            cbit = ((u >= t_a) & (u < t_ab)) | (u >= t_abc)    # quadrants b, d
            row <<= 1
            col <<= 1
            row |= rbit
            col |= cbit
        out.append((row << scale) | col)
        del row, col
    keys = np.concatenate(out)
    del out
    return np.unique(keys)


@dataclasses.dataclass
class RmatGrid:
    """One row-block of an R-MAT matrix split into a ``grid`` x ``grid`` tile grid."""

    tiles: List[CSR]             # the row-block's k-tiles, k = 0..grid-1
    tile_rows: int
    grid_nnz: np.ndarray         # nnz per tile over the whole grid, shape (grid, grid)

    @property
    def imbalance(self) -> float:
        """max/avg non-zeros per tile over the grid (the paper's Section 6 load imbalance)."""
        return float(self.grid_nnz.max() / self.grid_nnz.mean())


def rmat_row_block(scale: int, edge_factor: int, grid: int, row_block: int, seed: int,
                   probs: Sequence[float] = RMAT_GRAPH500) -> RmatGrid:
    """Tiles (row_block, k) for k in 0..grid-1 of an R-MAT matrix cut into a regular grid."""
    rs = streams(seed)
    keys = rmat_keys(scale, edge_factor, rs[0], probs)
    n = 1 << scale
    ts = -(-n // grid)
    vals_all = uniform_pm1(rs[1], keys.shape[0])
    row = keys >> scale
    col = keys & (n - 1)
    grid_nnz = np.bincount((row // ts) * grid + (col // ts), minlength=grid * grid).reshape(grid, grid)
    r0, r1 = row_block * ts, min(n, (row_block + 1) * ts)
    lo, hi = np.searchsorted(row, [r0, r1])
    row, col, vals = row[lo:hi] - r0, col[lo:hi], vals_all[lo:hi]
    del keys, vals_all
    rows = r1 - r0
    tiles = []
    for k in range(grid):
        c0, c1 = k * ts, min(n, (k + 1) * ts)
        sel = (col >= c0) & (col < c1)
        lengths = np.bincount(row[sel], minlength=rows)
        tiles.append(CSR(rows, c1 - c0, rowptr_from_lengths(lengths),
                         (col[sel] - c0).astype(np.int32), vals[sel].copy()))
    return RmatGrid(tiles, rows, grid_nnz)


def rmat_csr(scale: int, edge_factor: int, seed: int, probs: Sequence[float] = RMAT_GRAPH500) -> CSR:
    """The whole R-MAT matrix as one square CSR tile with U[-1,1) FP32 values."""
    rs = streams(seed)
    keys = rmat_keys(scale, edge_factor, rs[0], probs)
    n = 1 << scale
    vals = uniform_pm1(rs[1], keys.shape[0])
    row = keys >> scale
    col = (keys & (n - 1)).astype(np.int32)
    del keys
    lengths = np.bincount(row, minlength=n)
    del row
    return CSR(n, n, rowptr_from_lengths(lengths), col, vals)


# ---------------------------------------------------------------------------
# Heavy-tailed (power-law) row degrees, as in GNN adjacency matrices.
# ---------------------------------------------------------------------------
def pareto_degrees(rows: int, mean: int, dmax: int, alpha: float, rng: np.random.Generator) -> np.ndarray:
    """Row degrees from a continuous Pareto(alpha) tail, clipped to [1, dmax].

    ``x_min`` is chosen so that the clipped mean is close to ``mean``; the sum is
    then made exactly ``mean * rows`` by +-1 steps on random rows, and the
    largest row is set to exactly ``dmax``.
    """
    beta = alpha - 1.0                  # survival exponent: P(X > x) = (x_min / x)^beta
    e = -1.0 / beta

    def clipped_mean(xmin):
        # E[min(X, dmax)] = x_min + x_min/(beta-1) * (1 - (x_min/dmax)^(beta-1)); the floor
        # removes about one half on average.
        return xmin + xmin / (beta - 1.0) * (1.0 - (xmin / dmax) ** (beta - 1.0)) - 0.5

    lo, hi = 1.0, float(mean)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if clipped_mean(mid) < mean:
            lo = mid
        else:
            hi = mid
    xmin = 0.5 * (lo + hi)
    u = rng.random(rows)
    d = np.floor(xmin * (1.0 - u) ** e)
    d = np.clip(d, 1, dmax).astype(np.int64)
    top = int(np.argmax(d))
    d[top] = dmax
    target = mean * rows
    while True:
        diff = target - int(d.sum())
        if diff == 0:
            break
        idx = rng.integers(0, rows, size=min(abs(diff), rows))
        idx = np.unique(idx[idx != top])
        if diff > 0:
            idx = idx[d[idx] < dmax][:diff]
            d[idx] += 1
        else:
            idx = idx[d[idx] > 1][:-diff]
            d[idx] -= 1
    return d


def powerlaw_csr(rows: int, cols: int, mean: int, dmax: int, seed: int, alpha: float = 2.1) -> CSR:
    """Heavy-tailed row degrees, uniform distinct columns, values N(0,1)/sqrt(row degree)."""
    rs = streams(seed)
    d = pareto_degrees(rows, mean, dmax, alpha, rs[0])
    col = distinct_sorted_columns(rs[0], d, cols)
    deg = np.repeat(d, d).astype(np.float32)
    vals = normal_f32(rs[1], col.shape[0]) / np.sqrt(deg)
    return CSR(rows, cols, rowptr_from_lengths(d), col, vals.astype(np.float32))


# ---------------------------------------------------------------------------
# Many independent uneven tiles.
# ---------------------------------------------------------------------------
def uneven_tiles(count: int, seed: int, rows_lo: int = 1024, rows_hi: int = 65536,
                 per_row_lo: int = 4, per_row_hi: int = 256,
                 widths: Sequence[int] = (32, 64, 128, 256)) -> Tuple[List[CSR], List[int]]:
    """``count`` square tiles: rows log-uniform in [rows_lo, rows_hi]; each tile draws one
    per-row count r_t uniform in [per_row_lo, per_row_hi] (capped at the tile width) and
    every row holds r_t distinct uniform columns; values U[-1,1); dense width N_t drawn
    uniformly from ``widths``."""
    rs = streams(seed)
    rows = np.rint(np.exp(rs[2].uniform(math.log(rows_lo), math.log(rows_hi), size=count))).astype(np.int64)
    per_row = rs[2].integers(per_row_lo, per_row_hi + 1, size=count)
    per_row = np.minimum(per_row, rows)
    widths_t = rs[2].choice(np.asarray(widths, dtype=np.int64), size=count)
    tiles = []
    for t in range(count):
        m = int(rows[t])
        lengths = np.full(m, int(per_row[t]), dtype=np.int64)
        col = distinct_sorted_columns(rs[0], lengths, m)
        tiles.append(CSR(m, m, rowptr_from_lengths(lengths), col, uniform_pm1(rs[1], col.shape[0])))
    return tiles, [int(w) for w in widths_t]


# ---------------------------------------------------------------------------
# Dense operands (row-major).
# ---------------------------------------------------------------------------
def dense(rows: int, n: int, rng: np.random.Generator, kind: str = "pm1") -> np.ndarray:
    if kind == "pm1":
        return uniform_pm1(rng, (rows, n))
    if kind == "normal":
        return normal_f32(rng, (rows, n))
    return draw_values(rng, rows * n, kind).reshape(rows, n)
