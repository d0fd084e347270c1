"""FP64 CPU oracle for the local SpMM, its backward, BF16 rounding and the local SpGEMM.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package's smoke check
and by the bench's CPU-baseline leg, never by the product path.  The arithmetic
lives in ``oracle.c`` (plain C, OpenMP over rows, double precision); this module
only marshals NumPy arrays into it.  See ``oracle.c`` for the passages of the
paper each routine follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i64 = ctypes.c_int64
_int = ctypes.c_int
_vp = ctypes.c_void_p


def build(force: bool = True, src: str = _SRC, out: str = _LIB) -> str:
    """Compile ``oracle.c`` (or another source given as ``src``) with gcc -O2 -fopenmp."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wextra", "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def load(path: str) -> ctypes.CDLL:
    """Open a build of ``oracle.c`` and declare its signatures."""
    L = ctypes.CDLL(path)
    L.oracle_spmm.restype = None
    L.oracle_spmm.argtypes = [_i64, _vp, _int, _int, _vp, _vp, _vp, _vp, _vp,
                              _i64, _int, _vp, _i64, _vp, _vp, _i64]
    L.oracle_sddmm.restype = None
    L.oracle_sddmm.argtypes = [_i64, _vp, _vp, _i64, _vp, _vp, _i64, _vp, _i64, _i64, _vp, _vp]
    L.oracle_spmm_t.restype = _int
    L.oracle_spmm_t.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp, _i64, _i64, _i64, _vp, _vp, _vp, _i64]
    L.oracle_transpose.restype = None
    L.oracle_transpose.argtypes = [_i64, _i64, _vp, _vp, _vp, _vp, _vp]
    L.oracle_f32_to_bf16.restype = None
    L.oracle_f32_to_bf16.argtypes = [_i64, _vp, _vp]
    L.oracle_spgemm_count.restype = _int
    L.oracle_spgemm_count.argtypes = [_i64, _vp, _vp, _vp, _vp, _vp, _i64, _vp]
    L.oracle_spgemm_fill.restype = _int
    L.oracle_spgemm_fill.argtypes = [_i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _vp, _vp, _vp]
    return L


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = load(_LIB)
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr_array(arrs):
    return (ctypes.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])


def spmm(tiles: Sequence[Tuple[np.ndarray, np.ndarray, np.ndarray]], Bs: Sequence[np.ndarray],
         k_offset: int = 0, accumulate: bool = False, C0: Optional[np.ndarray] = None,
         rows: Optional[np.ndarray] = None, scale: bool = True) -> Tuple[np.ndarray, Optional[np.ndarray]]:
    """C = acc*C0 + sum_k A_k B_k over a tile row (k visited from ``k_offset``), in FP64.

    ``tiles[k]`` = (rowptr, colind, values) with tile-local columns; ``Bs[k]`` is a
    2-D FP32 array (cols_k x N, any leading dimension).  ``rows`` restricts the
    output to the listed rows.  Returns (C64, S) with S = sum |a||b| (or None).
    """
    K = len(tiles)
    assert K == len(Bs) and K >= 1
    M = tiles[0][0].shape[0] - 1
    N = Bs[0].shape[1]
    rp = [_c(t[0], np.int32) for t in tiles]
    ci = [_c(t[1], np.int32) for t in tiles]
    va = [_c(t[2], np.float32) for t in tiles]
    bs = []
    ldb = np.zeros(K, dtype=np.int64)
    for k, B in enumerate(Bs):
        assert B.dtype == np.float32 and B.ndim == 2 and B.shape[1] == N and B.strides[1] == 4
        bs.append(B)
        ldb[k] = B.strides[0] // 4
    rows_a = None if rows is None else _c(rows, np.int64)
    n_out = M if rows_a is None else rows_a.shape[0]
    C = np.empty((n_out, N), dtype=np.float64)
    S = np.empty((n_out, N), dtype=np.float64) if scale else None
    ldc0 = 0
    if accumulate:
        assert C0 is not None and C0.dtype == np.float32 and C0.strides[1] == 4
        ldc0 = C0.strides[0] // 4
    lib().oracle_spmm(n_out, _ptr(rows_a), K, int(k_offset), _ptr_array(rp), _ptr_array(ci), _ptr_array(va),
                      _ptr_array(bs), ldb.ctypes.data, N, int(bool(accumulate)),
                      _ptr(C0) if accumulate else None, ldc0, C.ctypes.data, _ptr(S), N)
    return C, S


def sddmm(rowptr: np.ndarray, colind: np.ndarray, dC: np.ndarray, B: np.ndarray,
          entries: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """dA[p] = <dC[row(p), :], B[colind[p], :]> in FP64 (all p, or the listed ones)."""
    rowptr = _c(rowptr, np.int32)
    colind = _c(colind, np.int32)
    assert dC.dtype == np.float32 and B.dtype == np.float32 and dC.shape[1] == B.shape[1]
    M = rowptr.shape[0] - 1
    ent = None if entries is None else _c(entries, np.int64)
    n = colind.shape[0] if ent is None else ent.shape[0]
    dA = np.empty(n, dtype=np.float64)
    S = np.empty(n, dtype=np.float64)
    lib().oracle_sddmm(M, rowptr.ctypes.data, colind.ctypes.data, n, _ptr(ent), dC.ctypes.data,
                       dC.strides[0] // 4, B.ctypes.data, B.strides[0] // 4, B.shape[1],
                       dA.ctypes.data, S.ctypes.data)
    return dA, S


def spmm_t(rowptr: np.ndarray, colind: np.ndarray, values: np.ndarray, K: int, dC: np.ndarray,
           out_rows: Optional[np.ndarray] = None) -> Tuple[np.ndarray, np.ndarray]:
    """dB = A^T dC in FP64 by direct scatter (all K rows of dB, or the listed ones)."""
    rowptr = _c(rowptr, np.int32)
    colind = _c(colind, np.int32)
    values = _c(values, np.float32)
    assert dC.dtype == np.float32 and dC.strides[1] == 4
    M = rowptr.shape[0] - 1
    N = dC.shape[1]
    orow = None if out_rows is None else _c(out_rows, np.int64)
    n_out = K if orow is None else orow.shape[0]
    dB = np.empty((n_out, N), dtype=np.float64)
    S = np.empty((n_out, N), dtype=np.float64)
    rc = lib().oracle_spmm_t(M, K, rowptr.ctypes.data, colind.ctypes.data, values.ctypes.data,
                             dC.ctypes.data, dC.strides[0] // 4, N, n_out, _ptr(orow),
                             dB.ctypes.data, S.ctypes.data, N)
    if rc != 0:
        raise MemoryError("oracle_spmm_t could not allocate its slot map")
    return dB, S


def transpose(rowptr: np.ndarray, colind: np.ndarray, K: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(rowptrT[K+1], colindT[nnz], perm[nnz]) by a stable counting sort on columns."""
    rowptr = _c(rowptr, np.int32)
    colind = _c(colind, np.int32)
    M = rowptr.shape[0] - 1
    nnz = colind.shape[0]
    rpT = np.empty(K + 1, dtype=np.int32)
    ciT = np.empty(nnz, dtype=np.int32)
    perm = np.empty(nnz, dtype=np.int32)
    lib().oracle_transpose(M, K, rowptr.ctypes.data, colind.ctypes.data, rpT.ctypes.data,
                           ciT.ctypes.data, perm.ctypes.data)
    return rpT, ciT, perm


def f32_to_bf16(x: np.ndarray) -> np.ndarray:
    """FP32 -> BF16 bit patterns (uint16), round to nearest even."""
    x = _c(x, np.float32)
    y = np.empty(x.shape, dtype=np.uint16)
    lib().oracle_f32_to_bf16(x.size, x.ctypes.data, y.ctypes.data)
    return y


def bf16_to_f32(h: np.ndarray) -> np.ndarray:
    """BF16 bit patterns (uint16) -> FP32, exact widening."""
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def spgemm(A: Tuple[np.ndarray, np.ndarray, np.ndarray], B: Tuple[np.ndarray, np.ndarray, np.ndarray], N: int,
           rows: Optional[np.ndarray] = None, scale: bool = True
           ) -> Tuple[np.ndarray, np.ndarray, np.ndarray, Optional[np.ndarray]]:
    """C = A B for CSR A (rowptr, colind, values) and B (K x N), in FP64.

    Returns (rowptr int64[n_out+1], colind int64[nnz], values float64[nnz], S) for the
    output rows ``rows`` (or all rows of A), columns sorted within each row, the
    pattern structural (products that cancel keep their entry); S = sum |a||b| per entry.
    """
    rpA, ciA, vaA = _c(A[0], np.int32), _c(A[1], np.int32), _c(A[2], np.float32)
    rpB, ciB, vaB = _c(B[0], np.int32), _c(B[1], np.int32), _c(B[2], np.float32)
    M = rpA.shape[0] - 1
    rows_a = None if rows is None else _c(rows, np.int64)
    n_out = M if rows_a is None else rows_a.shape[0]
    counts = np.empty(n_out, dtype=np.int64)
    if lib().oracle_spgemm_count(n_out, _ptr(rows_a), rpA.ctypes.data, ciA.ctypes.data, rpB.ctypes.data,
                                 ciB.ctypes.data, int(N), counts.ctypes.data) != 0:
        raise MemoryError("oracle_spgemm_count could not allocate its marker array")
    rowptr = np.zeros(n_out + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    colC = np.empty(max(nnz, 1), dtype=np.int64)
    valC = np.empty(max(nnz, 1), dtype=np.float64)
    S = np.empty(max(nnz, 1), dtype=np.float64) if scale else None
    if lib().oracle_spgemm_fill(n_out, _ptr(rows_a), rpA.ctypes.data, ciA.ctypes.data, vaA.ctypes.data,
                                rpB.ctypes.data, ciB.ctypes.data, vaB.ctypes.data, int(N), rowptr.ctypes.data,
                                colC.ctypes.data, valC.ctypes.data, _ptr(S)) != 0:
        raise MemoryError("oracle_spgemm_fill could not allocate its accumulators")
    return rowptr, colC[:nnz], valC[:nnz], (S[:nnz] if S is not None else None)
