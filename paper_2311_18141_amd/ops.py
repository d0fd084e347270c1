"""Python binding of the C ABI with the same names (include/spmm.h).

PyTorch tensors supply device memory and the current HIP stream; every step of
the computation runs in libspmm's kernels.  Tensors handed to spmm_tile_create
are kept referenced by the returned Tile so that they outlive the handle.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import SpmmCsr, SpmmError, SpmmTileOpts, SpmmTileStats, SpmmVariant, check, lib

_DTYPES = {torch.float32: _lib.SPMM_F32, torch.bfloat16: _lib.SPMM_BF16}


def _stream_ptr(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _need(t: torch.Tensor, dtype, name: str):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _row_major_ld(t: torch.Tensor, name: str) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("%s must be a 2-D row-major tensor (unit column stride)" % name)
    return max(t.stride(0), t.shape[1])


class Tile:
    """A tile-row handle: num_k CSR tiles sharing their rows (one tile for num_k = 1)."""

    def __init__(self, handle: int, rows: int, cols: List[int], nnz: List[int], keep: list, values: List[torch.Tensor]):
        self.handle = handle
        self.rows = rows
        self.cols = cols
        self.nnz = nnz
        self.values = values
        self._keep = keep
        self._ws = {}

    @property
    def num_k(self) -> int:
        return len(self.cols)

    def stats(self) -> dict:
        st = SpmmTileStats()
        check(lib().spmm_tile_get_stats(self.handle, ctypes.byref(st)))
        out = {f: getattr(st, f) for f, _ in SpmmTileStats._fields_}
        out["hist_log2"] = list(st.hist_log2)
        out["nnz_per_k"] = list(st.nnz_per_k)[: self.num_k]
        return out

    def workspace(self, N: int, kind: str = "fwd") -> Optional[torch.Tensor]:
        """A cached device workspace large enough for spmm_fwd / spmm_bwd at width N."""
        nbytes = spmm_fwd_workspace_bytes(self, N) if kind == "fwd" else spmm_bwd_workspace_bytes(self, N)
        if nbytes == 0:
            return None
        ws = self._ws.get(kind)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.values[0].device)
            self._ws[kind] = ws
        return ws

    def close(self):
        if self.handle:
            check(lib().spmm_tile_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spmm_tile_create(rows: int, tiles: Sequence[Tuple[torch.Tensor, torch.Tensor, torch.Tensor, int]],
                     validate: bool = False, transpose: bool = False, long_row: int = 0, segment: int = 0,
                     bwd_slice: int = 0, hot_rows: int = 0, stream: Optional[torch.cuda.Stream] = None) -> Tile:
    """Create a handle from k-tiles given as (rowptr int32, colind int32, values float32, cols).

    hot_rows: forward hot-row staging, -1 off, 0 library rule, n > 0 up to n rows per k-tile."""
    K = len(tiles)
    arr = (SpmmCsr * max(K, 1))()
    keep = []
    cols, nnz, vals = [], [], []
    for k, (rp, ci, va, nc) in enumerate(tiles):
        _need(rp, torch.int32, "rowptr")
        _need(ci, torch.int32, "colind")
        _need(va, torch.float32, "values")
        if rp.numel() != rows + 1:
            raise ValueError("rowptr of tile %d has %d entries, expected %d" % (k, rp.numel(), rows + 1))
        if ci.numel() != va.numel():
            raise ValueError("colind and values of tile %d differ in length" % k)
        arr[k].cols = int(nc)
        arr[k].nnz = ci.numel()
        arr[k].rowptr = rp.data_ptr()
        arr[k].colind = ci.data_ptr() if ci.numel() else None
        arr[k].values = va.data_ptr() if va.numel() else None
        keep += [rp, ci, va]
        cols.append(int(nc))
        nnz.append(ci.numel())
        vals.append(va)
    opts = SpmmTileOpts()
    opts.flags = (_lib.SPMM_TILE_VALIDATE if validate else 0) | (_lib.SPMM_TILE_TRANSPOSE if transpose else 0)
    opts.long_row = long_row
    opts.segment = segment
    opts.bwd_slice = bwd_slice
    opts.hot_rows = hot_rows
    h = ctypes.c_void_p()
    check(lib().spmm_tile_create(rows, K, arr, ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(h)))
    return Tile(h.value, rows, cols, nnz, keep, vals)


def spmm_tile_destroy(tile: Tile) -> None:
    tile.close()


def spmm_tile_export_transpose(tile: Tile, stream=None) -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    dev = tile.values[0].device
    rpT = torch.empty(tile.cols[0] + 1, dtype=torch.int32, device=dev)
    ciT = torch.empty(tile.nnz[0], dtype=torch.int32, device=dev)
    perm = torch.empty(tile.nnz[0], dtype=torch.int32, device=dev)
    check(lib().spmm_tile_export_transpose(tile.handle, rpT.data_ptr(), ciT.data_ptr() if tile.nnz[0] else None,
                                           perm.data_ptr() if tile.nnz[0] else None, _stream_ptr(stream)))
    return rpT, ciT, perm


KERNELS = {"auto": _lib.SPMM_KERNEL_AUTO, "rowsplit": _lib.SPMM_KERNEL_ROWSPLIT, "stream": _lib.SPMM_KERNEL_STREAM,
           "fused": _lib.SPMM_KERNEL_FUSED}


def spmm_tile_set_variant(tile: Tile, N: int, dtype=torch.float32, kind: Optional[str] = "auto",
                          lanes: int = 0, vec: int = 0) -> None:
    """Pin the forward kernel variant for width N (kind None clears the entry)."""
    if kind is None:
        check(lib().spmm_tile_set_variant(tile.handle, N, _DTYPES[dtype], None))
        return
    v = SpmmVariant(KERNELS[kind], lanes, vec)
    check(lib().spmm_tile_set_variant(tile.handle, N, _DTYPES[dtype], ctypes.byref(v)))


def spmm_tile_set_bwd_variant(tile: Tile, N: int, dtype=torch.float32, kind: Optional[str] = "auto",
                              lanes: int = 0, vec: int = 0, depth: int = 0) -> None:
    """Pin the backward's variant for width N: "fused" (lanes, vec, depth = entries in flight per
    group) or the two-pass form's dB-pass kernel ("rowsplit", "stream"); kind None clears the entry."""
    if kind is None:
        check(lib().spmm_tile_set_bwd_variant(tile.handle, N, _DTYPES[dtype], None))
        return
    v = SpmmVariant(KERNELS[kind], lanes, vec, depth)
    check(lib().spmm_tile_set_bwd_variant(tile.handle, N, _DTYPES[dtype], ctypes.byref(v)))


def spmm_tile_get_variant(tile: Tile, N: int, dtype=torch.float32, bwd: bool = False) -> Optional[dict]:
    """The forward's (or, with bwd, the dB pass's) variant entry for width N; None when unset."""
    v = SpmmVariant()
    check(lib().spmm_tile_get_variant(tile.handle, N, _DTYPES[dtype], 1 if bwd else 0, ctypes.byref(v)))
    if v.kind == KERNELS["auto"]:
        return None
    inv = {val: k for k, val in KERNELS.items()}
    out = {"kind": inv[v.kind], "lanes": v.lanes, "vec": v.vec}
    if v.kind == KERNELS["fused"]:
        out["depth"] = v.depth
    return out


def spmm_tile_autotune_bwd(tile: Tile, dC: torch.Tensor, dB: Optional[torch.Tensor] = None,
                           B: Optional[torch.Tensor] = None, dA: Optional[torch.Tensor] = None,
                           stream: Optional[torch.cuda.Stream] = None) -> dict:
    """Time the backward's variants on these operands and keep the fastest (dB, and dA when
    given, are overwritten).  With B given the whole backward is timed, fused shapes included;
    without it only the dB pass's kernels."""
    dt = dC.dtype
    if dt not in _DTYPES:
        raise ValueError("dC must be float32 or bfloat16")
    N = dC.shape[1]
    if dC.shape != (tile.rows, N):
        raise ValueError("dC must be (%d, N)" % tile.rows)
    if dB is None:
        dB = torch.empty(tile.cols[0], N, dtype=dt, device=dC.device)
    if dB.dtype != dt or dB.shape != (tile.cols[0], N):
        raise ValueError("dB must be %s of shape (%d, %d)" % (dt, tile.cols[0], N))
    ldb = 0
    if B is not None:
        if B.dtype != dt or B.shape != (tile.cols[0], N):
            raise ValueError("B must be %s of shape (%d, %d)" % (dt, tile.cols[0], N))
        ldb = _row_major_ld(B, "B")
        if dA is None:
            dA = torch.empty(tile.nnz[0], dtype=torch.float32, device=dC.device)
        if dA.dtype != torch.float32 or dA.numel() < tile.nnz[0]:
            raise ValueError("dA must be float32 with nnz entries")
    out = SpmmVariant()
    check(lib().spmm_tile_autotune_bwd(tile.handle, N, _DTYPES[dt], dC.data_ptr(), _row_major_ld(dC, "dC"),
                                       B.data_ptr() if B is not None else None, ldb,
                                       dA.data_ptr() if B is not None else None,
                                       dB.data_ptr(), _row_major_ld(dB, "dB"), _stream_ptr(stream), ctypes.byref(out)))
    inv = {v: k for k, v in KERNELS.items()}
    res = {"kind": inv[out.kind], "lanes": out.lanes, "vec": out.vec}
    if out.kind == KERNELS["fused"]:
        res["depth"] = out.depth
    return res


def spmm_tile_set_sddmm_variant(tile: Tile, N: int, lanes: int = 0, nnz_per_group: int = 4) -> None:
    """Shape of the backward's SDDMM kernel at width N (lanes = 0: library choice)."""
    check(lib().spmm_tile_set_sddmm_variant(tile.handle, N, lanes, nnz_per_group if lanes else 0))


def spmm_tile_autotune(tile: Tile, Bs: Sequence[torch.Tensor], C: torch.Tensor, tune_plan: bool = True,
                       stream: Optional[torch.cuda.Stream] = None) -> dict:
    """Time the forward variants (and split thresholds) on these operands; keep the fastest."""
    K = tile.num_k
    ptrs = (ctypes.c_void_p * K)(*[B.data_ptr() for B in Bs])
    lds = (ctypes.c_int64 * K)(*[_row_major_ld(B, "B") for B in Bs])
    dt = Bs[0].dtype
    N = Bs[0].shape[1]
    out = SpmmVariant()
    check(lib().spmm_tile_autotune(tile.handle, N, _DTYPES[dt], ptrs, lds, C.data_ptr(), _row_major_ld(C, "C"),
                                   1 if tune_plan else 0, _stream_ptr(stream), ctypes.byref(out)))
    tile._ws.pop("fwd", None)
    inv = {v: k for k, v in KERNELS.items()}
    return {"kind": inv[out.kind], "lanes": out.lanes, "vec": out.vec}


def spmm_fwd_workspace_bytes(tile: Tile, N: int) -> int:
    n = ctypes.c_size_t()
    check(lib().spmm_fwd_workspace_bytes(tile.handle, N, ctypes.byref(n)))
    return n.value


def spmm_bwd_workspace_bytes(tile: Tile, N: int) -> int:
    n = ctypes.c_size_t()
    check(lib().spmm_bwd_workspace_bytes(tile.handle, N, ctypes.byref(n)))
    return n.value


def spmm_fwd(tile: Tile, Bs: Sequence[torch.Tensor], C: Optional[torch.Tensor] = None, k_offset: int = 0,
             accumulate: bool = False, workspace: Optional[torch.Tensor] = None,
             stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """C = [C] + sum_k A_k B_k (k from k_offset).  B_k and C share one dtype (float32 or bfloat16)."""
    K = tile.num_k
    if len(Bs) != K:
        raise ValueError("expected %d dense operands, got %d" % (K, len(Bs)))
    dt = Bs[0].dtype
    if dt not in _DTYPES:
        raise ValueError("dense operands must be float32 or bfloat16")
    N = Bs[0].shape[1]
    ptrs = (ctypes.c_void_p * K)()
    lds = (ctypes.c_int64 * K)()
    for k, B in enumerate(Bs):
        if B.dtype != dt or not B.is_cuda or B.shape[1] != N or B.shape[0] != tile.cols[k]:
            raise ValueError("B[%d] must be a device %s tensor of shape (%d, %d)" % (k, dt, tile.cols[k], N))
        lds[k] = _row_major_ld(B, "B[%d]" % k)
        ptrs[k] = B.data_ptr()
    if C is None:
        if accumulate:
            raise ValueError("accumulate needs C")
        C = torch.empty(tile.rows, N, dtype=dt, device=Bs[0].device)
    if C.dtype != dt or C.shape != (tile.rows, N):
        raise ValueError("C must be %s of shape (%d, %d)" % (dt, tile.rows, N))
    ldc = _row_major_ld(C, "C")
    if workspace is None:
        workspace = tile.workspace(N, "fwd")
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_n = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().spmm_fwd(tile.handle, k_offset, ptrs, lds, _DTYPES[dt], C.data_ptr(), ldc, _DTYPES[dt], N,
                         1 if accumulate else 0, ws_ptr, ws_n, _stream_ptr(stream)))
    return C


def spmm_noalloc_scratch_bytes() -> int:
    """Size of the fixed per-GPU scratch array spmm_fwd_noalloc uses."""
    return int(lib().spmm_noalloc_scratch_bytes())


def spmm_fwd_noalloc(tile: Tile, Bs: Sequence[torch.Tensor], C: torch.Tensor, k_offset: int = 0,
                     accumulate: bool = False, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """spmm_fwd without a workspace (the library's fixed per-GPU scratch array); C is the caller's."""
    K = tile.num_k
    if len(Bs) != K:
        raise ValueError("expected %d dense operands, got %d" % (K, len(Bs)))
    dt = Bs[0].dtype
    if dt not in _DTYPES:
        raise ValueError("dense operands must be float32 or bfloat16")
    N = Bs[0].shape[1]
    ptrs = (ctypes.c_void_p * K)()
    lds = (ctypes.c_int64 * K)()
    for k, B in enumerate(Bs):
        if B.dtype != dt or not B.is_cuda or B.shape[1] != N or B.shape[0] != tile.cols[k]:
            raise ValueError("B[%d] must be a device %s tensor of shape (%d, %d)" % (k, dt, tile.cols[k], N))
        lds[k] = _row_major_ld(B, "B[%d]" % k)
        ptrs[k] = B.data_ptr()
    if C.dtype != dt or C.shape != (tile.rows, N):
        raise ValueError("C must be %s of shape (%d, %d)" % (dt, tile.rows, N))
    check(lib().spmm_fwd_noalloc(tile.handle, k_offset, ptrs, lds, _DTYPES[dt], C.data_ptr(), _row_major_ld(C, "C"),
                                 _DTYPES[dt], N, 1 if accumulate else 0, _stream_ptr(stream)))
    return C


def spmm_bwd(tile: Tile, dC: torch.Tensor, B: torch.Tensor, want_dA: bool = True, want_dB: bool = True,
             dA: Optional[torch.Tensor] = None, dB: Optional[torch.Tensor] = None,
             workspace: Optional[torch.Tensor] = None,
             stream: Optional[torch.cuda.Stream] = None) -> Tuple[Optional[torch.Tensor], Optional[torch.Tensor]]:
    """(dA on A's pattern, dB = A^T dC) for a single-tile handle built with transpose=True.

    dC and B share one dtype (float32 or bfloat16); dA is float32 (A's values are), dB has dC's dtype."""
    if tile.num_k != 1:
        raise ValueError("spmm_bwd needs a single-tile handle")
    N = dC.shape[1]
    dt = dC.dtype
    if dt not in _DTYPES or B.dtype != dt:
        raise ValueError("spmm_bwd takes dC and B of one dtype, float32 or bfloat16")
    if dC.shape != (tile.rows, N) or B.shape != (tile.cols[0], N):
        raise ValueError("dC must be (%d, N) and B (%d, N)" % (tile.rows, tile.cols[0]))
    lddc = _row_major_ld(dC, "dC")
    ldb = _row_major_ld(B, "B")
    if want_dA and dA is None:
        dA = torch.empty(tile.nnz[0], dtype=torch.float32, device=dC.device)
    if want_dB and dB is None:
        dB = torch.empty(tile.cols[0], N, dtype=dt, device=dC.device)
    if want_dA and (dA.dtype != torch.float32 or dA.numel() < tile.nnz[0]):
        raise ValueError("dA must be float32 with nnz entries")
    if want_dB and (dB.dtype != dt or dB.shape != (tile.cols[0], N)):
        raise ValueError("dB must be %s of shape (%d, %d)" % (dt, tile.cols[0], N))
    lddb = _row_major_ld(dB, "dB") if want_dB else 0
    if workspace is None and want_dB:
        workspace = tile.workspace(N, "bwd")
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_n = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().spmm_bwd(tile.handle, dC.data_ptr(), lddc, B.data_ptr(), ldb, N, _DTYPES[dt],
                         dA.data_ptr() if want_dA else None, dB.data_ptr() if want_dB else None, lddb,
                         ws_ptr, ws_n, _stream_ptr(stream)))
    return (dA if want_dA else None), (dB if want_dB else None)


def spmm_tile_accumulate_n(C: torch.Tensor, Ps: Sequence[torch.Tensor],
                           stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """C += Ps[0] + Ps[1] + ... in that order (the owner draining its queue of partial tiles)."""
    if C.dtype not in _DTYPES or not C.is_cuda:
        raise ValueError("C must be a device float32 or bfloat16 tensor")
    for P in Ps:
        if P.dtype != C.dtype or P.shape != C.shape or not P.is_cuda:
            raise ValueError("every partial must be a device tensor of C's shape and dtype")
    n = len(Ps)
    ptrs = (ctypes.c_void_p * max(n, 1))(*[P.data_ptr() for P in Ps])
    lds = (ctypes.c_int64 * max(n, 1))(*[_row_major_ld(P, "P") for P in Ps])
    rows, N = C.shape
    check(lib().spmm_tile_accumulate_n(C.data_ptr(), _row_major_ld(C, "C"), ptrs, lds, n, rows, N, _DTYPES[C.dtype],
                                       _stream_ptr(stream)))
    return C


def spmm_tile_accumulate(C: torch.Tensor, Ptile: torch.Tensor, stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """C += Ptile (the owner-side accumulate of a stationary-A partial product)."""
    if C.dtype != Ptile.dtype or C.dtype not in _DTYPES or C.shape != Ptile.shape or not (C.is_cuda and Ptile.is_cuda):
        raise ValueError("C and Ptile must be device tensors of one shape and dtype (float32 or bfloat16)")
    rows, N = C.shape
    check(lib().spmm_tile_accumulate(C.data_ptr(), _row_major_ld(C, "C"), Ptile.data_ptr(), _row_major_ld(Ptile, "Ptile"),
                                     rows, N, _DTYPES[C.dtype], _stream_ptr(stream)))
    return C


class Batch:
    """A batched launch over many single-tile handles (see spmm_batch_create)."""

    def __init__(self, handle: int, tiles: List[Tile], Ns: List[int], dtype):
        self.handle = handle
        self.tiles = tiles
        self.Ns = Ns
        self.dtype = dtype
        self._ws = None
        self._ptrs = {}

    def workspace_bytes(self) -> int:
        n = ctypes.c_size_t()
        check(lib().spmm_batch_workspace_bytes(self.handle, ctypes.byref(n)))
        return n.value

    def workspace(self) -> Optional[torch.Tensor]:
        nb = self.workspace_bytes()
        if nb == 0:
            return None
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device=self.tiles[0].values[0].device)
        return self._ws

    def variant(self, t: int) -> dict:
        v = SpmmVariant()
        check(lib().spmm_batch_get_variant(self.handle, t, ctypes.byref(v)))
        inv = {val: k for k, val in KERNELS.items()}
        return {"kind": inv[v.kind], "lanes": v.lanes, "vec": v.vec}

    def operand_arrays(self, Bs: Sequence[torch.Tensor], Cs: Sequence[torch.Tensor]):
        """Device arrays of pointers and leading dimensions (cached per set of tensors)."""
        key = tuple(B.data_ptr() for B in Bs) + tuple(C.data_ptr() for C in Cs)
        arr = self._ptrs.get(key)
        if arr is None:
            esize = 4 if self.dtype == torch.float32 else 2
            for t, (B, C) in enumerate(zip(Bs, Cs)):
                if B.dtype != self.dtype or C.dtype != self.dtype:
                    raise ValueError("operand %d has the wrong dtype" % t)
                if B.shape != (self.tiles[t].cols[0], self.Ns[t]) or C.shape != (self.tiles[t].rows, self.Ns[t]):
                    raise ValueError("operand %d has the wrong shape" % t)
                for X, name in ((B, "B"), (C, "C")):
                    ld = _row_major_ld(X, name)
                    if X.data_ptr() % 16 or (ld * esize) % 16:
                        raise ValueError("%s[%d] rows must start on 16-byte boundaries" % (name, t))
            dev = Bs[0].device
            mk = lambda xs: torch.tensor(xs, dtype=torch.int64).to(dev)
            arr = (mk([B.data_ptr() for B in Bs]), mk([_row_major_ld(B, "B") for B in Bs]),
                   mk([C.data_ptr() for C in Cs]), mk([_row_major_ld(C, "C") for C in Cs]))
            self._ptrs = {key: arr}
        return arr

    def close(self):
        if self.handle:
            check(lib().spmm_batch_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spmm_batch_create(tiles: Sequence[Tile], Ns: Sequence[int], dtype=torch.float32, item_nnz: int = 0,
                      persistent: bool = False, single: bool = False,
                      stream: Optional[torch.cuda.Stream] = None) -> Batch:
    """Work list for spmm_batched over single-tile handles (persistent: claim-counter hand-out;
    single: one launch for every kernel class, then a fix-up launch when some tile has split rows)."""
    arr = (ctypes.c_void_p * len(tiles))(*[t.handle for t in tiles])
    ns = (ctypes.c_int64 * len(tiles))(*[int(n) for n in Ns])
    h = ctypes.c_void_p()
    flags = (_lib.SPMM_BATCH_PERSISTENT if persistent else 0) | (_lib.SPMM_BATCH_SINGLE if single else 0)
    check(lib().spmm_batch_create(len(tiles), arr, ns, _DTYPES[dtype], item_nnz, flags,
                                  _stream_ptr(stream), ctypes.byref(h)))
    return Batch(h.value, list(tiles), [int(n) for n in Ns], dtype)


RESERVE_MODES = {"2d": _lib.SPMM_RESERVE_2D, "3d": _lib.SPMM_RESERVE_3D, "own": _lib.SPMM_RESERVE_OWN}


def spmm_batch_create_grid(tiles: Sequence[Tile], Ns: Sequence[int], coords: Sequence[Tuple[int, int, int]],
                           mode: str = "2d", dtype=torch.float32, item_nnz: int = 0,
                           stream: Optional[torch.cuda.Stream] = None) -> Batch:
    """A batch of component products C(i,j) (+)= A(i,k) B(k,j), tile t at coords[t] = (i, j, k), handed
    out through a reservation grid: "2d" (over (i, k), random stealing), "3d" (over (i, j, k),
    locality-aware stealing) or "own" (over (i, k), no stealing)."""
    if len(coords) != len(tiles):
        raise ValueError("one (i, j, k) per tile")
    arr = (ctypes.c_void_p * len(tiles))(*[t.handle for t in tiles])
    ns = (ctypes.c_int64 * len(tiles))(*[int(n) for n in Ns])
    cc = (ctypes.c_int32 * (3 * len(tiles)))(*[int(v) for c in coords for v in c])
    h = ctypes.c_void_p()
    check(lib().spmm_batch_create_grid(len(tiles), arr, ns, _DTYPES[dtype], cc, RESERVE_MODES[mode], item_nnz,
                                       _stream_ptr(stream), ctypes.byref(h)))
    return Batch(h.value, list(tiles), [int(n) for n in Ns], dtype)


def spmm_batched(batch: Batch, Bs: Sequence[torch.Tensor], Cs: Sequence[torch.Tensor], accumulate: bool = False,
                 workspace: Optional[torch.Tensor] = None, stream: Optional[torch.cuda.Stream] = None) -> None:
    """C_t = [C_t] + A_t B_t for every tile of the batch, in the launch form the batch was built with."""
    if len(Bs) != len(batch.tiles) or len(Cs) != len(batch.tiles):
        raise ValueError("one B and one C per tile")
    b, lb, c, lc = batch.operand_arrays(Bs, Cs)
    if workspace is None:
        workspace = batch.workspace()
    ws_ptr = workspace.data_ptr() if workspace is not None else None
    ws_n = workspace.numel() * workspace.element_size() if workspace is not None else 0
    check(lib().spmm_batched(batch.handle, b.data_ptr(), lb.data_ptr(), c.data_ptr(), lc.data_ptr(),
                             1 if accumulate else 0, ws_ptr, ws_n, _stream_ptr(stream)))


# ---------------------------------------------------------------- local SpGEMM

class SpgemmPlan:
    """Plan of C = A B (CSR x CSR): C's structure is known at creation; values come from spgemm_compute."""

    def __init__(self, handle: int, M: int, N: int, nnz_c: int, products: int, keep: list,
                 pattern_entries: int = 0):
        self.handle = handle
        self.M = M
        self.N = N
        self.nnz_c = nnz_c
        self.products = products
        self.pattern_entries = pattern_entries   # entries of C whose columns the plan keeps
        self._keep = keep

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                lib().spgemm_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def _csr_struct(rowptr, colind, values, cols, name):
    for t, dt in ((rowptr, torch.int32), (colind, torch.int32), (values, torch.float32)):
        if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
            raise ValueError("%s arrays must be contiguous device tensors (int32 rowptr/colind, float32 values)" % name)
    return SpmmCsr(int(cols), int(colind.numel()), rowptr.data_ptr(), colind.data_ptr(), values.data_ptr())


def spgemm_create(M: int, A: Tuple[torch.Tensor, torch.Tensor, torch.Tensor, int],
                  B: Tuple[torch.Tensor, torch.Tensor, torch.Tensor, int], validate: bool = True,
                  stream: Optional[torch.cuda.Stream] = None, keep_pattern: bool = True) -> SpgemmPlan:
    """Structure analysis and symbolic product of C = A B (A: M x A.cols, B: A.cols x B.cols).
    keep_pattern=False: keep no column pattern, find the columns on every compute call (SPGEMM_BITMAP_ONLY)."""
    a = _csr_struct(*A, "A")
    b = _csr_struct(*B, "B")
    if A[0].numel() != M + 1 or B[0].numel() != int(A[3]) + 1:
        raise ValueError("A needs M + 1 row pointers and B A.cols + 1")
    h = ctypes.c_void_p()
    flags = (1 if validate else 0) | (0 if keep_pattern else _lib.SPGEMM_BITMAP_ONLY)
    check(lib().spgemm_create(int(M), ctypes.byref(a), ctypes.byref(b), flags, _stream_ptr(stream),
                              ctypes.byref(h)))
    nnz = ctypes.c_int64()
    prods = ctypes.c_int64()
    pat = ctypes.c_int64()
    try:
        check(lib().spgemm_info(h.value, ctypes.byref(nnz), ctypes.byref(prods)))
        check(lib().spgemm_pattern_entries(h.value, ctypes.byref(pat)))
    except Exception:
        lib().spgemm_destroy(h.value)
        raise
    return SpgemmPlan(h.value, int(M), int(B[3]), nnz.value, prods.value, [A, B], pat.value)


def spgemm_rowptr(plan: SpgemmPlan, rowptrC: Optional[torch.Tensor] = None,
                  stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    if rowptrC is None:
        rowptrC = torch.empty(plan.M + 1, dtype=torch.int32, device=plan._keep[0][0].device)
    check(lib().spgemm_rowptr(plan.handle, rowptrC.data_ptr(), _stream_ptr(stream)))
    return rowptrC


def spgemm_compute(plan: SpgemmPlan, colindC: Optional[torch.Tensor] = None, valuesC: Optional[torch.Tensor] = None,
                   stream: Optional[torch.cuda.Stream] = None) -> Tuple[torch.Tensor, torch.Tensor]:
    """C's column indices (sorted per row) and values, reading A's and B's values live."""
    dev = plan._keep[0][0].device
    if colindC is None:
        colindC = torch.empty(max(plan.nnz_c, 1), dtype=torch.int32, device=dev)
    if valuesC is None:
        valuesC = torch.empty(max(plan.nnz_c, 1), dtype=torch.float32, device=dev)
    if colindC.numel() < plan.nnz_c or valuesC.numel() < plan.nnz_c:
        raise ValueError("outputs need nnz(C) = %d entries" % plan.nnz_c)
    check(lib().spgemm_compute(plan.handle, colindC.data_ptr(), valuesC.data_ptr(), _stream_ptr(stream)))
    return colindC[:plan.nnz_c], valuesC[:plan.nnz_c]


def spmm_gather_probe(table: torch.Tensor, row_bytes: int, idx: torch.Tensor, out: Optional[torch.Tensor] = None,
                      stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """Gather micro-benchmark: read rows idx of `table` (a contiguous device tensor viewed as
    rows of `row_bytes` bytes) whole; returns a one-word device tensor with the XOR of every
    32-bit word read."""
    if not table.is_cuda or not table.is_contiguous():
        raise ValueError("table must be a contiguous device tensor")
    nbytes = table.numel() * table.element_size()
    if row_bytes <= 0 or nbytes % row_bytes:
        raise ValueError("table size %d is not a multiple of row_bytes %d" % (nbytes, row_bytes))
    _need(idx, torch.int32, "idx")
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=table.device)
    check(lib().spmm_gather_probe(table.data_ptr(), nbytes // row_bytes, row_bytes, idx.data_ptr() if idx.numel() else None,
                                  idx.numel(), out.data_ptr(), _stream_ptr(stream)))
    return out
