"""Autotune cache: the kernel variants an autotuner chose, kept in a JSON file and applied
to later handles of the same structure, so that a process need not time the candidates
again (timing every tile of a 512-tile batch takes seconds).

A handle is identified by a fingerprint of the structure the library reports for it:
rows, k-tiles, non-zeros per k-tile, longest row, empty rows, the row-length histogram
and the split plan.  A variant only changes how the work is laid out on the GPU, never
which products are summed, so an entry applied to another matrix with the same
fingerprint can cost speed but not correctness (results stay within the rounding of the
FP32 sums, and equal bit for bit on integer data).

File format: ``{"version": 1, "entries": {key: {"kind", "lanes", "vec", "depth"}}}`` with
``key = "<fingerprint>|<N>|<f32|bf16>|<fwd|bwd>"``; written atomically.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional, Sequence

import torch

from . import ops

VERSION = 1
_DT = {torch.float32: "f32", torch.bfloat16: "bf16"}
_FIELDS = ("rows", "num_k", "nnz_total", "max_row", "empty_rows", "long_row", "segment", "hot_rows")


def fingerprint(tile: ops.Tile) -> str:
    """A short hash of the handle's structural statistics."""
    st = tile.stats()
    key = {f: int(st[f]) for f in _FIELDS}
    key["nnz_per_k"] = [int(x) for x in st["nnz_per_k"]]
    key["hist_log2"] = [int(x) for x in st["hist_log2"]]
    key["cols"] = [int(c) for c in tile.cols]
    return hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:32]


def _key(fp: str, N: int, dtype, bwd: bool) -> str:
    if dtype not in _DT:
        raise ValueError("dtype must be float32 or bfloat16")
    return "%s|%d|%s|%s" % (fp, int(N), _DT[dtype], "bwd" if bwd else "fwd")


def read(path: str) -> Dict[str, dict]:
    """The file's entries ({} when it does not exist)."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    if not isinstance(data, dict) or data.get("version") != VERSION or not isinstance(data.get("entries"), dict):
        raise ValueError("%s is not a version-%d autotune cache" % (path, VERSION))
    return data["entries"]


def _write(path: str, entries: Dict[str, dict]) -> None:
    tmp = "%s.tmp%d" % (path, os.getpid())
    with open(tmp, "w") as f:
        json.dump({"version": VERSION, "entries": entries}, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def save(path: str, tiles: Sequence[ops.Tile], Ns: Sequence[int], dtype=torch.float32, bwd: bool = False) -> int:
    """Add every tile's variant entry for its width to the file (merging with what it
    holds); tiles without an entry are skipped.  Returns the number of entries written."""
    if len(tiles) != len(Ns):
        raise ValueError("one N per tile")
    entries = read(path)
    n = 0
    for t, N in zip(tiles, Ns):
        v = ops.spmm_tile_get_variant(t, int(N), dtype, bwd=bwd)
        if v is None:
            continue
        entries[_key(fingerprint(t), N, dtype, bwd)] = {"kind": v["kind"], "lanes": int(v["lanes"]),
                                                        "vec": int(v["vec"]), "depth": int(v.get("depth", 0))}
        n += 1
    _write(path, entries)
    return n


def load(path: str, tiles: Sequence[ops.Tile], Ns: Sequence[int], dtype=torch.float32, bwd: bool = False,
         entries: Optional[Dict[str, dict]] = None) -> int:
    """Set the variant of every tile whose fingerprint, width and dtype the file holds.
    Returns the number of tiles set."""
    if len(tiles) != len(Ns):
        raise ValueError("one N per tile")
    entries = read(path) if entries is None else entries
    setter = ops.spmm_tile_set_bwd_variant if bwd else ops.spmm_tile_set_variant
    n = 0
    for t, N in zip(tiles, Ns):
        e = entries.get(_key(fingerprint(t), N, dtype, bwd))
        if e is None:
            continue
        if bwd:
            setter(t, int(N), dtype, e["kind"], int(e["lanes"]), int(e["vec"]), int(e.get("depth", 0)))
        else:
            setter(t, int(N), dtype, e["kind"], int(e["lanes"]), int(e["vec"]))
        n += 1
    return n


def autotune(path: str, tiles: Sequence[ops.Tile], Bs: Sequence[torch.Tensor], Cs: Sequence[torch.Tensor]) -> dict:
    """Forward variants for single-tile handles: taken from the file where it has them,
    timed by spmm_tile_autotune (variant only, the split plan kept) where it does not,
    and the file updated.  C_t is overwritten for the tiles that are timed."""
    if not (len(tiles) == len(Bs) == len(Cs)):
        raise ValueError("one B and one C per tile")
    Ns = [int(B.shape[1]) for B in Bs]
    dtypes = {B.dtype for B in Bs}
    if len(dtypes) != 1:
        raise ValueError("all B must share one dtype")
    dtype = dtypes.pop()
    entries = read(path)
    hits = tuned = 0
    for t, B, C, N in zip(tiles, Bs, Cs, Ns):
        if load(path, [t], [N], dtype, entries=entries):
            hits += 1
            continue
        ops.spmm_tile_autotune(t, [B], C, tune_plan=False)
        tuned += 1
    save(path, tiles, Ns, dtype)
    return {"from_cache": hits, "tuned": tuned}
