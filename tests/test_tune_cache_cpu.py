"""The autotune cache's file logic (fingerprints, keys, merge, load) with stand-in handles:
the library's variant getter and setters are replaced by a dictionary, so no GPU is needed."""
import json

import pytest
import torch

from paper_2311_18141_amd import ops, tune_cache


class FakeTile:
    def __init__(self, rows, nnz, cols, max_row=9):
        self.rows, self.cols = rows, [cols]
        self._st = {"rows": rows, "num_k": 1, "nnz_total": nnz, "max_row": max_row, "empty_rows": 0,
                    "long_row": 128, "segment": 64, "hot_rows": 0, "nnz_per_k": [nnz],
                    "hist_log2": [0] * 33}

    def stats(self):
        return dict(self._st)


@pytest.fixture
def table(monkeypatch):
    store = {}

    def get(t, N, dtype=torch.float32, bwd=False):
        return store.get((id(t), N, dtype, bwd))

    def setter(bwd):
        def f(t, N, dtype=torch.float32, kind="auto", lanes=0, vec=0, *depth):
            entry = {"kind": kind, "lanes": lanes, "vec": vec}
            if bwd and kind == "fused":
                entry["depth"] = depth[0] if depth else 0
            store[(id(t), N, dtype, bwd)] = entry
        return f

    monkeypatch.setattr(ops, "spmm_tile_get_variant", get)
    monkeypatch.setattr(ops, "spmm_tile_set_variant", setter(False))
    monkeypatch.setattr(ops, "spmm_tile_set_bwd_variant", setter(True))
    return store


def test_save_then_load_on_new_handles(tmp_path, table):
    path = str(tmp_path / "tune.json")
    a, b, c = FakeTile(100, 900, 80), FakeTile(200, 1500, 90), FakeTile(300, 10, 70)
    ops.spmm_tile_set_variant(a, 64, torch.float32, "stream", 0, 2)
    ops.spmm_tile_set_variant(b, 128, torch.float32, "rowsplit", 16, 4)
    assert tune_cache.save(path, [a, b, c], [64, 128, 32]) == 2          # c has no entry
    a2, b2, other = FakeTile(100, 900, 80), FakeTile(200, 1500, 90), FakeTile(100, 901, 80)
    assert tune_cache.load(path, [a2, b2, other], [64, 128, 64]) == 2
    assert ops.spmm_tile_get_variant(a2, 64) == {"kind": "stream", "lanes": 0, "vec": 2}
    assert ops.spmm_tile_get_variant(b2, 128) == {"kind": "rowsplit", "lanes": 16, "vec": 4}
    assert ops.spmm_tile_get_variant(other, 64) is None                  # another structure
    # width, dtype and direction are part of the key
    a3 = FakeTile(100, 900, 80)
    assert tune_cache.load(path, [a3], [32]) == 0
    assert tune_cache.load(path, [a3], [64], torch.bfloat16) == 0
    assert tune_cache.load(path, [a3], [64], bwd=True) == 0


def test_merge_and_bwd_entries(tmp_path, table):
    path = str(tmp_path / "tune.json")
    a, b = FakeTile(10, 50, 10), FakeTile(20, 70, 20)
    ops.spmm_tile_set_variant(a, 32, torch.float32, "stream", 0, 1)
    tune_cache.save(path, [a], [32])
    ops.spmm_tile_set_bwd_variant(b, 32, torch.bfloat16, "rowsplit", 64, 8)
    tune_cache.save(path, [b], [32], torch.bfloat16, bwd=True)
    entries = tune_cache.read(path)
    assert len(entries) == 2
    assert sorted(k.split("|", 1)[1] for k in entries) == ["32|bf16|bwd", "32|f32|fwd"]
    b2 = FakeTile(20, 70, 20)
    assert tune_cache.load(path, [b2], [32], torch.bfloat16, bwd=True) == 1
    assert ops.spmm_tile_get_variant(b2, 32, torch.bfloat16, bwd=True)["lanes"] == 64
    # a fused backward entry keeps its depth (entries in flight per group)
    c = FakeTile(30, 90, 30)
    ops.spmm_tile_set_bwd_variant(c, 128, torch.float32, "fused", 32, 4, 2)
    tune_cache.save(path, [c], [128], bwd=True)
    c2 = FakeTile(30, 90, 30)
    assert tune_cache.load(path, [c2], [128], bwd=True) == 1
    assert ops.spmm_tile_get_variant(c2, 128, bwd=True) == {"kind": "fused", "lanes": 32, "vec": 4, "depth": 2}
    assert not list(tmp_path.glob("*.tmp*"))


def test_rejects_foreign_files_and_mismatched_lists(tmp_path, table):
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"version": 99, "entries": {}}))
    with pytest.raises(ValueError):
        tune_cache.read(str(path))
    path.write_text(json.dumps([1, 2]))
    with pytest.raises(ValueError):
        tune_cache.load(str(path), [FakeTile(1, 1, 1)], [8])
    with pytest.raises(ValueError):
        tune_cache.save(str(tmp_path / "x.json"), [FakeTile(1, 1, 1)], [8, 16])
    assert tune_cache.read(str(tmp_path / "missing.json")) == {}


def test_fingerprint_tracks_structure():
    a, b = FakeTile(100, 900, 80), FakeTile(100, 900, 80)
    assert tune_cache.fingerprint(a) == tune_cache.fingerprint(b)
    for other in (FakeTile(101, 900, 80), FakeTile(100, 901, 80), FakeTile(100, 900, 81), FakeTile(100, 900, 80, 10)):
        assert tune_cache.fingerprint(other) != tune_cache.fingerprint(a)
