"""Host logic of bench.py (no GPU): the one-GPU refusal, the workload registry and its pinned
configurations, and the stored counter readings' parser with its kernel-source check."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_registry_and_pins():
    names = set(bench.workloads())
    assert "powerlaw2m_n128_fwdbwd" in names             # the default workload
    assert set(bench.PINNED) <= names
    for name, pin in bench.PINNED.items():
        kind, lanes, vec = pin["variant"]
        assert kind in ("stream", "rowsplit") and lanes in (4, 8, 16, 32, 64) and vec in (1, 2, 4, 8)
        assert pin["long_row"] > 0 and pin["segment"] > 0
        if "bwd_variant" in pin:                          # the fused backward: (kind, lanes, vec, depth)
            kind, lanes, vec, depth = pin["bwd_variant"]
            assert kind == "fused" and lanes in (4, 8, 16, 32, 64) and vec in (1, 2, 4, 8)
            assert depth in (1, 2, 4, 8) and depth <= lanes


def test_stored_traffic_parser(tmp_path, monkeypatch):
    wl = "rmat22_rowblock0_4x4_n128"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    csrc = tmp_path / "paper_2311_18141_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.FWD_SOURCES + ("bwd.hip",):
        (csrc / name).write_text("// %s\n" % name)
    assert bench.stored_traffic(wl) is None                 # no file
    good = bench.kernel_source_digest(wl)
    f = tmp_path / "profiles" / ("traffic_%s.md" % wl)
    f.write_text("# t\n\n- hbm_bytes_per_step: 12345\n- source_sha256: %s\n" % good)
    assert bench.stored_traffic(wl) == 12345.0
    (csrc / "fwd.hip").write_text("// changed\n")             # kernels changed since the reading
    assert bench.stored_traffic(wl) is None
    # the backward workload also depends on bwd.hip
    assert bench.kernel_source_digest("powerlaw2m_n128_fwdbwd") != bench.kernel_source_digest(wl)


def test_committed_readings_parse():
    """The committed counter files carry a byte count and a digest (fresh or not)."""
    for wl in ("rmat22_rowblock0_4x4_n128", "powerlaw2m_n128_fwdbwd"):
        path = os.path.join(ROOT, "profiles", "traffic_%s.md" % wl)
        if not os.path.exists(path):
            pytest.skip("no stored reading for %s" % wl)
        text = open(path).read()
        assert "- hbm_bytes_per_step:" in text and "- source_sha256:" in text


def test_gather_ceiling_interpolation(monkeypatch):
    """The ceiling time sums each part's bytes at the probe rate for its row width and table
    size, interpolated in log2 of the size between the probed sizes (rates given here, so no GPU)."""
    rates = {(512, m): 1e12 * (2.0 if m <= 4 else 1.0) for m in bench.PROBE_MIB}
    rates.update({(128, m): 5e11 for m in bench.PROBE_MIB})
    monkeypatch.setattr(bench, "_PROBE", dict(rates))
    mib = 1 << 20
    # exactly on a probed size: 2e12 bytes at 2 TB/s = 1 s
    r = bench.gather_ceiling_report([(2e12, 4 * mib, 512)], kernel_ms=2000.0)
    assert r["ceiling_ms"] == pytest.approx(1000.0) and r["frac"] == pytest.approx(0.5)
    # halfway (in log2) between 4 and 16 MiB: 1.5 TB/s; below 1 MiB clamps to 1 MiB
    r = bench.gather_ceiling_report([(1.5e12, 8 * mib, 512), (1e12, 1024, 128)], kernel_ms=1000.0)
    assert r["ceiling_ms"] == pytest.approx(1000.0 + 2000.0)
    assert r["gathered_GB"] == pytest.approx(2500.0)
    # rows wider than 1 KiB use the 1 KiB probe
    assert bench._probe_width(4096) == 1024 and bench._probe_width(256) == 256


def test_library_bwd_rule_mirror():
    """The bench's reading of the backward's library rule (which form runs without an entry):
    fused while 64-lane windows of the widest vector dividing N stay at least 256 columns wide
    (or one group covers N), else the two-pass form."""
    for dtype in ("f32", "bf16"):
        for N in (1, 3, 64, 100, 128, 256, 260, 300, 512, 600, 1024):
            assert bench._library_bwd_fused(N, dtype), (N, dtype)
        assert not bench._library_bwd_fused(258, dtype)          # two-element vectors: 128-column windows
    assert not bench._library_bwd_fused(1026, "f32")             # 1026 = 2 x 513: 128-column windows
    assert bench._library_bwd_fused(2048, "f32") and not bench._library_bwd_fused(2304, "f32")   # at most 8
    assert bench._library_bwd_fused(4096, "bf16") and not bench._library_bwd_fused(4608, "bf16")  # windows


def test_library_fwd_rule_mirror():
    """bench.py labels a workload without a pinned variant by the library's forward rule; the mirror
    follows the rule's cases (many empty rows: more than 1/8)."""
    rows, few, many = 1000, 125, 126
    # FP32: 64-column windows, 128-column ones for N >= 256 and, on sparse tiles, for N % 128 == 0
    assert bench._library_fwd(64, "f32", rows, few) == ("rowsplit", 1)
    assert bench._library_fwd(64, "f32", rows, many) == ("stream", 1)
    assert bench._library_fwd(128, "f32", rows, few) == ("rowsplit", 1)
    assert bench._library_fwd(128, "f32", rows, many) == ("stream", 2)
    assert bench._library_fwd(192, "f32", rows, many) == ("stream", 1)
    assert bench._library_fwd(512, "f32", rows, few) == ("rowsplit", 2)
    assert bench._library_fwd(512, "f32", rows, many) == ("stream", 2)
    assert bench._library_fwd(513, "f32", rows, few) == ("rowsplit", 1)   # odd N: one-element vectors
    # BF16: row-split over the fewest windows of at most 256 columns, narrowest vector for that count
    assert bench._library_fwd(64, "bf16", rows, many) == ("stream", 1)
    assert bench._library_fwd(64, "bf16", rows, few) == ("rowsplit", 1)
    for empty in (few, many):
        assert bench._library_fwd(128, "bf16", rows, empty) == ("rowsplit", 2)
        assert bench._library_fwd(192, "bf16", rows, empty) == ("rowsplit", 4)
        assert bench._library_fwd(256, "bf16", rows, empty) == ("rowsplit", 4)
        assert bench._library_fwd(320, "bf16", rows, empty) == ("rowsplit", 4)
        assert bench._library_fwd(1024, "bf16", rows, empty) == ("rowsplit", 4)
    # below 64: row-split covering N with the widest vector
    assert bench._library_fwd(32, "f32", rows, many) == ("rowsplit", 4)
    assert bench._library_fwd(6, "bf16", rows, many) == ("rowsplit", 2)


def test_fwdbwd_gather_items():
    """A forward + backward step gathers a row of e * N bytes per non-zero in the forward and in
    the backward (twice in the two-pass form) and one value per non-zero at random."""
    class A:
        nnz, rows, cols = 1000, 300, 200
    f = bench._fwdbwd_gather_items(A, 128, 2, True)
    assert f == [(1000 * 256.0, 200 * 256, 256), (1000 * 256.0, 300 * 256, 256), (1000 * 16.0, 4000, 16)]
    t = bench._fwdbwd_gather_items(A, 64, 4, False)
    assert len(t) == 4 and t[3] == (1000 * 256.0, 200 * 256, 256)
