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
    assert "rmat22_rowblock0_4x4_n128" in names          # the default workload
    assert set(bench.PINNED) <= names
    for name, pin in bench.PINNED.items():
        kind, lanes, vec = pin["variant"]
        assert kind in ("stream", "rowsplit") and lanes in (4, 8, 16, 32, 64) and vec in (1, 2, 4, 8)
        assert pin["long_row"] > 0 and pin["segment"] > 0


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
