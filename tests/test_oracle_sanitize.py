"""The CPU oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer: every exported
routine runs on small, exactly sized heap inputs (``oracle_sanitize.c``) with its edge cases,
and must neither read nor write out of bounds, leak, nor hit undefined behaviour.  A copy of
the oracle with a planted one-past-the-end read shows that the harness does catch one."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE_C = os.path.join(HERE, os.pardir, "oracle", "oracle.c")
DRIVER_C = os.path.join(HERE, "oracle_sanitize.c")
FLAGS = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fopenmp"]
ENV = dict(os.environ, OMP_NUM_THREADS="4",
           ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")


def _build(oracle_src, out):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    r = subprocess.run(["gcc", *FLAGS, DRIVER_C, oracle_src, "-lm", "-o", out],
                       capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        if "sanitize" in r.stderr or "asan" in r.stderr or "ubsan" in r.stderr:
            pytest.skip("gcc sanitizer runtime not available: " + r.stderr[-300:])
        raise AssertionError(r.stderr)
    return out


def _run(exe):
    return subprocess.run([exe], capture_output=True, text=True, timeout=120, env=ENV)


def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = _build(ORACLE_C, str(tmp_path / "drv"))
    r = _run(exe)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


def test_planted_overrun_is_caught(tmp_path):
    """The transposed product's loop over a row, widened by one entry: the last row then
    reads colind one past its block, which the sanitizer must report."""
    src = open(ORACLE_C).read()
    bug = src.replace("for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {\n      int64_t r = slot[colind[p]];",
                      "for (int64_t p = rowptr[i]; p <= rowptr[i + 1]; ++p) {\n      int64_t r = slot[colind[p]];")
    assert bug != src, "the planted change no longer applies to oracle.c"
    planted = tmp_path / "oracle_planted.c"
    planted.write_text(bug)
    exe = _build(str(planted), str(tmp_path / "drv_planted"))
    r = _run(exe)
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr and "heap-buffer-overflow" in r.stderr, r.stderr[-2000:]
