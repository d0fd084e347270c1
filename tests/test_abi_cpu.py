"""libspmm loads on a machine without a GPU, exports every entry point its header
declares, and rejects bad arguments before touching the HIP runtime."""
import ctypes
import os
import re

import pytest

from paper_2311_18141_amd import _lib
from paper_2311_18141_amd._lib import SpmmCsr, SpmmTileOpts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spmm.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:spmm|spgemm)_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = declared_functions()
    assert "spmm_fwd" in names and "spmm_bwd" in names and "spmm_tile_create" in names
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares every one of them
    assert set(names) <= set(_lib.EXPORTS), set(names) - set(_lib.EXPORTS)


def test_library_exports_only_declared_c_symbols():
    """No C-linkage symbol leaks beyond the header's declarations (C++ symbols are mangled)."""
    import shutil
    import subprocess
    if shutil.which("nm") is None:
        pytest.skip("nm not available")
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], check=True, capture_output=True,
                         text=True).stdout
    names = {line.split()[-1] for line in out.splitlines() if line.strip()}
    c_names = {n for n in names if not n.startswith("_Z") and not n.startswith("__") and not n.startswith("_")}
    c_names -= {"_init", "_fini"}
    assert c_names == set(declared_functions()), c_names ^ set(declared_functions())


def test_status_strings():
    L = _lib.lib()
    for code, name in _lib.STATUS_NAMES.items():
        assert L.spmm_status_string(code).decode() == name
    assert L.spmm_status_string(99).decode() == "unknown spmm_status"


def _create(rows, num_k, tiles, opts=None):
    L = _lib.lib()
    h = ctypes.c_void_p(1234)
    st = L.spmm_tile_create(rows, num_k, tiles, ctypes.byref(opts) if opts is not None else None, None,
                            ctypes.byref(h))
    return st, h.value, L.spmm_last_error().decode()


def _tiles(n=1, cols=10, nnz=5, ptr=0x1000):
    arr = (SpmmCsr * n)()
    for k in range(n):
        arr[k].cols, arr[k].nnz = cols, nnz
        arr[k].rowptr, arr[k].colind, arr[k].values = ptr, ptr, ptr
    return arr


@pytest.mark.parametrize("case,expect", [
    ("null_out", 1), ("neg_rows", 1), ("huge_rows", 1), ("k0", 1), ("k17", 1), ("null_tiles", 1),
    ("neg_cols", 1), ("neg_nnz", 1), ("big_nnz", 3), ("cap_nnz", 3), ("null_rowptr", 1), ("null_colind", 1),
    ("bad_flags", 1), ("transpose_k2", 3), ("neg_long_row", 1), ("huge_long_row", 1), ("hot_rows_m2", 1),
    ("hot_rows_huge", 1),
])
def test_create_argument_errors(case, expect):
    L = _lib.lib()
    t = _tiles()
    opts = SpmmTileOpts()
    rows, K = 4, 1
    if case == "null_out":
        assert L.spmm_tile_create(4, 1, t, None, None, None) == expect
        return
    if case == "neg_rows":
        rows = -1
    elif case == "huge_rows":
        rows = 1 << 31
    elif case == "k0":
        K = 0
    elif case == "k17":
        K = 17
        t = _tiles(17)
    elif case == "null_tiles":
        t = None
    elif case == "neg_cols":
        t[0].cols = -1
    elif case == "neg_nnz":
        t[0].nnz = -5
    elif case == "big_nnz":
        t[0].nnz = 1 << 31
    elif case == "cap_nnz":  # one past the largest count whose int32 positions keep stride headroom
        t[0].nnz = (1 << 31) - (1 << 16) + 1
    elif case == "null_rowptr":
        t[0].rowptr = None
    elif case == "null_colind":
        t[0].colind = None
    elif case == "bad_flags":
        opts.flags = 0x80
    elif case == "transpose_k2":
        t = _tiles(2)
        K = 2
        opts.flags = _lib.SPMM_TILE_TRANSPOSE
    elif case == "neg_long_row":
        opts.long_row = -3
    elif case == "huge_long_row":  # 64 unsplit rows of this length would overflow a 32-bit prefix sum
        opts.long_row = (1 << 31) // 64
    elif case == "hot_rows_m2":
        opts.hot_rows = -2
    elif case == "hot_rows_huge":
        opts.hot_rows = (1 << 24) + 1
    st, h, msg = _create(rows, K, t, opts)
    assert st == expect, (case, st, msg)
    assert h is None
    assert msg


def test_null_handle_calls():
    L = _lib.lib()
    n = ctypes.c_size_t()
    assert L.spmm_tile_destroy(None) == 1
    assert L.spmm_tile_get_stats(None, None) == 1
    assert L.spmm_fwd_workspace_bytes(None, 8, ctypes.byref(n)) == 1
    assert L.spmm_bwd_workspace_bytes(None, 8, ctypes.byref(n)) == 1
    assert L.spmm_fwd(None, 0, None, None, 0, None, 8, 0, 8, 0, None, 0, None) == 1
    assert L.spmm_bwd(None, None, 8, None, 8, 8, 0, None, None, 8, None, 0, None) == 1
    assert L.spmm_tile_export_transpose(None, None, None, None, None) == 1


def test_batch_and_variant_argument_errors():
    L = _lib.lib()
    n = ctypes.c_size_t()
    out = ctypes.c_void_p(7)
    ns = (ctypes.c_int64 * 1)(32)
    assert L.spmm_batch_create(1, None, ns, 0, 0, 0, None, ctypes.byref(out)) == 1
    assert L.spmm_batch_create(0, None, ns, 0, 0, 0, None, ctypes.byref(out)) == 1
    tiles = (ctypes.c_void_p * 1)(None)
    assert L.spmm_batch_create(1, tiles, ns, 0, 0, 0, None, ctypes.byref(out)) == 1
    assert L.spmm_batch_create(1, tiles, ns, 0, 0, 2, None, ctypes.byref(out)) == 1
    assert L.spmm_batch_create(1, tiles, ns, 0, 32, 0, None, ctypes.byref(out)) == 1
    assert L.spmm_batch_create(1, tiles, ns, 0, 0, 0, None, None) == 1
    assert L.spmm_batch_destroy(None) == 1
    assert L.spmm_batch_workspace_bytes(None, ctypes.byref(n)) == 1
    assert L.spmm_batch_get_variant(None, 0, None) == 1
    assert L.spmm_batched(None, None, None, None, None, 0, None, 0, None) == 1
    v = _lib.SpmmVariant(1, 8, 4)
    assert L.spmm_tile_set_variant(None, 32, 0, ctypes.byref(v)) == 1
    assert L.spmm_tile_autotune(None, 32, 0, None, None, None, 32, 0, None, None) == 1
    assert L.spmm_tile_set_sddmm_variant(None, 32, 8, 4) == 1


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of the header's structs have the C sizes and field offsets."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"spmm_csr": _lib.SpmmCsr, "spmm_tile_opts": _lib.SpmmTileOpts,
               "spmm_tile_stats": _lib.SpmmTileStats, "spmm_variant": _lib.SpmmVariant}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "spmm.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for field, _ in cls._fields_:
            assert got[(name, field)] == getattr(cls, field).offset, (name, field)


def test_spgemm_argument_errors():
    L = _lib.lib()
    out = ctypes.c_void_p(7)
    a = SpmmCsr(4, 0, None, None, None)
    assert L.spgemm_create(4, None, None, 0, None, ctypes.byref(out)) == 1
    assert L.spgemm_create(4, ctypes.byref(a), ctypes.byref(a), 0, None, None) == 1
    assert L.spgemm_create(-1, ctypes.byref(a), ctypes.byref(a), 0, None, ctypes.byref(out)) == 1
    assert L.spgemm_create(4, ctypes.byref(a), ctypes.byref(a), 0, None, ctypes.byref(out)) == 1  # rowptr null
    big = SpmmCsr(4, 1 << 31, 8, 8, 8)
    assert L.spgemm_create(4, ctypes.byref(big), ctypes.byref(a), 0, None, ctypes.byref(out)) == 3
    cap = SpmmCsr(4, (1 << 31) - (1 << 16) + 1, 8, 8, 8)
    assert L.spgemm_create(4, ctypes.byref(a), ctypes.byref(cap), 0, None, ctypes.byref(out)) == 3
    assert L.spgemm_destroy(None) == 1
    assert L.spgemm_info(None, None, None) == 1
    assert L.spgemm_rowptr(None, None, None) == 1
    assert L.spgemm_compute(None, None, None, None) == 1


@pytest.mark.parametrize("case", ["null_out", "no_rows", "null_table", "row_bytes_0", "row_bytes_24", "row_bytes_1040",
                                  "row_bytes_8192", "neg_n", "null_idx", "misaligned"])
def test_gather_probe_argument_errors(case):
    """The gather micro-benchmark checks its arguments before any HIP call."""
    L = _lib.lib()
    args = dict(table=0x1000, rows=8, row_bytes=64, idx=0x2000, n=5, out=0x3000)
    if case == "null_out":
        args["out"] = None
    elif case == "no_rows":
        args["rows"] = 0
    elif case == "null_table":
        args["table"] = None
    elif case.startswith("row_bytes_"):
        args["row_bytes"] = int(case.split("_")[-1])
    elif case == "neg_n":
        args["n"] = -1
    elif case == "null_idx":
        args["idx"] = None
    elif case == "misaligned":
        args["table"] = 0x1008
    st = L.spmm_gather_probe(args["table"], args["rows"], args["row_bytes"], args["idx"], args["n"], args["out"], None)
    assert st == 1, (case, st, L.spmm_last_error())


def test_bwd_variant_argument_errors():
    """The dB-pass variant setter and autotuner check their arguments before any HIP call."""
    L = _lib.lib()
    v = _lib.SpmmVariant(_lib.SPMM_KERNEL_ROWSPLIT, 16, 4)
    assert L.spmm_tile_set_bwd_variant(None, 64, 0, ctypes.byref(v)) == 1
    assert L.spmm_tile_get_variant(None, 64, 0, 0, ctypes.byref(v)) == 1
    assert L.spmm_tile_get_variant(None, 64, 0, 1, None) == 1
    assert L.spmm_tile_autotune_bwd(None, 64, 0, 0x1000, 64, None, 0, None, 0x2000, 64, None, None) == 1


def test_trace_ranges_switch_on_without_changing_results():
    """With SPMM_TRACE=1 the entry points open roctx ranges (the marker library is loaded on
    the first one); argument checks still return their status.  Run in a child process so
    that the switch, read once per process, starts fresh."""
    import subprocess
    import sys
    code = ("import ctypes\n"
            "from paper_2311_18141_amd import _lib\n"
            "L = _lib.lib()\n"
            "assert L.spmm_fwd(None, 0, None, None, 0, None, 8, 0, 8, 0, None, 0, None) == 1\n"
            "assert L.spmm_batched(None, None, None, None, None, 0, None, 0, None) == 1\n"
            "assert L.spgemm_compute(None, None, None, None) == 1\n"
            "print('ok')\n")
    for flag in ("1", "0"):
        env = dict(os.environ, SPMM_TRACE=flag)
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=120)
        assert r.returncode == 0 and r.stdout.strip() == "ok", (flag, r.stdout, r.stderr[-2000:])


def test_noalloc_forward_argument_errors():
    """The forward that allocates nothing checks its arguments before any HIP call; its scratch
    size is fixed."""
    L = _lib.lib()
    assert L.spmm_noalloc_scratch_bytes() == 64 << 20
    assert L.spmm_fwd_noalloc(None, 0, None, None, 0, None, 8, 0, 8, 0, None) == 1
    assert L.spmm_last_error()


def test_reservation_grid_and_accumulate_n_argument_errors():
    """The reservation-grid batch and the multi-partial accumulate check their arguments before any
    HIP call."""
    L = _lib.lib()
    h = ctypes.c_void_p()
    coords = (ctypes.c_int32 * 3)(0, 0, 0)
    assert L.spmm_batch_create_grid(1, None, None, 0, coords, 1, 0, None, None) == 1          # null out
    assert L.spmm_batch_create_grid(1, None, None, 0, coords, 9, 0, None, ctypes.byref(h)) == 1  # bad mode
    assert L.spmm_batch_create_grid(1, None, None, 0, None, 1, 0, None, ctypes.byref(h)) == 1    # null coords
    bad = (ctypes.c_int32 * 3)(0, -1, 0)
    assert L.spmm_batch_create_grid(1, None, None, 0, bad, 1, 0, None, ctypes.byref(h)) == 1     # negative coord
    assert L.spmm_batch_create_grid(1, None, None, 0, coords, 1, 0, None, ctypes.byref(h)) == 1  # null tiles
    assert L.spmm_batch_create_grid(1, None, None, 0, coords, 1, 7, None, ctypes.byref(h)) == 1  # item_nnz
    assert h.value is None
    ptrs = (ctypes.c_void_p * 1)(0x1000)
    lds = (ctypes.c_int64 * 1)(8)
    assert L.spmm_tile_accumulate_n(0x2000, 8, ptrs, lds, 1, 4, 8, 7, None) == 1   # bad dtype
    assert L.spmm_tile_accumulate_n(0x2000, 8, None, None, 1, 4, 8, 0, None) == 1  # null partial arrays
    lds[0] = 4
    assert L.spmm_tile_accumulate_n(0x2000, 8, ptrs, lds, 1, 4, 8, 0, None) == 1   # ldp < N
    assert L.spmm_tile_accumulate_n(0x2000, 8, ptrs, lds, -1, 4, 8, 0, None) == 1  # negative count


def test_spgemm_pattern_entries_arguments():
    L = _lib.lib()
    x = ctypes.c_int64(7)
    assert L.spgemm_pattern_entries(None, ctypes.byref(x)) == 1 and x.value == 7
    assert L.spgemm_pattern_entries(None, None) == 1
    # an unknown flag bit beside SPGEMM_BITMAP_ONLY is refused before any device work
    out = ctypes.c_void_p()
    a = SpmmCsr(4, 0, 8, None, None)   # a non-null (never read) row pointer, no entries
    assert L.spgemm_create(4, ctypes.byref(a), ctypes.byref(a), 32, None, ctypes.byref(out)) == 1
    assert b"flag" in L.spmm_last_error()
