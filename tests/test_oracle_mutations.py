"""Plant plausible mistakes in a copy of the oracle (on the CPU) and check that the pins catch each one.

Each mutant is the oracle's C source with one edit (a dropped term, a wrong sign
or index, a transposed operand, an unstable order, a wrong tie rule).  The pins
of test_oracle.py run against the mutant build; at least one of them must fail.
"""
import json
import os

import pytest

import oracle
import test_oracle as T
import test_oracle_spgemm as TS

MUTANTS = {
    "drop_accumulate_term": ("c[n] = accumulate ? (double)C0[i * ldc0 + n] : 0.0;", "c[n] = 0.0;"),
    "wrong_sign": ("c[n] += a * (double)b[n];", "c[n] -= a * (double)b[n];"),
    "row_instead_of_column": ("B[k] + (int64_t)colind[k][p] * ldb[k]", "B[k] + (int64_t)i * ldb[k]"),
    "drop_last_nonzero": ("p < rowptr[k][i + 1]; ++p) {\n        double a", "p < rowptr[k][i + 1] - 1; ++p) {\n        double a"),
    "always_first_tile": ("int k = (int)(((int64_t)kk + k_offset) % num_k);", "int k = 0;"),
    "scale_without_abs": ("if (s) s[n] += fabs(a) * fabs((double)b[n]);", "if (s) s[n] += a * (double)b[n];"),
    "sddmm_wrong_operand": ("const float* b = B + (int64_t)colind[p] * ldb;", "const float* b = B + (int64_t)i * ldb;"),
    "row_search_off_by_one": ("if ((int64_t)rowptr[mid] <= p) lo = mid;", "if ((int64_t)rowptr[mid] < p) lo = mid;"),
    "spmm_t_drop_value": ("dB[r * ldo + n] += a * (double)g[n];", "dB[r * ldo + n] += (double)g[n];"),
    "transpose_unstable": ("  for (int64_t i = 0; i < M; ++i)\n    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {\n      int64_t q",
                           "  for (int64_t i = M - 1; i >= 0; --i)\n    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {\n      int64_t q"),
    "bf16_ties_away": ("(lower == 0x8000u && (upper & 1u))", "(lower == 0x8000u)"),
    "bf16_truncate": ("upper += 1u;", "upper += 0u;"),
    "bf16_nan_passthrough": ("      y[t] = 0x7FC0u;\n      continue;", "      y[t] = (uint16_t)(bits >> 16);\n      continue;"),
    "spgemm_first_b_row_only": ("          int64_t k = colA[p];\n          double a", "          int64_t k = colA[rowptrA[i]];\n          double a"),
    "spgemm_count_all_products": ("            if (mark[j] != r) {\n              mark[j] = r;\n              ++cnt;",
                                  "            if (1) {\n              mark[j] = r;\n              ++cnt;"),
    "spgemm_unsorted_row": ("        qsort(cols, (size_t)cnt, sizeof(int64_t), cmp_i64);\n", ""),
    "spgemm_drop_b_value": ("            acc[j] += a * (double)valB[q];", "            acc[j] += a;"),
    "spgemm_skip_last_b": ("          for (int64_t q = rowptrB[k]; q < rowptrB[k + 1]; ++q) {\n            int64_t j = colB[q];\n            if (mark[j] != r) {\n              mark[j] = r;\n              acc",
                           "          for (int64_t q = rowptrB[k]; q < rowptrB[k + 1] - 1; ++q) {\n            int64_t j = colB[q];\n            if (mark[j] != r) {\n              mark[j] = r;\n              acc"),
}


def _pins():
    with open(os.path.join(T.GOLDEN, "spmm_worked_example.json")) as f:
        g = json.load(f)
    return [
        lambda: T.test_golden_forward(g),
        lambda: T.test_golden_k_tiles(g),
        lambda: T.test_golden_backward(g),
        lambda: T.test_golden_bf16(g),
        lambda: T.test_spmm_vs_dense(50, 40, 32, 4),
        lambda: T.test_spmm_brute_force_3x3(),
        lambda: T.test_spmm_accumulate(),
        lambda: T.test_identity_and_permutation_exact(),
        lambda: T.test_k_tile_decomposition(3),
        lambda: T.test_sddmm_vs_dense(),
        lambda: T.test_spmm_t_vs_dense_and_scipy(),
        lambda: T.test_transpose_vs_scipy(300, 200, 1),
        lambda: T.test_bf16_vs_torch_stratified(),
        lambda: TS.test_spgemm_vs_dense(40, 30, 50, 0.1),
        lambda: TS.test_spgemm_integer_exact(),
        lambda: TS.test_spgemm_exhaustive_2x2_patterns(),
        lambda: TS.test_spgemm_cancellation_keeps_entry(),
        lambda: TS.test_spgemm_identity_and_permutation(),
    ]


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    with open(oracle._SRC) as f:
        src = f.read()
    old, new = MUTANTS[name]
    assert src.count(old) == 1, "mutation site not found uniquely"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = oracle.build(force=True, src=str(path), out=str(tmp_path / "libmutant.so"))
    saved = oracle.lib()
    oracle._lib = oracle.load(so)
    caught = []
    try:
        for i, pin in enumerate(_pins()):
            try:
                pin()
            except (AssertionError, IndexError, ValueError):
                # a failed comparison, or output so malformed that the pin cannot index it
                caught.append(i)
    finally:
        oracle._lib = saved
    assert caught, "no pin caught mutant %s" % name


# Planted mistakes in the acceptance logic (oracle/compare.py, and the BF16 widening in
# oracle/__init__.py): a copy of the module with one edit is loaded under another name and
# the pins of test_compare.py run against it; at least one of them must fail.
import importlib.util  # noqa: E402

import test_compare as TC  # noqa: E402

_COMPARE_SRC = os.path.join(os.path.dirname(oracle._SRC), "compare.py")
_ORACLE_PY = os.path.join(os.path.dirname(oracle._SRC), "__init__.py")

COMPARE_MUTANTS = {
    "tol_x10": ('"n_over_tol": int(np.count_nonzero((rel > tol) |', '"n_over_tol": int(np.count_nonzero((rel > 10 * tol) |'),
    "fp32_drop_zero_scale": ("(rel > tol) | zero_bad | nonfinite", "(rel > tol) | nonfinite"),
    "fp32_nan_passthrough": ("(rel > tol) | zero_bad | nonfinite", "(rel > tol) | zero_bad"),
    "fp32_scale_is_abs_ref": ("rel[pos] = err[pos] / S[pos]", "rel[pos] = err[pos] / np.abs(ref[pos])"),
    "fp32_ok_ignores_gamma": ('return stats["n_over_tol"] == 0 and stats.get("n_over_gamma_bound", 0) == 0',
                              'return stats["n_over_tol"] == 0'),
    "bf16_nan_passthrough": ("(err > bound) | zero_bad | nonfinite", "(err > bound) | zero_bad"),
    # (dropping zero_bad from the BF16 count is an equivalent edit: where ref = 0 and S = 0 the
    # bound is exactly 0, so err > bound already fails the entry)
    "bf16_wrong_bound_factor": ("bound = U_BF16 * np.abs(ref)", "bound = 2 * U_BF16 * np.abs(ref)"),
    "bf16_bound_drops_scale_term": ("bound = U_BF16 * np.abs(ref) + tol * S * (1.0 + U_BF16)",
                                    "bound = U_BF16 * np.abs(ref)"),
    "gamma_no_denominator": ("return n * u / (1.0 - n * u)", "return n * u"),
    "unit_roundoff_wrong": ("U32 = 2.0 ** -24", "U32 = 2.0 ** -23"),
    "relative_floor_dropped": ('the relative error reported per result."""\n    got = np.asarray(got, dtype=np.float64)\n'
                               '    err = np.abs(got - ref)\n    denom = np.maximum(np.abs(ref), 2.0 ** -20 * S)',
                               'the relative error reported per result."""\n    got = np.asarray(got, dtype=np.float64)\n'
                               '    err = np.abs(got - ref)\n    denom = np.abs(ref)'),
    "relative_nan_hidden": ('"nonfinite": int(np.count_nonzero(~np.isfinite(got))),\n            "normwise"',
                            '"nonfinite": 0,\n            "normwise"'),
}

WIDEN_MUTANTS = {
    "widen_shift_15": ("astype(np.uint32) << 16).view(np.float32)", "astype(np.uint32) << 15).view(np.float32)"),
    "widen_drops_sign": ("(np.asarray(h, dtype=np.uint16).astype(np.uint32) << 16)",
                         "((np.asarray(h, dtype=np.uint16) & 0x7FFF).astype(np.uint32) << 16)"),
}


def _load_mutant(src_path, old, new, tmp_path, name):
    with open(src_path) as f:
        src = f.read()
    assert src.count(old) == 1, "mutation site not found uniquely"
    path = tmp_path / (name + ".py")
    path.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location("mutant_" + name, str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _caught(pins, mod):
    caught = []
    for i, pin in enumerate(pins):
        try:
            pin(mod)
        except (AssertionError, IndexError, ValueError, ZeroDivisionError):
            caught.append(i)
    return caught


@pytest.mark.parametrize("name", sorted(COMPARE_MUTANTS))
def test_compare_pins_catch_mutant(name, tmp_path):
    old, new = COMPARE_MUTANTS[name]
    mod = _load_mutant(_COMPARE_SRC, old, new, tmp_path, name)
    assert _caught(TC.COMPARE_PINS, mod), "no pin caught compare mutant %s" % name


@pytest.mark.parametrize("name", sorted(WIDEN_MUTANTS))
def test_widening_pin_catches_mutant(name, tmp_path):
    old, new = WIDEN_MUTANTS[name]
    mod = _load_mutant(_ORACLE_PY, old, new, tmp_path, name)
    assert _caught([TC.pin_bf16_widening_all_patterns], mod), "widening mutant %s not caught" % name


def test_unmutated_compare_passes_every_pin(tmp_path):
    """The harness itself: the unedited module loaded the same way passes every pin."""
    mod = _load_mutant(_COMPARE_SRC, "U32 = 2.0 ** -24", "U32 = 2.0 ** -24", tmp_path, "identity")
    assert _caught(TC.COMPARE_PINS, mod) == []
