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
