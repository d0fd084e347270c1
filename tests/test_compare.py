"""Pins of the acceptance logic every parity verdict goes through (oracle/compare.py and
oracle.bf16_to_f32), on the CPU.

Each pin takes the module under test as an argument, so that test_oracle_mutations.py
can run the same pins against copies of compare.py with one planted mistake.  The
expected values come from what the mathematics fixes, not from the module:
  * gamma_n = n u / (1 - n u) with u = 2^-24 equals n / (2^24 - n) exactly, which is
    evaluated here in rational arithmetic (Higham, Accuracy and Stability of Numerical
    Algorithms, 2nd ed., Lemma 3.1);
  * a sequential FP32 sum of n terms stays within gamma_{n-1} * sum|x| of the exact sum,
    and adversarial sums come close to n u * sum|x| (checked on real FP32 sums);
  * errors planted at a fraction of each bound just inside or just outside it, NaN and
    infinite outputs, and the rule that an entry with zero scale must match exactly;
  * the BF16 widening is a 16-bit shift, checked over all 2^16 patterns against torch.
"""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
from oracle import compare as COMPARE

U32 = Fraction(1, 2 ** 24)


# --- gamma ---------------------------------------------------------------------------

def pin_gamma_closed_form(C):
    for n in [0, 1, 2, 3, 100, 4096, 97_538, 2 ** 20, 2 ** 23, 2 ** 24 - 2]:
        exact = Fraction(n, 2 ** 24 - n)  # n u / (1 - n u) with u = 2^-24
        got = Fraction(float(C.gamma(n)))
        assert abs(got - exact) <= exact * Fraction(1, 2 ** 50), (n, float(got), float(exact))
    # vectorised over an array of term counts
    ns = np.array([1, 10, 1000])
    g = C.gamma(ns)
    assert g.shape == ns.shape
    for n, x in zip(ns, g):
        exact = Fraction(int(n), 2 ** 24 - int(n))
        assert abs(Fraction(float(x)) - exact) <= exact * Fraction(1, 2 ** 50)


def pin_gamma_bounds_real_sums(C):
    """Sequential FP32 sums (numpy float32 adds, round to nearest) stay within gamma_{n-1} S."""
    rng = np.random.Generator(np.random.PCG64(11))
    for n in [2, 17, 256, 4096]:
        for _ in range(20):
            x = rng.uniform(-1, 1, n).astype(np.float32)
            s = np.float32(0)
            for v in x:
                s = np.float32(s + v)
            exact = float(sum(Fraction(float(v)) for v in x))
            S = float(np.abs(x.astype(np.float64)).sum())
            assert abs(float(s) - exact) <= float(C.gamma(n - 1)) * S
    # An adversarial sum: 1 followed by n-1 copies of u/2*(1+2^-20) rounds up at every step,
    # so its error is close to (n-1) u/2 * ... -- it must still sit under gamma_{n-1} S,
    # and the bound must not be loose by more than a factor ~2 there.
    n = 1000
    tiny = np.float32(2.0 ** -24 * (1 + 2.0 ** -20))
    s = np.float32(1.0)
    for _ in range(n - 1):
        s = np.float32(s + tiny)
    exact = 1.0 + (n - 1) * float(tiny)
    S = exact
    err = abs(float(s) - exact)
    assert err <= float(C.gamma(n - 1)) * S
    assert err >= 0.4 * float(C.gamma(n - 1)) * S


# --- fp32_stats / fp32_ok ---------------------------------------------------------

def _ref_case(n=64, seed=3):
    rng = np.random.Generator(np.random.PCG64(seed))
    ref = rng.uniform(-1, 1, n)
    S = np.abs(ref) + rng.uniform(0.5, 2.0, n)
    return ref, S


def pin_fp32_planted_tolerance(C):
    ref, S = _ref_case()
    tol = 1e-5
    for frac, ok in [(0.0, True), (0.5, True), (0.99, True), (1.01, False), (3.0, False)]:
        got = ref.copy()
        got[7] += frac * tol * S[7]
        st = C.fp32_stats(got, ref, S)
        assert (st["n_over_tol"] == 0) == ok, (frac, st)
        assert C.fp32_ok(st) == ok, (frac, st)
        assert abs(st["max_rel_to_scale"] - frac * tol) <= 1e-12
    # the error's sign does not matter
    got = ref.copy()
    got[9] -= 1.01 * tol * S[9]
    assert not C.fp32_ok(C.fp32_stats(got, ref, S))
    # mean over entries
    got = ref.copy()
    got[0] += 0.5 * tol * S[0]
    assert abs(C.fp32_stats(got, ref, S)["mean_rel_to_scale"] - 0.5 * tol / ref.size) <= 1e-15


def pin_fp32_gamma_bound(C):
    """With one term gamma_1 S (6e-8 S) is far tighter than 1e-5 S; with 10^4 terms, looser."""
    ref, S = _ref_case()
    n1 = np.ones_like(ref)
    g1 = float(C.gamma(1))
    got = ref.copy()
    got[4] += 0.9 * g1 * S[4]
    assert C.fp32_ok(C.fp32_stats(got, ref, S, n_terms=n1))
    got[4] = ref[4] + 2.0 * g1 * S[4]
    st = C.fp32_stats(got, ref, S, n_terms=n1)
    assert st["n_over_tol"] == 0 and st["n_over_gamma_bound"] == 1
    assert not C.fp32_ok(st)
    big = np.full_like(ref, 10_000.0)  # gamma ~ 6e-4 > tol
    got = ref.copy()
    got[4] += 2e-5 * S[4]
    st = C.fp32_stats(got, ref, S, n_terms=big)
    assert st["n_over_gamma_bound"] == 0 and st["n_over_tol"] == 1 and not C.fp32_ok(st)


def pin_fp32_nonfinite(C):
    ref, S = _ref_case()
    for bad in [np.nan, np.inf, -np.inf]:
        got = ref.copy()
        got[11] = bad
        st = C.fp32_stats(got, ref, S)
        assert st["nonfinite"] == 1 and st["n_over_tol"] == 1 and not C.fp32_ok(st), (bad, st)
        st = C.fp32_stats(got, ref, S, n_terms=np.ones_like(ref))
        assert not C.fp32_ok(st)


def pin_fp32_zero_scale_exact(C):
    ref, S = _ref_case()
    ref[3] = 0.0
    S[3] = 0.0  # an empty row: the result must be exactly the oracle's
    got = ref.copy()
    assert C.fp32_ok(C.fp32_stats(got, ref, S))
    got[3] = 1e-30
    st = C.fp32_stats(got, ref, S)
    assert st["zero_scale_mismatch"] == 1 and not C.fp32_ok(st)
    got[3] = -0.0  # equal to zero
    assert C.fp32_ok(C.fp32_stats(got, ref, S))
    # accumulate into an initial value with zero scale: exact equality with the initial value
    ref[5] = 0.25
    S[5] = 0.0
    got = ref.copy()
    assert C.fp32_ok(C.fp32_stats(got, ref, S))
    got[5] = np.nextafter(0.25, 1.0)
    assert not C.fp32_ok(C.fp32_stats(got, ref, S))


# --- bf16_stats ---------------------------------------------------------------------

def pin_bf16_planted_bound(C):
    ref, S = _ref_case(seed=5)
    tol = 1e-5
    i = 13
    bound = 2.0 ** -8 * abs(ref[i]) + tol * S[i] * (1 + 2.0 ** -8)
    for frac, ok in [(0.0, True), (0.5, True), (0.999, True), (1.001, False), (2.0, False)]:
        got = ref.copy()
        got[i] += frac * bound
        st = C.bf16_stats(got, ref, S)
        assert (st["n_over_bound"] == 0) == ok, (frac, st)
    # the bound's relative part alone (S tiny): 2^-8 |ref|
    ref2 = np.array([1.0, -3.0, 0.5])
    S2 = np.array([1e-12, 1e-12, 1e-12])
    got = ref2 * (1 + 0.99 * 2.0 ** -8)
    assert C.bf16_stats(got, ref2, S2)["n_over_bound"] == 0
    got = ref2 * (1 + 1.01 * 2.0 ** -8)
    assert C.bf16_stats(got, ref2, S2)["n_over_bound"] == 3


def pin_bf16_nonfinite(C):
    ref, S = _ref_case(seed=6)
    for bad in [np.nan, np.inf, -np.inf]:
        got = ref.copy()
        got[2] = bad
        st = C.bf16_stats(got, ref, S)
        assert st["n_over_bound"] == 1 and st["nonfinite"] == 1, (bad, st)
    got = ref.copy()
    got[[1, 2, 3]] = [np.nan, np.nan, np.inf]
    assert C.bf16_stats(got, ref, S)["n_over_bound"] == 3


def pin_bf16_zero_scale_exact(C):
    ref = np.array([0.0, 1.0, 0.0])
    S = np.array([0.0, 1.0, 0.0])
    assert C.bf16_stats(ref.copy(), ref, S)["n_over_bound"] == 0
    got = ref.copy()
    got[2] = 2.0 ** -40
    st = C.bf16_stats(got, ref, S)
    assert st["n_over_bound"] == 1 and st["zero_scale_mismatch"] == 1


def pin_bf16_relative_values(C):
    ref = np.array([1.0, 2.0, -4.0, 0.5])
    S = np.array([1.0, 2.0, 4.0, 0.5])
    got = ref.copy()
    got[1] = 2.0 * (1 + 2.0 ** -9)
    st = C.bf16_stats(got, ref, S)
    assert st["max_rel"] == 2.0 ** -9 and st["mean_rel"] == 2.0 ** -9 / 4
    # where |ref| << S, the denominator is 2^-20 S
    ref = np.array([0.0])
    S = np.array([1.0])
    got = np.array([2.0 ** -30])
    assert C.bf16_stats(got, ref, S)["max_rel"] == 2.0 ** -10


# --- relative_stats -----------------------------------------------------------------

def pin_relative_stats(C):
    ref = np.array([1.0, -2.0, 8.0, 0.0])
    S = np.array([1.0, 2.0, 8.0, 0.0])
    got = np.array([1.0 + 2.0 ** -10, -2.0, 8.0 - 2.0 ** -6, 0.0])
    st = C.relative_stats(got, ref, S)
    assert st["max_rel"] == 2.0 ** -9
    assert st["mean_rel"] == (2.0 ** -10 + 2.0 ** -9) / 4
    assert st["nonfinite"] == 0
    expect_norm = np.sqrt(2.0 ** -20 + 2.0 ** -12) / np.sqrt(1 + 4 + 64)
    assert abs(st["normwise"] - expect_norm) <= 1e-15
    got[0] = np.nan
    assert C.relative_stats(got, ref, S)["nonfinite"] == 1
    # the 2^-20 S floor of the denominator
    st = C.relative_stats(np.array([2.0 ** -21]), np.array([0.0]), np.array([1.0]))
    assert st["max_rel"] == 0.5


COMPARE_PINS = [pin_gamma_closed_form, pin_gamma_bounds_real_sums, pin_fp32_planted_tolerance,
                pin_fp32_gamma_bound, pin_fp32_nonfinite, pin_fp32_zero_scale_exact, pin_bf16_planted_bound,
                pin_bf16_nonfinite, pin_bf16_zero_scale_exact, pin_bf16_relative_values, pin_relative_stats]


@pytest.mark.parametrize("pin", COMPARE_PINS, ids=lambda f: f.__name__)
def test_compare_pin(pin):
    pin(COMPARE)


# --- bf16_to_f32 ------------------------------------------------------------------

def pin_bf16_widening_all_patterns(O):
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    got = O.bf16_to_f32(bits)
    assert got.dtype == np.float32 and got.shape == bits.shape
    ref = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).float().numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    # a few values by hand: 0x3F80 = 1.0, 0xC000 = -2.0, 0x0001 = smallest subnormal 2^-133
    assert O.bf16_to_f32(np.array([0x3F80, 0xC000, 0x0001], dtype=np.uint16)).tolist() == [1.0, -2.0, 2.0 ** -133]


def test_bf16_widening_all_patterns():
    pin_bf16_widening_all_patterns(oracle)
