"""Error statistics and acceptance bounds for comparing a computed result with the FP64 oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Bounds used (none of them is from the paper, which fixes only FP32 values):
  * FP32 results, any summation order, with or without fused multiply-add:
    |C_hat - C| <= gamma_n * S  with  gamma_n = n u / (1 - n u),  u = 2^-24,
    S = sum |a||b| and n the number of terms (Higham, Accuracy and Stability of
    Numerical Algorithms, 2nd ed., Section 3.1).  The acceptance gate is the much
    tighter  |C_hat - C| <= tol * S  with tol = 1e-5; where S == 0 the result
    must equal the oracle exactly.
  * BF16 storage (B rounded to BF16 before the product, C rounded once at the
    store): against the oracle evaluated on the rounded B,
    |C_hat - C| <= 2^-8 |C| + tol * S * (1 + 2^-8), 2^-8 being the unit roundoff
    of an 8-bit significand under round-to-nearest.
"""
from __future__ import annotations

from typing import Dict, Optional

import numpy as np

U32 = 2.0 ** -24
U_BF16 = 2.0 ** -8
FP32_TOL = 1e-5


def gamma(n, u: float = U32):
    n = np.asarray(n, dtype=np.float64)
    return n * u / (1.0 - n * u)


def fp32_stats(got: np.ndarray, ref: np.ndarray, S: np.ndarray, tol: float = FP32_TOL,
               n_terms: Optional[np.ndarray] = None) -> Dict[str, float]:
    """Per-entry |got - ref| / S statistics; entries with S == 0 must match exactly."""
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    pos = S > 0
    rel = np.zeros_like(err)
    rel[pos] = err[pos] / S[pos]
    zero_bad = ~pos & (err != 0)
    # A NaN compares false with every bound, so non-finite results are counted on their own.
    nonfinite = ~np.isfinite(got)
    out = {
        "max_rel_to_scale": float(rel.max()) if rel.size else 0.0,
        "mean_rel_to_scale": float(rel.mean()) if rel.size else 0.0,
        "n_over_tol": int(np.count_nonzero((rel > tol) | zero_bad | nonfinite)),
        "zero_scale_mismatch": int(np.count_nonzero(zero_bad)),
        "nonfinite": int(np.count_nonzero(nonfinite)),
        "normwise": float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)),
        "entries": int(err.size),
    }
    if n_terms is not None:
        bound = gamma(n_terms) * S
        out["n_over_gamma_bound"] = int(np.count_nonzero((err > bound) | nonfinite))
    return out


def fp32_ok(stats: Dict[str, float]) -> bool:
    return stats["n_over_tol"] == 0 and stats.get("n_over_gamma_bound", 0) == 0


def bf16_stats(got: np.ndarray, ref: np.ndarray, S: np.ndarray, tol: float = FP32_TOL) -> Dict[str, float]:
    """``got`` is the BF16 result widened to FP32; ``ref``/``S`` are the oracle on the rounded B."""
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bound = U_BF16 * np.abs(ref) + tol * S * (1.0 + U_BF16)
    denom = np.maximum(np.abs(ref), 2.0 ** -20 * S)
    rel = np.zeros_like(err)
    pos = denom > 0
    rel[pos] = err[pos] / denom[pos]
    zero_bad = ~pos & (err != 0)
    # A NaN compares false with every bound, so non-finite results are counted on their own.
    nonfinite = ~np.isfinite(got)
    return {
        "max_rel": float(rel.max()) if rel.size else 0.0,
        "mean_rel": float(rel.mean()) if rel.size else 0.0,
        "n_over_bound": int(np.count_nonzero((err > bound) | zero_bad | nonfinite)),
        "zero_scale_mismatch": int(np.count_nonzero(zero_bad)),
        "nonfinite": int(np.count_nonzero(nonfinite)),
        "normwise": float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)),
        "entries": int(err.size),
    }


def relative_stats(got: np.ndarray, ref: np.ndarray, S: np.ndarray) -> Dict[str, float]:
    """max / mean of |got - ref| / max(|ref|, 2^-20 S): the relative error reported per result."""
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    denom = np.maximum(np.abs(ref), 2.0 ** -20 * S)
    pos = denom > 0
    rel = np.zeros_like(err)
    rel[pos] = err[pos] / denom[pos]
    return {"max_rel": float(rel.max()) if rel.size else 0.0,
            "mean_rel": float(rel.mean()) if rel.size else 0.0,
            "nonfinite": int(np.count_nonzero(~np.isfinite(got))),
            "normwise": float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))}
