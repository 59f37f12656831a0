"""Simulated low-precision preconditioner (Section 3.1, Cholesky variant).

The paper computes the factor in a low precision u_q and, for Cholesky,
applies two-sided diagonal scaling H = D^{-1} fl(A^T A) D^{-1} with
D = diag(A^T A)^{1/2} first. This module reproduces the project's version
of that factor on the CPU:

1. d_j = ||A e_j||_2 in float64 (so D^2 = diag(A^T A));
2. A-hat = fl_q(A D^{-1}), each entry rounded to nearest-even in u_q
   (fp16 or bf16: ``round_to``);
3. H = A-hat^T A-hat with exact products and float32 sums;
4. R-hat = chol(H) in float32, stored rounded to u_q;
5. R = R-hat D, so that R^T R ~ A^T A.

Rounding to nearest-even is written from the IEEE 754 definition: keep p
significant bits (p = 11 for fp16, 8 for bf16), with the quantum floored
at the smallest subnormal and overflow to infinity.

Pins: tests/test_oracle_misc.py (rounding against numpy's float16
cast, which is IEEE RNE, against exhaustive bf16 neighbours, and the
backward-error size of the scaled factor; the split pair against its
defining bounds |x - hi - lo| <= 2^-8 |x - hi| <= 2^-16 |x|).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

FORMATS = {
    # name: (significand bits incl. implicit, min normal exponent, max finite)
    "fp16": (11, -14, 65504.0),
    "bf16": (8, -126, float(np.ldexp(255.0 / 128.0, 127))),
    "fp32": (24, -126, float(np.finfo(np.float32).max)),
}


def round_to(x, fmt: str) -> np.ndarray:
    """Round float64 values to the nearest ``fmt`` value (ties to even),
    returned as float64."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "fp64":
        return x.copy()
    p, emin, fmax = FORMATS[fmt]
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    m, e = np.frexp(x[nz])               # x = m * 2**e, 0.5 <= |m| < 1
    # quantum exponent: p significant bits, not below the subnormal quantum
    q = np.maximum(e - p, emin - (p - 1))
    r = np.ldexp(np.rint(np.ldexp(x[nz], -q)), q)   # np.rint: ties to even
    r[np.abs(r) > fmax] = np.copysign(np.inf, r[np.abs(r) > fmax])
    out[nz] = r
    keep = ~nz                      # zeros keep their sign; Inf and NaN pass through
    out[keep] = x[keep]
    return out


def split_bf16(x):
    """The split BF16 pair of each value: hi = bf16(x), lo = bf16(x - hi)
    (x - hi is exact in float64). hi + lo carries x to 2^-16 relative
    (two 8-bit significands), the representation of the project's split BF16
    Gram matrix (a project addition; the paper's u_q is a single format).
    Returns (hi, lo) as float64."""
    x = np.asarray(x, dtype=np.float64)
    hi = round_to(x, "bf16")
    return hi, round_to(x - hi, "bf16")


def split_gram(Ah_hi, Ah_lo):
    """hi^T hi + hi^T lo + lo^T hi in float64 (lo^T lo is dropped): the Gram
    matrix the split BF16 route forms, up to its FP32 accumulation."""
    return Ah_hi.T @ Ah_hi + Ah_hi.T @ Ah_lo + Ah_lo.T @ Ah_hi


def column_norms(A) -> np.ndarray:
    if hasattr(A, "val"):
        d2 = np.zeros(A.n)
        np.add.at(d2, A.col_idx, A.val * A.val)
        return np.sqrt(d2)
    A = np.asarray(A, dtype=np.float64)
    return np.sqrt(np.sum(A * A, axis=0))


def scaled_factor(A, fmt: str = "fp16", store: str | None = None):
    """Steps 1-5 above. Returns (R_hat as float64 holding ``store``-rounded
    values, d). ``store`` defaults to ``fmt``."""
    store = fmt if store is None else store
    d = column_norms(A)
    if hasattr(A, "val"):
        rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
        Ah = np.zeros((A.m, A.n), dtype=np.float32)
        Ah[rows, A.col_idx] = round_to(A.val / d[A.col_idx], fmt).astype(np.float32)
    else:
        Ah = round_to(np.asarray(A) / d, fmt).astype(np.float32)
    H = Ah.T @ Ah                                  # float32 accumulation
    Rh = sla.cholesky(H.astype(np.float32), lower=False)
    Rh = np.triu(Rh).astype(np.float64)
    return round_to(Rh, store), d
