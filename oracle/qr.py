"""Householder QR preconditioner (Section 3, QR variant).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this module; the library never does.

The mixed-precision method computes the R-factor of A = Q [R; 0] by
Householder QR in precision u_q instead of the Cholesky factor of A^T A
(Section 3). For full-rank A the two factors coincide in exact arithmetic
(Section 3), but the QR route keeps the condition number unsquared:
constraint (5) asks u_q <~ kappa(A)^{-1} for QR against kappa(A)^{-2} for
Cholesky of fl(A^T A). The backward error of the computed factor is
A + Delta A = Q_1 R_hat with ||Delta A||_F <= gamma_mn ||A||_F (Section 3.1).

This module:

1. ``householder_r``: the textbook column-by-column Householder QR, each
   reflector H_j = I - tau_j v_j v_j^T with v_j(j) = 1 chosen so that H_j
   maps column j (rows j..m-1) to beta_j e_j, beta_j = -sign(alpha) ||x||
   (the sign that avoids cancellation); no reflection when the column is
   already zero below the diagonal. With ``fmt`` below fp64 the stored
   quantities (the updated trailing block and the diagonal) are rounded to
   ``fmt`` after every column step, the arithmetic of each step itself being
   float64: a simulation of QR carried out in u_q with wide accumulation.
   The rows of R are given a nonnegative diagonal (R^T R is unchanged).
2. ``scaled_qr_factor``: the preconditioner as the library forms it for a
   u_q below fp64: d_j = ||A e_j||, A-hat = fl_q(A D^{-1}) (round to nearest
   even), R_hat = R(A-hat) in u_q, stored rounded to ``store``; R = R_hat D.

Pins: tests/test_oracle_qr.py (LAPACK's R through numpy, the Cholesky
factor of A^T A, closed forms for one and two columns, invariance under row
permutations and the stacking identity R([A1; A2]) = R([R(A1); R(A2)]), the
backward-error and preconditioned-spectrum bounds of Section 3.1 in fp16
and bf16).
"""
from __future__ import annotations

import numpy as np

from .lowprec import column_norms, round_to


def _densify(A) -> np.ndarray:
    if hasattr(A, "val"):
        rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
        D = np.zeros((A.m, A.n))
        D[rows, A.col_idx] = A.val
        return D
    return np.array(A, dtype=np.float64)


def householder_r(A, fmt: str = "fp64") -> np.ndarray:
    """R (n x n, nonnegative diagonal) of the Householder QR of A (m x n,
    m >= n), computed column by column (step 1 of the module text)."""
    W = np.array(_densify(A), dtype=np.float64)
    m, n = W.shape
    if m < n:
        raise ValueError("householder_r needs m >= n")
    rnd = (lambda v: v) if fmt == "fp64" else (lambda v: round_to(v, fmt))
    W = rnd(W)
    for j in range(n):
        x = W[j:, j].copy()
        alpha = x[0]
        s = float(x[1:] @ x[1:])
        if s == 0.0:
            continue                           # already triangular here: H_j = I
        beta = -np.copysign(np.sqrt(alpha * alpha + s), alpha)
        v = x / (alpha - beta)
        v[0] = 1.0
        tau = (beta - alpha) / beta
        W[j, j] = rnd(np.array([beta]))[0]
        W[j + 1:, j] = 0.0
        if j + 1 < n:
            w = v @ W[j:, j + 1:]              # v^T (trailing block)
            W[j:, j + 1:] = rnd(W[j:, j + 1:] - tau * np.outer(v, w))
    R = np.triu(W[:n, :])
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return R * s[:, None]


def scaled_qr_factor(A, fmt: str = "fp16", store: str | None = None):
    """Step 2 of the module text. Returns (R_hat as float64 holding
    ``store``-rounded values, d); R = R_hat * d[None, :]."""
    store = fmt if store is None else store
    d = column_norms(A)
    Ah = round_to(_densify(A) / d[None, :], fmt)
    Rh = householder_r(Ah, fmt)
    return round_to(Rh, store), d
