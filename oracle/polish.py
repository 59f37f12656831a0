"""Extended-precision evaluation of the Rayleigh quotient and residuals.

The paper evaluates its plotted errors in (simulated) quadruple precision
(Section 4). Here x86-64 ``long double`` (64-bit significand) is used: the
residual r = b - A x is accumulated in long double, so that the Rayleigh
quotient sigma^2 = ||r||^2 / (1 + ||x||^2) (Algorithm 2) is free of the
cancellation that limits its float64 value when ||r|| << ||b||.

``polish`` additionally takes Newton corrections of the system f = 0,
g = 0 (eq. 2) whose residuals f, g are evaluated in long double and whose
linear solves run in float64 (mixed-precision refinement of an RQI
iterate); this moves x from float64's u*kappa_TLS accuracy towards u.

Pins: tests/test_oracle_misc.py (the Rayleigh quotient against the mpmath
route and its second-order stationarity; the polished x against the SVD
solution of the Van Huffel problem).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

LD = np.longdouble


def _residual_ld(A, b, x):
    xl = np.asarray(x, dtype=LD)
    bl = np.asarray(b, dtype=LD)
    if hasattr(A, "row_ptr"):
        prod = A.val.astype(LD) * xl[A.col_idx]
        rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
        Ax = np.zeros(A.m, dtype=LD)
        np.add.at(Ax, rows, prod)
    else:
        Al = np.asarray(A, dtype=LD)
        Ax = Al @ xl
    return bl - Ax


def _rmatvec_ld(A, r):
    rl = np.asarray(r, dtype=LD)
    if hasattr(A, "row_ptr"):
        rows = np.repeat(np.arange(A.m), np.diff(A.row_ptr))
        out = np.zeros(A.n, dtype=LD)
        np.add.at(out, A.col_idx, A.val.astype(LD) * rl[rows])
        return out
    return np.asarray(A, dtype=LD).T @ rl


def rayleigh_ld(A, b, x) -> float:
    """sigma = sqrt(||b - A x||^2 / (1 + ||x||^2)) evaluated in long double."""
    r = _residual_ld(A, b, x)
    xl = np.asarray(x, dtype=LD)
    s2 = (r @ r) / (1 + xl @ xl)
    return float(np.sqrt(s2))


def newton_residual_ld(A, b, x, sigma2=None):
    """f = -A^T r - sigma^2 x, g = -b^T r + sigma^2 (eq. 2) in long double,
    with sigma^2 the long-double Rayleigh quotient unless given."""
    r = _residual_ld(A, b, x)
    xl = np.asarray(x, dtype=LD)
    if sigma2 is None:
        sigma2 = (r @ r) / (1 + xl @ xl)
    s2 = LD(sigma2)
    f = -_rmatvec_ld(A, r) - s2 * xl
    g = -(np.asarray(b, dtype=LD) @ r) + s2
    return f, g, s2


def polish(A, b, x, R=None, steps: int = 2):
    """Newton corrections of (f, g) = 0 at the Rayleigh quotient shift with
    long-double residuals and float64 solves:
    (A^T A - s I) dx = -f solved densely from the float64 Gram matrix,
    followed by the Rayleigh quotient in long double.

    Returns (x, sigma)."""
    from .rqi import gram
    G = gram(A)
    n = G.shape[0]
    x = np.asarray(x, dtype=np.float64).copy()
    for _ in range(steps):
        f, g, s2 = newton_residual_ld(A, b, x)
        J = G - float(s2) * np.eye(n)
        # bordered Newton system for [x; sigma^2] (derivative of eq. 2)
        Atb = _rmatvec_ld(A, np.asarray(b, dtype=LD)).astype(np.float64)
        # eliminate via two solves with J (block Gaussian elimination, Section 2)
        lu = sla.lu_factor(J)
        w = sla.lu_solve(lu, -f.astype(np.float64))
        z = sla.lu_solve(lu, x)
        # linearised g: -b^T(b - A(x+dx)) + s2 + ds = 0 ; dx = w + ds z
        # -> ds (1 + (A^T b)^T z) = -(g + (A^T b)^T w)
        ds = -(float(g) + float(Atb @ w)) / (1.0 + float(Atb @ z))
        x = x + w + ds * z
    return x, rayleigh_ld(A, b, x)
