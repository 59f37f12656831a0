"""Warm-start features of a TLS problem, by their definitions (float64).

A project addition (not in the paper). The quantities are those of the
initial step of Algorithm 2: x_0 = x_LS, r_0 = b - A x_0,
sigma_0^2 = ||r_0||^2 / (1 + ||x_0||^2), u_0 = (A^T A)^{-1} x_0, plus
u_1 = (A^T A)^{-1} u_0, the Ritz values of (A^T A)^{-1} on span{x_0, u_0}
and the column norms d_j = ||A e_j||. The index list is the one of the
library's header (32 values, natural logarithms).

Here every quantity is computed from its definition with dense LAPACK
routines (least squares by an orthogonal factorization, solves with A^T A,
Ritz values as eigenvalues of the projected operator on an orthonormal
basis); the library takes them from the factor R and a closed-form 2x2
eigenproblem. Pinned by tests/test_oracle_features.py (Cauchy interlacing of
the Ritz values, the exact eigenvector case, direct identities).
"""
from __future__ import annotations

import math

import numpy as np


def _dense(A):
    if hasattr(A, "to_dense"):
        return A.to_dense()
    return np.asarray(A, dtype=np.float64)


def ritz_values(G, x0, u0):
    """Ritz values (max, min) of G^{-1} on span{x0, u0} (orthonormal basis).
    When u0 is parallel to x0 to within an angle of 1e-6 the span is read as
    one-dimensional and both values are the Rayleigh quotient at x0."""
    Q, R = np.linalg.qr(np.column_stack([x0, u0]))
    if abs(R[1, 1]) <= 1e-6 * np.linalg.norm(u0):
        th = float(x0 @ np.linalg.solve(G, x0) / (x0 @ x0))
        return th, th
    Mq = np.linalg.solve(G, Q)
    T = Q.T @ Mq
    ev = np.linalg.eigvalsh(0.5 * (T + T.T))
    return float(ev[-1]), float(ev[0])


def gauss_gap(G, x0, u0, rr, floor=1e-13):
    """Relative gap 1 - lam / sigma_0^2 with lam solving
    lam (1 + x0^T (I - lam G^{-1})^{-1} x0) = rr, the quadratic form taken by
    the two-point Gauss rule of the Krylov space span{x0, G^{-1} x0}:
    nodes = eigenvalues of the projected G^{-1} on an orthonormal basis whose
    first vector is x0 / ||x0||, weights ||x0||^2 times the squared first
    components of the eigenvectors. The scalar equation is solved by
    bisection on [0, min(rr, 1 / node_max))."""
    xx = x0 @ x0
    Q, R = np.linalg.qr(np.column_stack([x0, u0]))
    if abs(R[1, 1]) <= 1e-6 * np.linalg.norm(u0):
        nodes = np.array([x0 @ np.linalg.solve(G, x0) / xx])
        weights = np.array([xx])
    else:
        T = Q.T @ np.linalg.solve(G, Q)
        nodes, Z = np.linalg.eigh(0.5 * (T + T.T))
        weights = xx * Z[0, :] ** 2
    lo, hi = 0.0, min(rr, 1.0 / nodes.max())
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        val = mid * (1.0 + np.sum(weights / (1.0 - mid * nodes))) - rr
        if val > 0:
            hi = mid
        else:
            lo = mid
    s02 = rr / (1.0 + xx)
    return max(1.0 - 0.5 * (lo + hi) / s02, floor)


def warm_features(A, b):
    """The 32 features and the intermediate quantities (dict)."""
    A = _dense(A)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    x0 = np.linalg.lstsq(A, b, rcond=None)[0]
    G = A.T @ A
    u0 = np.linalg.solve(G, x0)
    u1 = np.linalg.solve(G, u0)
    r0 = b - A @ x0
    xx, xu, uu, uv, vv = x0 @ x0, x0 @ u0, u0 @ u0, u0 @ u1, u1 @ u1
    rr = r0 @ r0
    s02 = rr / (1.0 + xx)
    s0 = math.sqrt(s02)
    t = s02 * xu / (1.0 + xx)
    thmax, thmin = ritz_values(G, x0, u0)
    d = np.linalg.norm(A, axis=0)
    ld = np.log(d)
    nA = np.linalg.norm(A)
    nb = np.linalg.norm(b)
    natb = np.linalg.norm(A.T @ b)
    L = math.log
    f = np.zeros(32)
    f[0], f[1] = L(m), L(n)
    f[2], f[3], f[4] = L(nA), L(nb), L(natb)
    f[5], f[6], f[7] = L(s0), 0.5 * L(xx), 0.5 * L(rr)
    f[8] = f[7] - f[3]
    f[9] = L(t)
    f[10] = 0.5 * L(uu / xx)
    f[11], f[12] = -0.5 * L(thmax), -0.5 * L(thmin)
    f[13] = f[5] - f[11]
    f[14] = s02 * thmax
    f[15] = t / (1.0 + t)
    f[16], f[17], f[18], f[19] = ld.min(), ld.max(), ld.mean(), ld.std()
    f[20] = f[4] - f[2] - f[3]
    f[21] = math.log1p(xx)
    f[22] = L(uv * xx / (xu * uu))
    f[23] = L(uu * xx / (xu * xu))
    f[24] = f[2] - 0.5 * f[1] - f[5]
    f[25] = f[3] - 0.5 * f[0]
    f[26] = 0.5 * L(thmax / thmin)
    f[27] = L(s02 * uv / uu)
    f[28] = L(s02 * math.sqrt(vv / uu))
    f[29] = 0.5 * L(s02 * s02 * vv / xx)
    f[30] = 1.0
    f[31] = L(gauss_gap(G, x0, u0, rr))
    return f, {"x0": x0, "u0": u0, "u1": u1, "sigma0": s0, "thmax": thmax, "thmin": thmin,
               "G": G}
