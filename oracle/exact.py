"""The TLS solution by its definitions (three independent routes).

Problem (abstract, Section 1): min ||[E, r]||_F subject to
(A + E) x = b + r, A m x n, m >= n. With [A, b] = U Sigma V^T the minimal
correction has norm sigma_{n+1} and x_TLS = -v_{1:n,n+1} / v_{n+1,n+1}
(Section 1). The solution exists and is unique when sigma'_n(A) >
sigma_{n+1}([A, b]) (Section 2, conditions for convergence).

Routes:
* ``svd_tls``      LAPACK SVD of [A, b] (and of A for sigma'_n).
* ``mp_svd_tls``   the same definition evaluated in mpmath (brute force in
                   high precision, tiny inputs only).
* ``secular_tls``  the root of the secular equation obtained from the
                   Newton system f = 0, g = 0 (eq. 2) in the SVD basis of
                   A; independent of the SVD of [A, b].

Pins (tests/test_oracle_exact.py): mpmath vs LAPACK on tiny inputs, the
planted-spectrum closed form, the normal-equation identity
(A^T A - sigma^2 I) x = A^T b and sigma^2 = b^T (b - A x), agreement of the
secular and SVD routes.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class TLSSolution:
    sigma: float            # sigma_{n+1}([A, b])
    x: np.ndarray           # x_TLS
    sigma_n_A: float        # sigma'_n(A)
    sigma_1_A: float        # sigma'_1(A)
    sigma_1_Ab: float       # sigma_1([A, b])
    v: np.ndarray | None = None   # right singular vector of sigma_{n+1}

    @property
    def unique(self) -> bool:
        return self.sigma_n_A > self.sigma

    @property
    def kappa_tls(self) -> float:
        """kappa_TLS = sigma'_1 / (sigma'_n - sigma_{n+1}) (Section 1)."""
        return self.sigma_1_A / (self.sigma_n_A - self.sigma)


def _dense(A):
    if hasattr(A, "to_dense"):
        return A.to_dense()
    return np.asarray(A, dtype=np.float64)


def svd_tls(A, b) -> TLSSolution:
    """x_TLS = -v_{1:n,n+1}/v_{n+1,n+1} from the SVD of [A, b] (Section 1)."""
    A = _dense(A)
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[1]
    C = np.column_stack([A, b])
    _, s, Vt = np.linalg.svd(C, full_matrices=False)
    v = Vt[n, :]
    if v[n] == 0.0:
        raise ValueError("v_{n+1,n+1} = 0: TLS solution does not exist")
    x = -v[:n] / v[n]
    sA = np.linalg.svd(A, compute_uv=False)
    return TLSSolution(sigma=float(s[n]), x=x, sigma_n_A=float(sA[-1]),
                       sigma_1_A=float(sA[0]), sigma_1_Ab=float(s[0]), v=v)


def mp_svd_tls(A, b, dps: int = 50) -> TLSSolution:
    """The same definition evaluated with mpmath at ``dps`` digits.

    Tiny inputs only (m <= ~40, n <= ~6): brute force in high precision."""
    import mpmath as mp
    A = _dense(A)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    with mp.workdps(dps):
        C = mp.matrix(m, n + 1)
        for i in range(m):
            for j in range(n):
                C[i, j] = mp.mpf(float(A[i, j]))
            C[i, n] = mp.mpf(float(b[i]))
        # eigen-decomposition of C^T C in high precision: exact squares of
        # the singular values, right singular vectors as eigenvectors
        CtC = C.T * C
        E, Q = mp.eigsy(CtC)
        order = sorted(range(n + 1), key=lambda k: E[k])
        k0 = order[0]
        v = [Q[i, k0] for i in range(n + 1)]
        sigma = mp.sqrt(max(E[k0], mp.mpf(0)))
        sigma1 = mp.sqrt(E[order[-1]])
        x = [-(v[i] / v[n]) for i in range(n)]
        AtA = mp.matrix(n, n)
        for i in range(n):
            for j in range(n):
                AtA[i, j] = CtC[i, j]
        EA = mp.eigsy(AtA, eigvals_only=True)
        EA = sorted([EA[k] for k in range(n)])
        sn = mp.sqrt(max(EA[0], mp.mpf(0)))
        s1 = mp.sqrt(EA[-1])
        return TLSSolution(sigma=float(sigma), x=np.array([float(t) for t in x]),
                           sigma_n_A=float(sn), sigma_1_A=float(s1),
                           sigma_1_Ab=float(sigma1),
                           v=np.array([float(t) for t in v]))


def secular_tls(A, b, iters: int = 400) -> TLSSolution:
    """TLS solution from the Newton system f = 0, g = 0 (eq. 2).

    With A = U' S' V'^T (thin SVD), c = U'^T b and rho^2 = ||b - U' c||^2,
    f = 0 gives x = V' (S'^2 - lam I)^{-1} S' c, and g = 0 (lam = b^T r)
    then reads rho^2 = lam (1 + sum_i c_i^2 / (s_i^2 - lam)). The left side
    is constant and the right side increases from 0 to +inf on
    [0, s_n^2) (when c_n != 0), so the smallest root lam = sigma_{n+1}^2 is
    unique there; it is found by bisection in long double."""
    A = _dense(A)
    b = np.asarray(b, dtype=np.float64)
    n = A.shape[1]
    U, s, Vt = np.linalg.svd(A, full_matrices=False)
    c = U.T @ b
    resid = b - U @ c
    rho2 = np.longdouble(resid.astype(np.longdouble) @ resid.astype(np.longdouble))
    sl = s.astype(np.longdouble)
    cl = c.astype(np.longdouble)
    s2 = sl * sl
    c2 = cl * cl

    def h(lam):
        return lam * (1 + np.sum(c2 / (s2 - lam))) - rho2

    lo = np.longdouble(0)
    hi = s2[-1]
    if c2[-1] == 0:
        raise ValueError("b orthogonal to the last left singular vector: non-unique")
    for _ in range(iters):
        mid = (lo + hi) / 2
        if mid <= lo or mid >= hi:
            break
        if h(mid) > 0:
            hi = mid
        else:
            lo = mid
    lam = (lo + hi) / 2
    x = (Vt.T.astype(np.longdouble) @ (sl * cl / (s2 - lam))).astype(np.float64)
    sigma = float(np.sqrt(lam))
    Cs = np.linalg.svd(np.column_stack([A, b]), compute_uv=False)
    return TLSSolution(sigma=sigma, x=x, sigma_n_A=float(s[-1]),
                       sigma_1_A=float(s[0]), sigma_1_Ab=float(Cs[0]))


def tls_correction(A, b, x) -> tuple[np.ndarray, np.ndarray]:
    """Minimal correction [E, r] = -[A, b] [x; -1] [x; -1]^T / (1 + ||x||^2)
    (rank one, Section 1). Returns (E, r)."""
    A = _dense(A)
    z = np.append(x, -1.0)
    res = A @ x - b
    Er = -np.outer(res, z) / (1.0 + x @ x)
    return Er[:, :-1], Er[:, -1]


def planted_gap_solution(A, x_true, lam):
    """Closed form of the planted-gap instance b = A x_true + e, A^T e = 0,
    with sigma_{n+1}^2 = lam: from f = 0 in eq. (2),
    (A^T A - lam I) x = A^T b = A^T A x_true, so
    x_TLS = x_true + lam (A^T A - lam I)^{-1} x_true. The solve runs on the
    column-equilibrated matrix D^{-1}(A^T A - lam I)D^{-1} by Cholesky.

    Returns (sigma, x_TLS)."""
    import scipy.linalg as sla
    if hasattr(A, "to_scipy"):
        S = A.to_scipy()
        G = (S.T @ S).toarray()
    else:
        A = np.asarray(A, dtype=np.float64)
        G = A.T @ A
    d = np.sqrt(np.diag(G))
    M = G / np.outer(d, d) - lam * np.diag(1.0 / (d * d))
    y = sla.cho_solve(sla.cho_factor(M, lower=False), x_true / d) / d
    return float(np.sqrt(lam)), x_true + lam * y
