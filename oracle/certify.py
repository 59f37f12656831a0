"""A-posteriori certificates of a computed TLS pair (sigma, x).

Each check restates a fact of the paper about the exact solution:

* Newton residual (eq. 2): at the solution f = -A^T r - sigma^2 x = 0 and
  g = -b^T r + sigma^2 = 0 with r = b - A x, i.e. the normal-equation
  identity (A^T A - sigma^2 I) x = A^T b and sigma^2 = b^T (b - A x).
* Rayleigh quotient (Algorithm 2): sigma^2 = ||r||^2 / (1 + ||x||^2).
* Smallest root: the solution is the one with sigma < sigma'_n(A)
  (existence and uniqueness condition, Section 2), certified by the
  success of a Cholesky factorization of A^T A - sigma^2 (1 + tau) I.
* Existence margin (sigma'_n - sigma_{n+1}) / sigma'_n and
  kappa_TLS = sigma'_1 / (sigma'_n - sigma_{n+1}) (Section 1).

The scales are chosen so that float64 round-off of a correct answer gives
values of order one times the unit roundoff (see each function).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla

from .polish import _residual_ld, _rmatvec_ld, LD
from .rqi import gram

U64 = 2.0 ** -53


@dataclasses.dataclass
class Certificate:
    normal_eq: float        # ||(A^TA - s^2 I)x - A^T b|| / (||A||_F^2 ||x|| + ||A^T b||)
    g_rel: float            # |s^2 - b^T(b - Ax)| / (||b|| (||b|| + ||A||_F ||x||))
    rq_rel: float           # |s - sqrt(||r||^2/(1+||x||^2))| / s
    smallest_root: bool     # chol(A^TA - s^2(1+tau) I) succeeds


def normA_F(A) -> float:
    if hasattr(A, "val"):
        return float(np.linalg.norm(A.val))
    return float(np.linalg.norm(np.asarray(A)))


def certify(A, b, x, sigma, tau: float = 1e-8, G=None) -> Certificate:
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = _residual_ld(A, b, x)
    s2 = LD(sigma) ** 2
    f = _rmatvec_ld(A, r) + s2 * np.asarray(x, dtype=LD)   # = A^T b - (A^TA - s^2 I) x
    nA = normA_F(A)
    Atb = _rmatvec_ld(A, np.asarray(b, dtype=LD))
    nx = float(np.linalg.norm(x))
    ne = float(np.sqrt(f @ f)) / (nA * nA * nx + float(np.sqrt(Atb @ Atb)))
    g = float(s2 - np.asarray(b, dtype=LD) @ r)
    nb = float(np.linalg.norm(b))
    g_rel = abs(g) / (nb * (nb + nA * nx))
    rq = float(np.sqrt((r @ r) / (1 + LD(nx) ** 2)))
    rq_rel = abs(rq - sigma) / max(sigma, 1e-300)
    if G is None:
        G = gram(A)
    try:
        sla.cholesky(G - (sigma ** 2) * (1.0 + tau) * np.eye(G.shape[0]), lower=False)
        ok = True
    except np.linalg.LinAlgError:
        ok = False
    return Certificate(normal_eq=ne, g_rel=g_rel, rq_rel=rq_rel, smallest_root=ok)


def existence_margin(sigma_n_A: float, sigma: float) -> float:
    """(sigma'_n - sigma_{n+1}) / sigma'_n; positive iff the TLS solution is
    unique (Section 2)."""
    return (sigma_n_A - sigma) / sigma_n_A


def kappa_tls(sigma_1_A: float, sigma_n_A: float, sigma: float) -> float:
    """kappa_TLS = sigma'_1 / (sigma'_n - sigma_{n+1}) (Section 1)."""
    return sigma_1_A / (sigma_n_A - sigma)


def attainable(sigma_1_Ab: float, sigma: float, kap_tls: float, u: float = U64):
    """Rounding-level accuracy to expect from any float64 method: for sigma
    about u sigma_1([A,b]) / sigma_{n+1} (a Weyl bound on the data), for x
    about u kappa_TLS (Section 1). Returns (bound_sigma, bound_x)."""
    return u * sigma_1_Ab / max(sigma, 1e-300), u * kap_tls
