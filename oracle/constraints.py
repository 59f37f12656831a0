"""Constraints on the factorization precision u_q (Section 3.1).

All formulas take exact singular values (from a dense SVD), so that the
GPU gate's estimates can be checked against them. The paper's heuristics
drop their constants ("roughly"); they are evaluated here constant-free,
which reproduces the magnitudes printed for the model problems of
Section 4.

* ``bound_qr_nonsingular``    u_q < 1/(c m n^{3/2} kappa(A)) (Householder QR,
                              R-hat nonsingular), with c = 1.
* ``bound_qr_probabilistic``  u_q < 1/(c m^{1/2} n^{3/4} kappa(A)).
* ``bound5``                  heuristic (5): u_q <~ kappa(A)^{-1}.
* ``bound_wilkinson``         Cholesky of fl(A^T A) succeeds if
                              u_q <= 1/(20 n^{3/2} kappa(A)^2).
* ``bound_chol``              heuristic u_q <~ kappa(A)^{-2}.
* ``bound_hp``                two-sided scaling H = D^{-1} fl(A^T A) D^{-1}:
                              u_q < lam_min(H) / ((2 lam_min(H) + n)(n+1)).
* ``bound6``                  heuristic (6): u_q <~ kappa_F(A)^{-1}
                              (1 - sigma_{n+1}^2 / sigma'_n^2), which depends
                              on b through sigma_{n+1}.

Reading: kappa_F(A) = ||A||_F ||A^+||_2 = ||A||_F / sigma'_n, the
combination that appears in the bound on ||Delta||_2 (the product of
||Delta A||_F <~ gamma ||A||_F and ||R-hat^{-1}||_2 = 1/sigma'_n).

Pins: tests/test_oracle_misc.py (every bound in closed form on a diagonal
A and on two columns at a given angle, where kappa, kappa_F, lambda_min(H),
sigma'_n and sigma_{n+1} are known exactly; constant-free magnitudes on the
model problems against the values printed in Section 4).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

UNIT_ROUNDOFF = {   # Table 2, plus bfloat16 (8-bit significand)
    "fp16": 2.0 ** -11,      # 4.88e-4
    "fp32": 2.0 ** -24,      # 5.96e-8
    "fp64": 2.0 ** -53,      # 1.11e-16
    "fp128": 2.0 ** -113,    # 9.63e-35
    "bf16": 2.0 ** -8,       # 3.91e-3 (not in the paper)
}


@dataclasses.dataclass
class Bounds:
    kappa: float
    kappa_F: float
    sigma_n_A: float
    sigma: float
    qr_nonsingular: float
    qr_probabilistic: float
    bound5: float
    wilkinson: float
    chol: float
    hp: float
    bound6: float


def _dense(A):
    if hasattr(A, "to_dense"):
        return A.to_dense()
    return np.asarray(A, dtype=np.float64)


def bounds(A, b, scaled: bool = False) -> Bounds:
    """Every bound of Section 3.1 for the data (A, b).

    With ``scaled``, kappa and kappa_F refer to the column-equilibrated
    A D^{-1} (D = diag(||A e_j||)), the matrix a scaled low-precision
    factorization actually sees; sigma'_n and sigma_{n+1} stay those of the
    TLS problem (A, b)."""
    A = _dense(A)
    b = np.asarray(b, dtype=np.float64)
    m, n = A.shape
    sA = np.linalg.svd(A, compute_uv=False)
    sC = np.linalg.svd(np.column_stack([A, b]), compute_uv=False)
    sigma = float(sC[-1])
    sn = float(sA[-1])
    if scaled:
        d = np.linalg.norm(A, axis=0)
        As = A / d
        ss = np.linalg.svd(As, compute_uv=False)
        kap = float(ss[0] / ss[-1])
        kapF = float(np.linalg.norm(As) / ss[-1])
    else:
        kap = float(sA[0] / sA[-1])
        kapF = float(np.linalg.norm(A) / sA[-1])
    G = A.T @ A
    d = np.sqrt(np.diag(G))
    H = G / np.outer(d, d)
    lam_min = float(np.linalg.eigvalsh(H)[0])
    hp = lam_min / ((2 * lam_min + n) * (n + 1))
    gap = 1.0 - (sigma / sn) ** 2
    return Bounds(
        kappa=kap, kappa_F=kapF, sigma_n_A=sn, sigma=sigma,
        qr_nonsingular=1.0 / (m * n ** 1.5 * kap),
        qr_probabilistic=1.0 / (math.sqrt(m) * n ** 0.75 * kap),
        bound5=1.0 / kap,
        wilkinson=1.0 / (20 * n ** 1.5 * kap ** 2),
        chol=1.0 / kap ** 2,
        hp=hp,
        bound6=gap / kapF,
    )


def ctilde_interval(sigma_n_A: float, sigma: float):
    """Eigenvalue interval of C-tilde = I - sigma^2 R^{-T} R^{-1} for the
    exact factor at sigma = sigma_{n+1}: [1 - sigma^2/sigma'_n^2, 1]
    (Section 3.1)."""
    return 1.0 - (sigma / sigma_n_A) ** 2, 1.0
