"""Rayleigh quotient iteration for TLS, as the paper writes it.

* ``textbook_rqi``  Algorithm 1 on a symmetric matrix B.
* ``pcgtls``        Algorithm 3: l-step PCG for (A^T A - sigma^2 I) w = f
                    that touches only the triangular factor R (A^T A ~ R^T R).
* ``rqi_pcgtls``    Algorithm 2 (RQI for TLS) with the inner solves of
                    Algorithm 3, i.e. RQI-PCGTLS; with ``prec_p`` below
                    float64 it is RQI-PCGTLS-MP (Algorithm 4) with the inner
                    solver run in that precision.
* ``csne_ls``       x_LS by corrected semi-normal equations with R (the
                    paper does not say how x_LS is obtained).

Readings of the paper (each listed in the design notes):
* f_k = -A^T r_k - sigma_k^2 x_k: the x in Algorithm 2's f line is x_k,
  as in eq. (2) and Algorithm 4.
* the k-th RQI runs PCGTLS with l = k, i.e. j = 0..k, k+1 steps (Section 2
  and the cost model of Section 3.2 count k+1 steps).
* the PCGTLS loop ends when delta_j = 0 (as printed) and also when
  eta_j = 0 or delta_j, alpha_j is not finite (the step would divide zero
  by zero or carry an overflow into omega), or when eta_j <= u_p^2 eta_0
  (s_j is zero in the working precision relative to s_0); delta_j < 0 means the shifted
  system lost positive definiteness: the loop continues as printed, or
  raises ``IndefiniteError`` when ``strict`` is set.
* the initial step (Algorithm 4, lines 1-5) is in the working precision u
  = float64: u_0 = R^{-1} R^{-T} x_0 with float64 solves on the given
  factor, independent of u_p.
* termination (eq. 4): stop when psi_{k+1} > psi_k (``stop_ge`` uses >= as
  in Example 2); ``patience`` p stops after p consecutive iterations that
  do not improve on the smallest psi; the loop also ends when psi is 0 or
  exactly repeats the previous psi (the iterate no longer moves).
* the returned iterate (the paper does not say which): the latest x_k
  whose psi_k is within a factor ``psi_tie`` (4) of the smallest psi seen
  up to k. psi values that close are at the rounding floor of eq. (4),
  where psi stops telling iterates apart while RQI's iterates still
  converge; a real divergence raises psi by more. psi_tie = 1 returns the
  last iterate that attained the minimum.

Pins: tests/test_oracle_rqi.py (psi_at against a direct evaluation of
eq. (4); the warm candidate against the shifted solve it truncates and its
choice rule; Algorithm 1 equivalence with exact inner
solves, Algorithm 3 special cases sigma = 0 (float64 and float32) and
l >= n, the end of the loop at an underflowed eta and at a non-finite
delta, first-step beta = sigma_0^2, the first iterate independent of u_p
and equal to an LU solve on A^T A, convergence to the SVD solution on the
paper's fixtures and the small dense workload).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable

import numpy as np
import scipy.linalg as sla


class IndefiniteError(RuntimeError):
    """delta_j <= 0 inside PCGTLS: A^T A - sigma^2 I is not positive definite."""


# ----------------------------------------------------------------------------
# operators
# ----------------------------------------------------------------------------

def _as_operator(A):
    """Return (matvec, rmatvec, m, n) for a dense array, scipy sparse or CSR."""
    if hasattr(A, "to_scipy"):
        S = A.to_scipy()
        return (lambda v: S @ v), (lambda v: S.T @ v), A.m, A.n
    if hasattr(A, "tocsr"):
        S = A.tocsr()
        return (lambda v: S @ v), (lambda v: S.T @ v), S.shape[0], S.shape[1]
    A = np.asarray(A, dtype=np.float64)
    return (lambda v: A @ v), (lambda v: A.T @ v), A.shape[0], A.shape[1]


def gram(A) -> np.ndarray:
    """A^T A in float64 (dense result)."""
    if hasattr(A, "to_scipy"):
        S = A.to_scipy()
        return (S.T @ S).toarray()
    A = np.asarray(A, dtype=np.float64)
    return A.T @ A


def cholesky_R(A) -> np.ndarray:
    """Upper triangular R with R^T R = fl(A^T A) (Cholesky of the Gram
    matrix, the preconditioner of Section 2)."""
    G = gram(A)
    return sla.cholesky(G, lower=False)


def _tri_solvers(R: np.ndarray, dtype=np.float64):
    Rp = np.asarray(R, dtype=dtype)

    def solve_R(v):      # R^{-1} v
        return sla.solve_triangular(Rp, np.asarray(v, dtype=dtype), lower=False)

    def solve_RT(v):     # R^{-T} v
        return sla.solve_triangular(Rp, np.asarray(v, dtype=dtype), lower=False, trans="T")

    return solve_R, solve_RT


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

def textbook_rqi(B: np.ndarray, x0: np.ndarray, iters: int):
    """Algorithm 1: rho_0 = x0^T B x0; solve (B - rho I) w = x; x = w/||w||;
    rho = x^T B x. Returns the list of iterates and Rayleigh quotients."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    rho = float(x @ B @ x)
    xs, rhos = [x], [rho]
    I = np.eye(B.shape[0])
    for _ in range(iters):
        w = np.linalg.solve(B - rho * I, x)
        x = w / np.linalg.norm(w)
        rho = float(x @ B @ x)
        xs.append(x)
        rhos.append(rho)
    return xs, rhos


# ----------------------------------------------------------------------------
# Algorithm 3
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class PCGTrace:
    eta: list
    delta: list
    steps: int
    negatives: int = 0


def pcgtls(solve_R: Callable, solve_RT: Callable, sigma2: float, f: np.ndarray,
           l: int, dtype=np.float64, trace: bool = False, strict: bool = False,
           eta_floor: float | None = None):
    """Algorithm 3, l-step PCGTLS for (A^T A - sigma^2 I) w = f.

    CG on the preconditioned matrix C = I - sigma^2 R^{-T} R^{-1} with the
    solution carried back as w = R^{-1} y. Iterations j = 0, 1, ..., l.
    All vectors and scalars are held in ``dtype``.

    When the loop ends early. The printed condition is delta_j != 0. Step j
    also does not run when eta_j = 0 (s_j = 0 in the working precision:
    omega_j already solves the system, and the next beta would be 0/0), or
    when delta_j or alpha_j = eta_j / delta_j is not a finite number, or
    (j > 0) when eta_j <= eta_floor eta_0: s_j is then zero in the working
    precision relative to s_0 and further steps only add rounding to omega.
    eta_floor defaults to u_p^2 of ``dtype`` (2^-48 for float32, 2^-106 for
    float64); 0 turns that test off. The check comes before the step's
    update, so a step either runs whole or not at all. A negative delta_j (the shifted system is indefinite) is
    counted in the trace and the iteration continues, unless ``strict``
    asks for ``IndefiniteError``."""
    dt = np.dtype(dtype)
    s2 = dt.type(sigma2)
    f = np.asarray(f, dtype=dt)
    omega = np.zeros_like(f)
    s = np.asarray(solve_RT(f), dtype=dt)            # s_0 = R^{-T} f
    p = s.copy()                                     # p_0 = s_0
    eta = dt.type(s @ s)                             # eta_0 = ||s_0||^2
    etas, deltas = [float(eta)], []
    steps = 0
    negatives = 0
    if eta_floor is None:
        eta_floor = 2.0 ** -48 if dt == np.float32 else 2.0 ** -106
    floor = dt.type(eta_floor) * eta                 # eta_floor eta_0 (0: off)
    for _ in range(l + 1):
        if eta == 0 or (steps > 0 and eta <= floor):  # s_j = 0 in the working precision
            break
        q = np.asarray(solve_R(p), dtype=dt)         # q_j = R^{-1} p_j
        delta = dt.type(p @ p) - s2 * dt.type(q @ q)  # delta_j = ||p||^2 - sigma^2 ||q||^2
        deltas.append(float(delta))
        if delta == 0 or not np.isfinite(delta):
            break
        with np.errstate(over="ignore"):
            alpha = eta / delta                      # alpha_j
        if not np.isfinite(alpha):
            break
        if delta < 0:
            if strict:
                raise IndefiniteError(f"delta_{steps} = {float(delta):.3e} <= 0")
            negatives += 1
        omega = omega + alpha * q                    # omega_{j+1}
        q = np.asarray(solve_RT(q), dtype=dt)        # q_j = R^{-T} q_j
        s = s - alpha * (p - s2 * q)                 # s_{j+1}
        eta_new = dt.type(s @ s)                     # eta_{j+1}
        etas.append(float(eta_new))
        steps += 1
        if eta_new == 0:                             # beta_j and p_{j+1} are not needed
            break
        beta = eta_new / eta                         # beta_j
        p = s + beta * p                             # p_{j+1}
        eta = eta_new
    if trace:
        return omega, PCGTrace(etas, deltas, steps, negatives)
    return omega


# ----------------------------------------------------------------------------
# x_LS
# ----------------------------------------------------------------------------

def csne_ls(A, b, R, corrections: int = 1) -> np.ndarray:
    """Least-squares solution by corrected semi-normal equations:
    x = R^{-1} R^{-T} A^T b, then ``corrections`` steps
    x += R^{-1} R^{-T} A^T (b - A x) with the residual in float64."""
    mv, rmv, _, _ = _as_operator(A)
    solve_R, solve_RT = _tri_solvers(R)
    x = solve_R(solve_RT(rmv(b)))
    for _ in range(corrections):
        x = x + solve_R(solve_RT(rmv(b - mv(x))))
    return x


# ----------------------------------------------------------------------------
# Algorithms 2 and 4
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class RQIResult:
    x: np.ndarray             # the returned iterate (latest within psi_tie of the smallest psi)
    sigma: float              # its Rayleigh quotient sqrt
    k_best: int
    iters: int                # RQI iterations performed (k of the last psi)
    psi: list                 # psi_k, k = 1..iters
    sigma_hist: list          # sigma_k, k = 1..iters
    x_hist: list              # x_k, k = 1..iters (x_k that gave psi_k)
    pcg_steps: int
    stopped: str              # "psi", "kmax", "converged" (psi 0 or repeated)


def rayleigh(A_mv, b, x):
    """r = b - A x, sigma^2 = r^T r / (1 + x^T x) (Algorithm 2)."""
    r = b - A_mv(x)
    return r, float(r @ r) / (1.0 + float(x @ x))


def rqi_pcgtls(A, b, R=None, *, x0=None, kmax: int = 100, patience: int = 1,
               stop_ge: bool = False, prec_p=np.float64, steps_rule=None,
               ls_corrections: int = 1, shift_clamp: float | None = None,
               solvers=None, record: bool = True, psi_tie: float = 4.0,
               eta_floor: float | None = None) -> RQIResult:
    """RQI-PCGTLS (Algorithm 2 with Algorithm 3 inner solves).

    The working precision u is float64 throughout; ``prec_p`` is the
    PCGTLS precision u_p of Algorithm 4 (the vectors entering PCGTLS are
    rounded to it and its arithmetic runs in it). ``R`` may be any upper
    triangular factor with R^T R ~ A^T A (computed in any precision u_q);
    ``solvers`` overrides how R^{-1} and R^{-T} are applied.

    ``steps_rule(k)`` gives l for the k-th RQI (default l = k: k+1 steps).
    ``shift_clamp``: if given (a value mu_max), the shift used in the k-th
    iteration is min(sigma_k^2, mu_max) (a deviation for starts that violate
    the positive definiteness assumption; off by default).
    ``psi_tie`` (>= 1): which iterate is returned (see the module notes)."""
    if not psi_tie >= 1.0:
        raise ValueError("psi_tie must be >= 1")
    mv, rmv, m, n = _as_operator(A)
    b = np.asarray(b, dtype=np.float64)
    if R is None and solvers is None:
        R = cholesky_R(A)
    if solvers is None:
        solve_R, solve_RT = _tri_solvers(R, prec_p)
    else:
        solve_R, solve_RT = solvers
    if steps_rule is None:
        steps_rule = lambda k: k

    def inner(sig2, rhs, l):
        w = pcgtls(solve_R, solve_RT, sig2, np.asarray(rhs, dtype=prec_p), l, dtype=prec_p,
                   eta_floor=eta_floor)
        return np.asarray(w, dtype=np.float64)

    # lines 1-5: x_0 = x_LS, one inverse-iteration step with shift 0
    if x0 is None:
        x = x_ls(A, b, R if R is not None else None, ls_corrections,
                 solvers=None if R is not None else (solve_R, solve_RT))
    else:
        x = np.asarray(x0, dtype=np.float64).copy()
    r0, sig0_2 = rayleigh(mv, b, x)
    # Algorithm 4 runs the initial solve A^T A u_0 = x_0 in the working
    # precision u (float64) with the factor as given, whatever u_p is
    if R is not None:
        u_R, u_RT = _tri_solvers(R)
    else:
        u_R, u_RT = solve_R, solve_RT
    u0 = np.asarray(u_R(u_RT(x)), dtype=np.float64)
    x = x + sig0_2 * u0
    pcg_total = 2
    best = (math.inf, None, None, 0)
    psi_min = math.inf
    psis, sigs, xs = [], [], []
    no_improve = 0
    stopped = "kmax"
    k = 0
    for k in range(1, kmax + 1):
        r, sig2 = rayleigh(mv, b, x)                 # r_k, sigma_k^2
        shift = sig2 if shift_clamp is None else min(sig2, shift_clamp)
        Atr = rmv(r)
        f = -Atr - shift * x                         # f_k
        g = -float(b @ r) + shift                    # g_k
        if shift != sig2:                            # psi always at sigma_k^2
            fp, gp = -Atr - sig2 * x, -float(b @ r) + sig2
        else:
            fp, gp = f, g
        psi = math.sqrt((float(fp @ fp) + gp * gp) / (float(x @ x) + 1.0))   # eq. (4)
        psis.append(psi)
        sigs.append(math.sqrt(sig2))
        if record:
            xs.append(x.copy())
        if k == 1 or psi <= psi_tie * psi_min:      # the latest iterate within the band
            best = (psi, x.copy(), math.sqrt(sig2), k)
        if psi < psi_min:
            psi_min = psi
            no_improve = 0
        elif (psi >= psi_min) if stop_ge else (psi > psi_min):
            no_improve += 1
        if psi == 0.0 or (k > 1 and psi == psis[-2]):
            stopped = "converged"
            break
        if no_improve >= patience:
            stopped = "psi"
            break
        l = steps_rule(k)
        omega = inner(shift, -f, l)                  # (A^T A - s I) w = -f
        z = x + omega
        beta = (float(z @ f) - g) / (float(z @ x) + 1.0)
        u = inner(shift, x, l)                       # (A^T A - s I) u = x
        x = z + beta * u
        pcg_total += 2 * (l + 1)
    psi_b, x_b, s_b, k_b = best
    return RQIResult(x=x_b, sigma=s_b, k_best=k_b, iters=k, psi=psis,
                     sigma_hist=sigs, x_hist=xs, pcg_steps=pcg_total, stopped=stopped)


def x_ls(A, b, R, corrections: int = 1, solvers=None):
    """x_LS by the semi-normal equations R^T R x = A^T b with the factor in
    float64, then ``corrections`` corrected steps x += (R^T R)^{-1} A^T (b - A x)
    (the paper does not say how x_LS is computed; this is the reading used)."""
    mv, rmv, _, _ = _as_operator(A)
    b = np.asarray(b, dtype=np.float64)
    sR, sRT = _tri_solvers(R) if solvers is None else solvers
    x = sR(sRT(rmv(b)))
    for _ in range(corrections):
        x = x + sR(sRT(rmv(b - mv(x))))
    return np.asarray(x, dtype=np.float64)


def psi_at(A, b, x):
    """psi of eq. (4) at x, with sigma^2 the Rayleigh quotient of Algorithm 2:
    r = b - A x, sigma^2 = ||r||^2 / (1 + ||x||^2), f = -A^T r - sigma^2 x,
    g = -b^T r + sigma^2, psi = ((||f||^2 + g^2) / (||x||^2 + 1))^{1/2}."""
    mv, rmv, _, _ = _as_operator(A)
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r = b - mv(x)
    s2 = float(r @ r) / (1.0 + float(x @ x))
    f = -rmv(r) - s2 * x
    g = -float(b @ r) + s2
    return math.sqrt((float(f @ f) + g * g) / (float(x @ x) + 1.0))


def warm_candidate(A, b, R, x0, sigma_hat):
    """The warm start's candidate for x_1 (a project addition, not in the
    paper). At x_0 = x_LS (A^T r_0 = 0), the Algorithm 2 body at a shift lam
    solves (A^T A - lam I) y = x_0 for the correction; its Neumann series in
    lam (A^T A)^{-1} truncated after two terms gives
    x_1w = x_0 + lam u_0 + lam^2 u_1 with u_0 = (A^T A)^{-1} x_0 and
    u_1 = (A^T A)^{-1} u_0, applied through the factor (R^T R = A^T A) in
    float64. sigma_hat is capped at sigma_0 = ||r_0|| / (1 + ||x_0||^2)^{1/2}
    (sigma_{n+1} <= sigma_0). The plain x_1 = x_0 + sigma_0^2 u_0 is the
    shift-0 step of Algorithm 2 (lines 1-5); the start kept is the one with
    the smaller psi (eq. 4), the plain one on a tie.

    Returns (x_kept, warm_taken, psi_warm, psi_plain, sigma_hat_used)."""
    mv, _, _, _ = _as_operator(A)
    x0 = np.asarray(x0, dtype=np.float64)
    sR, sRT = _tri_solvers(R)
    u0 = sR(sRT(x0))
    u1 = sR(sRT(u0))
    r0 = np.asarray(b, dtype=np.float64) - mv(x0)
    s0 = math.sqrt(float(r0 @ r0) / (1.0 + float(x0 @ x0)))
    sh = min(float(sigma_hat), s0)
    lam = sh * sh
    xw = x0 + lam * u0 + (lam * lam) * u1
    xp = x0 + (s0 * s0) * u0
    pw, pp = psi_at(A, b, xw), psi_at(A, b, xp)
    take = pw < pp
    return (xw if take else xp), bool(take), pw, pp, sh


def inverse_step_body(A, b, x, shift, solve):
    """One body of Algorithm 2 at a given shift with an exact solver
    ``solve(shift, rhs)`` for (A^T A - shift I) y = rhs. With shift = 0 and
    x = x_LS it reproduces the initial step (lines 1-5), since then
    f = 0, omega = 0 and beta = sigma_0^2."""
    mv, rmv, _, _ = _as_operator(A)
    r = b - mv(x)
    f = -rmv(r) - shift * x
    g = -float(b @ r) + shift
    omega = solve(shift, -f)
    z = x + omega
    beta = (float(z @ f) - g) / (float(z @ x) + 1.0)
    u = solve(shift, x)
    return z + beta * u, beta
