"""Pins of oracle.rqi: Algorithms 1-4 against facts fixed independently.

* Algorithm 2 with exact inner solves is inverse iteration on
  B = [A b]^T [A b] at the Rayleigh quotient shift, i.e. Algorithm 1,
  normalised to last component -1.
* Algorithm 3 at sigma = 0 returns R^{-1} R^{-T} f after one step; with
  l >= n steps it returns the dense solve of (A^T A - sigma^2 I) w = f.
* The body of Algorithm 2 at shift 0 from x_LS gives beta = sigma_0^2
  (lines 1-5 are that body).
* RQI-PCGTLS converges to the SVD solution on the small workloads.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import tlsgen
from oracle import exact, rqi, certify, constraints


def _exact_solver(A):
    G = rqi.gram(A)
    return lambda s, rhs: np.linalg.solve(G - s * np.eye(G.shape[0]), rhs)


def test_algorithm2_equals_algorithm1_with_exact_solves():
    A, b, _ = tlsgen.dense_gaussian(40, 4, seed=21)
    B = np.column_stack([A, b]).T @ np.column_stack([A, b])
    x = np.linalg.lstsq(A, b, rcond=None)[0] + 0.3      # a start away from x_TLS
    solve = _exact_solver(A)
    v = np.append(x, -1.0)
    xs_tb, rhos = rqi.textbook_rqi(B, v, 3)
    xk = x.copy()
    for k in range(1, 4):
        r = b - A @ xk
        sig2 = r @ r / (1 + xk @ xk)
        # Algorithm 1's Rayleigh quotient is the same number
        assert abs(sig2 - rhos[k - 1]) / rhos[k - 1] < 1e-10
        xk, _ = rqi.inverse_step_body(A, b, xk, sig2, solve)
        w = xs_tb[k]
        x_tb = -w[:-1] / w[-1]
        assert np.linalg.norm(xk - x_tb) / np.linalg.norm(x_tb) < 1e-9


def test_pcgtls_sigma_zero_is_two_triangular_solves():
    A, b, _ = tlsgen.dense_gaussian(30, 6, seed=2)
    R = rqi.cholesky_R(A)
    sR, sRT = rqi._tri_solvers(R)
    f = np.random.default_rng(0).standard_normal(6)
    w, tr = rqi.pcgtls(sR, sRT, 0.0, f, l=5, trace=True)
    expect = sla.solve_triangular(R, sla.solve_triangular(R, f, trans="T"))
    assert np.allclose(w, expect, rtol=1e-13, atol=0)
    # s_1 = 0 -> eta_1 = 0 -> p_1 = 0 -> delta_1 = 0 ends the loop
    assert tr.steps == 1 and tr.eta[1] == 0.0 and tr.delta[1] == 0.0


def test_pcgtls_full_steps_is_dense_solve():
    A, b, _ = tlsgen.dense_gaussian(50, 8, seed=4)
    R = rqi.cholesky_R(A)
    sR, sRT = rqi._tri_solvers(R)
    s = exact.svd_tls(A, b)
    sig2 = (0.5 * s.sigma_n_A) ** 2
    f = np.random.default_rng(1).standard_normal(8)
    w = rqi.pcgtls(sR, sRT, sig2, f, l=3 * 8)
    ref = np.linalg.solve(A.T @ A - sig2 * np.eye(8), f)
    assert np.linalg.norm(w - ref) / np.linalg.norm(ref) < 1e-12


def test_pcgtls_is_cg_on_preconditioned_system():
    # first step by hand: alpha_0 = eta_0/delta_0 along p_0 = s_0 = R^{-T} f
    A, b, _ = tlsgen.dense_gaussian(30, 5, seed=8)
    R = rqi.cholesky_R(A)
    sR, sRT = rqi._tri_solvers(R)
    f = np.random.default_rng(3).standard_normal(5)
    sig2 = 0.3
    w = rqi.pcgtls(sR, sRT, sig2, f, l=0)
    Ri = np.linalg.inv(R)
    C = np.eye(5) - sig2 * Ri.T @ Ri
    s0 = Ri.T @ f
    alpha = (s0 @ s0) / (s0 @ C @ s0)
    assert np.allclose(w, alpha * Ri @ s0, rtol=1e-12, atol=0)


def test_first_step_beta_is_sigma0_squared():
    A, b, _ = tlsgen.dense_gaussian(80, 7, seed=5)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    r0 = b - A @ x_ls
    sig0 = r0 @ r0 / (1 + x_ls @ x_ls)
    x1, beta = rqi.inverse_step_body(A, b, x_ls, 0.0, _exact_solver(A))
    assert abs(beta - sig0) / sig0 < 1e-9
    u0 = np.linalg.solve(A.T @ A, x_ls)
    assert np.allclose(x1, x_ls + sig0 * u0, rtol=1e-9, atol=0)


def test_csne_is_least_squares():
    A, b, _, _ = tlsgen.sparse_scaled(3000, 200, seed=9)
    R = rqi.cholesky_R(A)
    x = rqi.csne_ls(A, b, R)
    ref = np.linalg.lstsq(A.to_dense(), b, rcond=None)[0]
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-12


def _check(res, sol, tol_s, tol_x):
    assert abs(res.sigma - sol.sigma) / sol.sigma < tol_s
    assert np.linalg.norm(res.x - sol.x) / np.linalg.norm(sol.x) < tol_x


def test_rqi_dense_small_workload():
    A, b, _ = tlsgen.dense_gaussian()
    sol = exact.svd_tls(A, b)
    res = rqi.rqi_pcgtls(A, b)
    _check(res, sol, 1e-12, 1e-12)
    assert res.psi[1] < res.psi[0]


@pytest.mark.parametrize("gen,kw", [
    ("paper_random", dict(patience=1)),
    ("paper_vanhuffel", dict(patience=1)),
    ("paper_delta", dict(patience=3)),
    ("paper_toeplitz", dict(patience=3)),
])
def test_rqi_paper_fixtures(gen, kw):
    A, b = getattr(tlsgen, gen)()
    sol = exact.svd_tls(A, b)
    res = rqi.rqi_pcgtls(A, b, **kw)
    bs, bx = certify.attainable(sol.sigma_1_Ab, sol.sigma, sol.kappa_tls)
    _check(res, sol, max(1e-12, 100 * bs), max(1e-11, 100 * bx))


def test_rqi_shift_clamp_recovers_smallest_root():
    # the Bjorck fixture starts with sigma_0^LS far above sigma'_n and a
    # tiny gap: unclamped RQI converges to another singular value
    A, b = tlsgen.paper_bjorck()
    sol = exact.svd_tls(A, b)
    wrong = rqi.rqi_pcgtls(A, b, patience=3, kmax=60)
    assert abs(wrong.sigma - sol.sigma) / sol.sigma > 0.1
    assert not certify.certify(A, b, wrong.x, wrong.sigma).smallest_root
    res = rqi.rqi_pcgtls(A, b, patience=3, kmax=60, shift_clamp=(0.9 * sol.sigma_n_A) ** 2)
    _check(res, sol, 1e-13, 1e-11)
    assert certify.certify(A, b, res.x, res.sigma).smallest_root


def test_ctilde_spectrum_interval():
    for gen in ("dense_gaussian", "paper_random", "paper_vanhuffel"):
        out = getattr(tlsgen, gen)()
        A, b = out[0], out[1]
        sol = exact.svd_tls(A, b)
        R = rqi.cholesky_R(A)
        Ri = np.linalg.inv(R)
        C = np.eye(R.shape[0]) - sol.sigma ** 2 * Ri.T @ Ri
        ev = np.linalg.eigvalsh(C)
        lo, hi = constraints.ctilde_interval(sol.sigma_n_A, sol.sigma)
        assert ev[0] >= lo - 1e-10 and ev[-1] <= hi + 1e-12
        assert abs(ev[0] - lo) < 1e-8     # attained at the last right singular vector of A


@pytest.mark.slow
def test_rqi_sparse_workload_certified():
    from oracle import polish
    A, b, _, _ = tlsgen.sparse_scaled()
    res = rqi.rqi_pcgtls(A, b, patience=2)
    sig_ld = polish.rayleigh_ld(A, b, res.x)
    c = certify.certify(A, b, res.x, sig_ld)
    assert c.normal_eq < 1e-13 and c.g_rel < 1e-15 and c.smallest_root
    assert abs(sig_ld - res.sigma) / sig_ld < 1e-9
