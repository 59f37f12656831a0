"""Pins of oracle.rqi: Algorithms 1-4 against facts fixed independently.

* Algorithm 2 with exact inner solves is inverse iteration on
  B = [A b]^T [A b] at the Rayleigh quotient shift, i.e. Algorithm 1,
  normalised to last component -1.
* Algorithm 3 at sigma = 0 returns R^{-1} R^{-T} f after one step (in
  float64 and, to float32 rounding, in float32); with l >= n steps it
  returns the dense solve of (A^T A - sigma^2 I) w = f. A right-hand side
  whose eta underflows to zero ends the loop without a 0/0.
* Algorithm 4 runs lines 1-5 in precision u: x_1 does not depend on u_p
  and equals x_0 + sigma_0^2 (A^T A)^{-1} x_0 solved by LU on the Gram
  matrix.
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
    # alpha_0 = eta_0 / delta_0 = 1 exactly (p_0 = s_0, C = I), so s_1 = 0
    # and eta_1 = 0 end the loop after one step
    assert tr.steps == 1 and tr.eta[1] == 0.0 and len(tr.delta) == 1


def test_pcgtls_fp32_sigma_zero_is_two_triangular_solves():
    # the same identity in float32: one step, and the result is R^{-1} R^{-T} f
    # to float32 rounding of two triangular solves (relative error of order
    # n u_32 kappa(R)^2; kappa(R) is small here)
    A, b, _ = tlsgen.dense_gaussian(60, 12, seed=7)
    R = rqi.cholesky_R(A)
    sR, sRT = rqi._tri_solvers(R, np.float32)
    f = np.random.default_rng(4).standard_normal(12)
    with np.errstate(all="raise"):
        w, tr = rqi.pcgtls(sR, sRT, 0.0, f, l=6, dtype=np.float32, trace=True)
    assert w.dtype == np.float32
    expect = sla.solve_triangular(R, sla.solve_triangular(R, f, trans="T"))
    kap = np.linalg.cond(R)
    u32 = 2.0 ** -24
    err = np.linalg.norm(w.astype(np.float64) - expect) / np.linalg.norm(expect)
    assert err <= 4 * 12 * u32 * kap ** 2, (err, kap)
    assert err > 0                                  # it did run in float32
    assert tr.steps == 1 and tr.eta[1] == 0.0


def test_pcgtls_eta_underflow_ends_without_nan():
    # R = 1e-3 I, f = 1e-27: in float32 s_0 = R^{-T} f = 1e-24 has squares
    # below the smallest subnormal, so eta_0 = 0 while s_0 != 0, and
    # q_0 = R^{-1} p_0 = 1e-21 gives delta_0 = -sigma^2 ||q_0||^2, a nonzero
    # subnormal. Run as printed, alpha_0 = -0, eta_1 = 0 and beta_0 = 0/0 is
    # NaN. With the eta check the loop ends at once and returns omega = 0,
    # the initial iterate.
    n = 8
    R = 1e-3 * np.eye(n)
    sR, sRT = rqi._tri_solvers(R, np.float32)
    f = np.full(n, 1e-27)
    q0 = np.float32(1e-21)
    assert np.float32(1e-24) ** 2 == 0 and n * q0 * q0 > 0   # the premise, in float32
    with np.errstate(divide="raise", invalid="raise"):
        w, tr = rqi.pcgtls(sR, sRT, 0.5, f, l=4, dtype=np.float32, trace=True)
    assert np.all(w == 0) and tr.steps == 0 and tr.eta == [0.0] and tr.delta == []
    # in float64 the same right-hand side is an ordinary solve: C = I - 0.5e6 I
    # is negative definite, so one step along p_0 solves it (delta_0 < 0)
    w64, tr64 = rqi.pcgtls(*rqi._tri_solvers(R), 0.5, f, l=4, trace=True)
    ref = np.linalg.solve(R.T @ R - 0.5 * np.eye(n), f)
    assert np.allclose(w64, ref, rtol=1e-12, atol=0) and tr64.negatives >= 1


def test_pcgtls_nonfinite_delta_ends_before_the_update():
    # sigma^2 so large that ||q||^2 sigma^2 overflows float32: delta_0 = -inf,
    # the step must not run (it would put NaN into omega)
    n = 4
    R = 1e-20 * np.eye(n)
    sR, sRT = rqi._tri_solvers(R, np.float32)
    with np.errstate(all="ignore"):
        w, tr = rqi.pcgtls(sR, sRT, 1e30, np.ones(n), l=3, dtype=np.float32, trace=True)
    assert np.all(w == 0) and tr.steps == 0 and len(tr.delta) == 1
    assert not np.isfinite(tr.delta[0])


@pytest.mark.parametrize("prec_p", [np.float32, np.float16])
def test_mixed_first_step_is_in_working_precision(prec_p):
    # Algorithm 4, line 5: A^T A u_0 = x_0 is solved in u, so the first
    # iterate x_1 = x_0 + sigma_0^2 u_0 is the same for every u_p; it is
    # checked here against the textbook step with an LU solve on A^T A
    A, b, _ = tlsgen.dense_gaussian(120, 10, seed=12)
    R = rqi.cholesky_R(A)
    plain = rqi.rqi_pcgtls(A, b, R, kmax=2, patience=5)
    mixed = rqi.rqi_pcgtls(A, b, R, kmax=2, patience=5, prec_p=prec_p)
    assert np.array_equal(plain.x_hist[0], mixed.x_hist[0])
    x0 = rqi.csne_ls(A, b, R)
    r0 = b - A @ x0
    sig0 = r0 @ r0 / (1 + x0 @ x0)
    x1 = x0 + sig0 * np.linalg.solve(A.T @ A, x0)
    assert np.linalg.norm(mixed.x_hist[0] - x1) / np.linalg.norm(x1) < 1e-13


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


def test_psi_at_closed_form_and_solution():
    # A = [I_n; 0], b = beta e_{n+1} (orthogonal to range(A)): at x = t e_1,
    # r = b - t e_1, sigma^2 = (beta^2 + t^2)/(1 + t^2), f = t (1 - sigma^2) e_1,
    # g = sigma^2 - beta^2 (eq. 2), so psi^2 = (t^2 (1 - s2)^2 + (s2 - beta^2)^2)/(1 + t^2)
    n, m, beta = 4, 7, 0.3
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = 1.0
    b = np.zeros(m)
    b[n] = beta
    for t in (0.0, 0.2, -1.5):
        x = np.zeros(n)
        x[0] = t
        s2 = (beta * beta + t * t) / (1 + t * t)
        want = math.sqrt((t * t * (1 - s2) ** 2 + (s2 - beta * beta) ** 2) / (1 + t * t))
        assert rqi.psi_at(A, b, x) == pytest.approx(want, rel=1e-14, abs=1e-300)
    # at the TLS solution of a generic problem f = g = 0: psi is at rounding level
    A, b, _ = tlsgen.dense_gaussian(80, 6, seed=3)
    ref = exact.svd_tls(A, b)
    assert rqi.psi_at(A, b, ref.x) < 1e-13 * np.linalg.norm(A) ** 2
    assert rqi.psi_at(A, b, ref.x + 1e-3) > 1e-6


def test_warm_candidate_truncates_the_shifted_solve():
    # with the exact factor, x_1w differs from x_0 + lam (A^T A - lam I)^{-1} x_0
    # by the Neumann tail sum_{k>=3} lam^k M^k x_0, M = (A^T A)^{-1}
    A, b, _ = tlsgen.dense_gaussian(60, 5, seed=11, noise_b=0.3)
    R = rqi.cholesky_R(A)
    x0 = rqi.x_ls(A, b, R, 2)
    G = A.T @ A
    mu = 1.0 / np.linalg.eigvalsh(G)[0]               # ||M||_2
    r0 = b - A @ x0
    s0 = math.sqrt(float(r0 @ r0) / (1 + x0 @ x0))
    for frac in (0.3, 0.9):
        sh = frac * s0
        lam = sh * sh
        xk, taken, pw, pp, used = rqi.warm_candidate(A, b, R, x0, sh)
        assert used == sh
        xw = x0 + lam * np.linalg.solve(G, x0) + lam * lam * np.linalg.solve(G, np.linalg.solve(G, x0))
        exact_step = x0 + lam * np.linalg.solve(G - lam * np.eye(5), x0)
        tail = (lam * mu) ** 3 / (1 - lam * mu) * np.linalg.norm(x0)
        assert np.linalg.norm(xw - exact_step) <= tail * (1 + 1e-9)
        assert pw == pytest.approx(rqi.psi_at(A, b, xw), rel=1e-12)
        # the kept start is the one with the smaller psi
        xp = x0 + s0 * s0 * np.linalg.solve(G, x0)
        assert pp == pytest.approx(rqi.psi_at(A, b, xp), rel=1e-12)
        assert taken == (pw < pp)
        assert np.allclose(xk, xw if taken else xp, rtol=1e-12, atol=0)
    # a hint above sigma_0 is capped at sigma_0; a zero hint leaves x_0
    assert rqi.warm_candidate(A, b, R, x0, 10 * s0)[4] == s0
    xk, taken, pw, pp, used = rqi.warm_candidate(A, b, R, x0, 0.0)
    assert pw == pytest.approx(rqi.psi_at(A, b, x0), rel=1e-14)


@pytest.mark.parametrize("tie", [1.0, 4.0])
def test_returned_iterate_rule(tie):
    """The returned iterate is the latest x_k with psi_k within the factor
    psi_tie of the smallest psi before it (k = 1 always); with a patience of
    3 on a paper fixture the run goes past the float64 floor, where several
    iterates qualify, and every one of them is a converged iterate: the
    returned x matches the SVD solution to the attainable accuracy."""
    A, b = tlsgen.paper_random()[:2]
    ref = exact.svd_tls(A, b)
    o = rqi.rqi_pcgtls(A, b, patience=3, kmax=30, psi_tie=tie)
    psi = o.psi
    kept = [k for k in range(1, o.iters + 1) if k == 1 or psi[k - 1] <= tie * min(psi[: k - 1])]
    assert o.k_best == kept[-1]
    assert np.array_equal(o.x, o.x_hist[o.k_best - 1])
    # never before the last iterate that attained the minimum
    assert o.k_best >= max(k for k in range(1, o.iters + 1) if psi[k - 1] == min(psi))
    bs, bx = certify.attainable(ref.sigma_1_Ab, ref.sigma, ref.kappa_tls)
    assert np.linalg.norm(o.x - ref.x) / np.linalg.norm(ref.x) < max(1e-12, 100 * bx)
    with pytest.raises(ValueError):
        rqi.rqi_pcgtls(A, b, psi_tie=0.5)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_pcgtls_precision_floor_exit(dtype):
    """The loop stops before step j > 0 once eta_j <= u_p^2 eta_0: on a
    well-preconditioned shifted system (sigma far below sigma'_n) that
    happens after a few steps, and the steps it skips change omega by no
    more than the working precision (the run without the test, to l = 40,
    agrees to a few u_p)."""
    A, b, _ = tlsgen.dense_gaussian(600, 60, seed=11)
    R = rqi.cholesky_R(A)
    sR, sRT = rqi._tri_solvers(R, dtype)
    s_n = np.linalg.svd(A, compute_uv=False)[-1]
    f = np.random.default_rng(5).standard_normal(60)
    w, t = rqi.pcgtls(sR, sRT, (0.3 * s_n) ** 2, f.astype(dtype), 40, dtype=dtype, trace=True)
    w0, t0 = rqi.pcgtls(sR, sRT, (0.3 * s_n) ** 2, f.astype(dtype), 40, dtype=dtype, trace=True, eta_floor=0.0)
    u = float(np.finfo(dtype).eps) / 2
    assert t.steps < t0.steps
    assert t.eta[t.steps] <= u * u * t.eta[0] < t.eta[t.steps - 1]
    assert np.linalg.norm(w.astype(np.float64) - w0) <= 20 * u * np.linalg.norm(w0)
