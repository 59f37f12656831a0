"""Pins of the warm-start feature oracle (oracle.features)."""
import math

import numpy as np

import tlsgen
from oracle import features


def test_ritz_values_interlace_the_spectrum():
    # Cauchy interlacing: Ritz values of G^{-1} on a 2-D subspace lie in
    # [1/s_1^2, 1/s_n^2], and the largest one bounds 1/s_n^2 from below
    A, b, _ = tlsgen.dense_gaussian(200, 20, seed=1000)
    f, q = features.warm_features(A, b)
    s = np.linalg.svd(A, compute_uv=False)
    assert 1 / s[0] ** 2 * (1 - 1e-12) <= q["thmin"] <= q["thmax"] <= 1 / s[-1] ** 2 * (1 + 1e-12)
    # feature 11 = -ln(th_max)/2 >= ln sigma'_n
    assert f[11] >= math.log(s[-1]) - 1e-12


def test_exact_eigenvector_case():
    # A = U diag(s), b = A e_k + r_perp: x_0 = e_k is an eigenvector of A^T A,
    # so u_0 = e_k / s_k^2, both Ritz values collapse to 1/s_k^2 and
    # t = sigma_0^2 / (s_k^2 (1 + 1))
    g = np.random.default_rng(3)
    m, n, k = 50, 6, 2
    U, _ = np.linalg.qr(g.standard_normal((m, n + 1)))
    s = np.array([3.0, 2.0, 1.5, 1.0, 0.7, 0.5])
    A = U[:, :n] * s
    b = A[:, k] + 0.1 * U[:, n]
    f, q = features.warm_features(A, b)
    assert np.allclose(q["x0"], np.eye(n)[k], atol=1e-12)
    assert np.allclose(q["u0"], np.eye(n)[k] / s[k] ** 2, atol=1e-12)
    sig0 = 0.1 / math.sqrt(2.0)
    assert q["sigma0"] == pytest_approx(sig0)
    assert math.exp(f[9]) == pytest_approx(sig0 ** 2 / s[k] ** 2 / 2.0)
    assert math.exp(-2 * f[11]) == pytest_approx(1 / s[k] ** 2, rel=1e-6)


def pytest_approx(v, rel=1e-12):
    import pytest
    return pytest.approx(v, rel=rel)


def test_direct_identities():
    A, b, _ = tlsgen.dense_gaussian(120, 10, seed=1001)
    f, q = features.warm_features(A, b)
    assert f[0] == math.log(120) and f[1] == math.log(10)
    assert f[30] == 1.0 and f[31] >= math.log(1e-13)
    # sigma_0 of Algorithm 2's initial step
    r = b - A @ q["x0"]
    assert math.exp(f[5]) == pytest_approx(math.sqrt(r @ r / (1 + q["x0"] @ q["x0"])))
    # u_1 solves A^T A u_1 = u_0
    assert np.allclose(A.T @ (A @ q["u1"]), q["u0"], rtol=1e-10, atol=1e-14)
    # Cauchy-Schwarz makes features 22 and 23 non-negative
    assert f[23] >= -1e-12


def _exact_gap(A, b):
    from oracle import exact
    ref = exact.svd_tls(A, b)
    x0 = np.linalg.lstsq(A, b, rcond=None)[0]
    r = b - A @ x0
    s02 = r @ r / (1 + x0 @ x0)
    return 1 - ref.sigma ** 2 / s02


def test_gauss_gap_exact_when_the_krylov_space_is_everything():
    # n = 2: span{x_0, (A^T A)^{-1} x_0} is the whole space, so the two-point
    # Gauss rule integrates the quadratic form exactly and the secular
    # equation gives sigma_{n+1}^2 itself
    g = np.random.default_rng(7)
    for trial in range(5):
        A = g.standard_normal((30, 2)) * np.array([3.0, 0.5])
        b = A @ g.standard_normal(2) + 0.3 * g.standard_normal(30)
        f, _ = features.warm_features(A, b)
        assert math.exp(f[31]) == pytest_approx(_exact_gap(A, b), rel=1e-9)


def test_gauss_gap_exact_for_an_eigenvector_start():
    # b in span{A e_k} + range(A)^perp: one-point rule, exact
    g = np.random.default_rng(8)
    m, n, k = 40, 5, 3
    U, _ = np.linalg.qr(g.standard_normal((m, n + 1)))
    s = np.array([2.0, 1.7, 1.2, 0.9, 0.6])
    A = U[:, :n] * s
    b = 1.3 * A[:, k] + 0.2 * U[:, n]
    f, _ = features.warm_features(A, b)
    assert math.exp(f[31]) == pytest_approx(_exact_gap(A, b), rel=1e-9)


def test_gauss_gap_close_on_random_problems():
    # in general the rule is an approximation; on a Gaussian problem with a
    # moderate gap it is within a few percent of the exact gap
    A, b, _ = tlsgen.dense_gaussian(200, 20, seed=1000, noise_A=1e-3, noise_b=0.3)
    f, _ = features.warm_features(A, b)
    assert math.exp(f[31]) == pytest_approx(_exact_gap(A, b), rel=0.05)
