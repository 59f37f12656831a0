"""Pins of oracle.exact: the TLS solution by its definitions.

The three routes (LAPACK SVD of [A,b], the same definition in 50-digit
mpmath, the secular equation from the Newton system) are checked against
each other and against instances whose answer is known in closed form.
"""
import numpy as np
import pytest

import tlsgen
from oracle import exact, certify


def _rand(m, n, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal((m, n)), g.standard_normal(m)


@pytest.mark.parametrize("m,n,seed", [(6, 2, 0), (12, 3, 1), (25, 4, 2), (40, 6, 3)])
def test_lapack_matches_mpmath_tiny(m, n, seed):
    A, b = _rand(m, n, seed)
    ref = exact.mp_svd_tls(A, b)
    s = exact.svd_tls(A, b)
    assert abs(s.sigma - ref.sigma) / ref.sigma < 1e-13
    assert np.linalg.norm(s.x - ref.x) / np.linalg.norm(ref.x) < 1e-12
    assert abs(s.sigma_n_A - ref.sigma_n_A) / ref.sigma_n_A < 1e-13


@pytest.mark.parametrize("m,n,seed", [(20, 3, 5), (300, 12, 6), (64, 30, 7)])
def test_planted_spectrum_closed_form(m, n, seed):
    # [A,b] = Y diag(sig) W^T, W = I - 2ww^T: sigma_{n+1} = min(sig) and
    # v = W e_{n+1} = e_{n+1} - 2 w w_{n+1}, so x = 2 w_{n+1} w_{1:n} / (1 - 2 w_{n+1}^2)
    sig = np.linspace(3.0, 1.0, n + 1)
    sig[-1] = 0.05
    A, b, sig, w = tlsgen.planted_svd(m, n, sig, seed=seed)
    x_planted = 2 * w[n] * w[:n] / (1 - 2 * w[n] ** 2)
    for route in (exact.svd_tls, exact.secular_tls):
        s = route(A, b)
        assert abs(s.sigma - 0.05) / 0.05 < 1e-13
        assert np.linalg.norm(s.x - x_planted) / np.linalg.norm(x_planted) < 1e-12


@pytest.mark.parametrize("gen", ["dense_gaussian", "paper_random", "paper_vanhuffel", "paper_delta"])
def test_secular_matches_svd(gen):
    out = getattr(tlsgen, gen)()
    A, b = out[0], out[1]
    s = exact.svd_tls(A, b)
    t = exact.secular_tls(A, b)
    bs, bx = certify.attainable(s.sigma_1_Ab, s.sigma, s.kappa_tls)
    assert abs(s.sigma - t.sigma) / s.sigma < max(1e-12, 50 * bs)
    assert np.linalg.norm(s.x - t.x) / np.linalg.norm(s.x) < max(1e-12, 50 * bx)


def test_normal_equation_identity_and_rq():
    A, b, _ = tlsgen.dense_gaussian()
    s = exact.svd_tls(A, b)
    c = certify.certify(A, b, s.x, s.sigma)
    assert c.normal_eq < 1e-14
    assert c.g_rel < 1e-15
    assert c.rq_rel < 1e-13
    assert c.smallest_root


def test_certificate_catches_wrong_root():
    # the second-smallest singular pair of [A,b] also solves f = g = 0 when
    # normalised, but it is not below sigma'_n: the Cholesky test must fail
    A, b, _ = tlsgen.dense_gaussian(60, 5, seed=11)
    C = np.column_stack([A, b])
    _, s, Vt = np.linalg.svd(C, full_matrices=False)
    v = Vt[-2]
    x = -v[:-1] / v[-1]
    c = certify.certify(A, b, x, s[-2])
    assert c.normal_eq < 1e-12
    assert not c.smallest_root


def test_existence_condition():
    for gen in ("dense_gaussian", "paper_random", "paper_vanhuffel"):
        out = getattr(tlsgen, gen)()
        s = exact.svd_tls(out[0], out[1])
        assert s.unique and certify.existence_margin(s.sigma_n_A, s.sigma) > 0
    # nonunique: orthonormal columns and b orthogonal to range(A) with the
    # same norm: all singular values of [A,b] equal sigma'_n
    A = np.zeros((5, 2))
    A[0, 0] = A[1, 1] = 1.0
    b = np.zeros(5)
    b[2] = 1.0
    s = np.linalg.svd(np.column_stack([A, b]), compute_uv=False)
    assert np.allclose(s, 1.0)
    with pytest.raises(ValueError):
        exact.secular_tls(A, b)


def test_minimal_correction():
    A, b, _ = tlsgen.dense_gaussian(50, 6, seed=3)
    s = exact.svd_tls(A, b)
    E, r = exact.tls_correction(A, b, s.x)
    assert abs(np.linalg.norm(np.column_stack([E, r])) - s.sigma) / s.sigma < 1e-12
    assert np.linalg.norm((A + E) @ s.x - (b + r)) < 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("rel_gap,seed", [(1e-3, 4001), (1e-2, 4003)])
def test_planted_gap_closed_form(rel_gap, seed):
    # the planted-gap construction and its closed form against the SVD of [A, b]
    A, b, x_t, lam, sn = tlsgen.planted_gap(m=4000, n=300, density=0.01, scale_decades=6.0,
                                            rel_gap=rel_gap, seed=seed)
    sig, x = exact.planted_gap_solution(A, x_t, lam)
    s = exact.svd_tls(A.to_dense(), b)
    bs, bx = certify.attainable(s.sigma_1_Ab, s.sigma, s.kappa_tls)
    assert abs(s.sigma - sig) / sig < max(1e-12, 10 * bs)
    assert np.linalg.norm(s.x - x) / np.linalg.norm(x) < max(1e-10, 10 * bx)
    gap = (s.sigma_n_A - s.sigma) / s.sigma_n_A
    assert 0.5 * rel_gap < gap < 2 * rel_gap
