"""Pins of the oracle's Householder QR preconditioner (oracle.qr) against
facts that do not come from it: LAPACK's R (through numpy), the Cholesky
factor of A^T A (equal to R for full-rank A, Section 3), closed forms for
one and two columns, the row-permutation invariance and stacking identity
that a tree (TSQR) reduction relies on, and the Section 3.1 bounds for the
factor computed in fp16 / bf16."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import lowprec, qr

U = {"fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


def _sign_fix(R):
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return R * s[:, None]


def _graded(m, n, kappa, seed):
    rng = np.random.default_rng(seed)
    U_, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.geomspace(1.0, 1.0 / kappa, n)
    return (U_ * s) @ V.T


@pytest.mark.parametrize("m,n,seed", [(7, 3, 0), (40, 40, 1), (300, 57, 2), (129, 64, 3)])
def test_matches_lapack_r(m, n, seed):
    A = np.random.default_rng(seed).standard_normal((m, n)) * np.geomspace(1, 1e3, n)
    R = qr.householder_r(A)
    Rl = _sign_fix(np.linalg.qr(A, mode="r"))
    assert np.allclose(np.tril(R, -1), 0)
    assert np.all(np.diag(R) > 0)
    assert np.linalg.norm(R - Rl) <= 1e-13 * np.linalg.norm(Rl)


def test_equals_cholesky_of_gram():
    A = _graded(200, 30, 1e2, 4)
    R = qr.householder_r(A)
    C = sla.cholesky(A.T @ A, lower=False)
    assert np.linalg.norm(R - C) <= 1e-11 * np.linalg.norm(C)


def test_closed_forms():
    a = np.array([[3.0], [4.0], [0.0]])
    assert qr.householder_r(a)[0, 0] == pytest.approx(5.0, rel=1e-15)
    A = np.array([[1.0, 2.0], [2.0, 0.0], [2.0, 1.0]])
    a1, a2 = A[:, 0], A[:, 1]
    r11 = np.linalg.norm(a1)
    r12 = a1 @ a2 / r11
    r22 = np.sqrt(a2 @ a2 - r12 * r12)
    assert np.allclose(qr.householder_r(A), [[r11, r12], [0.0, r22]], rtol=1e-14, atol=1e-15)
    # a column already zero below the diagonal, and a negative pivot
    B = np.array([[-2.0, 1.0], [0.0, 3.0], [0.0, 4.0]])
    assert np.allclose(qr.householder_r(B), [[2.0, -1.0], [0.0, 5.0]], rtol=1e-15)


def test_row_permutation_and_stacking():
    rng = np.random.default_rng(5)
    A = rng.standard_normal((260, 20))
    R = qr.householder_r(A)
    assert np.allclose(qr.householder_r(A[rng.permutation(260)]), R, rtol=1e-12, atol=1e-12)
    # tree reduction: R of the stacked R-factors of row blocks is R(A),
    # also with a block of fewer rows than columns
    parts = [A[:100], A[100:250], A[250:]]
    tops = [qr.householder_r(p) if p.shape[0] >= 20 else p for p in parts]
    assert np.allclose(qr.householder_r(np.vstack(tops)), R, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
@pytest.mark.parametrize("kappa", [10.0, 200.0])
def test_low_precision_bounds(fmt, kappa):
    m, n = 240, 24
    A = _graded(m, n, kappa, 6) * np.geomspace(1.0, 1e4, n)   # column scales over 4 decades
    Rh, d = qr.scaled_qr_factor(A, fmt)
    Ah = lowprec.round_to(A / d, fmt)
    u = U[fmt]
    # backward error (Section 3.1): R^T R - A^T A = A^T dA + dA^T A + dA^T dA
    rel = np.linalg.norm(Rh.T @ Rh - Ah.T @ Ah) / np.linalg.norm(Ah) ** 2
    assert 0.01 * u < rel < 2 * m * n * u
    # the computed factor is nonsingular and A-hat R_hat^{-1} = Q_1 - dA
    # R_hat^{-1} has singular values within 1 +- ||dA|| ||R_hat^{-1}||, of
    # order u kappa_F(A-hat): linear in kappa (constraint (5)), where a
    # factor of fl(A^T A) would deviate by u kappa^2. Measured: about
    # 0.07 u kappa_F at both condition numbers
    sv = np.linalg.svd(Ah, compute_uv=False)
    kF = np.linalg.norm(Ah) / sv[-1]
    s = np.linalg.svd(sla.solve_triangular(Rh, Ah.T, trans="T", lower=False).T, compute_uv=False)
    dev = max(abs(s[0] - 1.0), abs(s[-1] - 1.0))
    assert 0.005 * u * kF < dev <= u * kF
    # the factor differs from R(A D^{-1}) in fp64 by the same order
    R64 = qr.householder_r(A / d)
    assert np.linalg.norm(Rh - R64) <= u * kF * np.linalg.norm(R64)


def test_low_precision_rounds_stored_values():
    A = _graded(120, 16, 30.0, 7)
    Rh, _ = qr.scaled_qr_factor(A, "fp16")
    assert np.array_equal(lowprec.round_to(Rh, "fp16"), Rh)
    # every stored quantity of the fp16 run is an fp16 value, so the factor
    # differs from the one computed in fp64 on the same rounded input
    Rx = qr.householder_r(lowprec.round_to(A / lowprec.column_norms(A), "fp16"))
    assert not np.array_equal(lowprec.round_to(Rx, "fp16"), Rx)
    assert not np.array_equal(Rx, Rh)
