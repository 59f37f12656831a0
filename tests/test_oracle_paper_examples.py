"""The paper's five test problems (Section 4) through the oracle, plain
(FP64 factor and PCGTLS) against mixed precision (the scaled factor rounded
to FP16 as the library builds it, PCGTLS in u_p): the qualitative claims of
the examples.

- Mixed precision reaches the same limiting accuracy as the plain method
  (Examples 1, 2, 4, 5) and needs at least as many RQIs to get there.
- A u_p below FP32 limits the attainable accuracy (Example 3 reports
  rerrx of about 1e-4 with u_p = half).
- The stopping rule with >= (Example 2) stops no later than with >.

Stop rule: patience 3 (reading 5); the Björck problem starts above
sigma'_n and takes the shift clamp (reading 6). Iteration counts differ
from the paper's: its instances come from MATLAB's generator and its half
precision is simulated on a QR factor."""
import numpy as np
import pytest

import tlsgen
from oracle import exact, lowprec, qr, rqi

CASES = ["paper_random", "paper_delta", "paper_toeplitz", "paper_vanhuffel"]


def _problem(gen):
    out = getattr(tlsgen, gen)()
    A, b = out[0], out[1]
    return A, b, exact.svd_tls(A, b)


def _mp_factor(A, fmt="fp16"):
    Rh, d = lowprec.scaled_factor(A, fmt)
    return Rh * d[None, :]


def _first_within(res, ref, tol=1e-10):
    errs = [np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) for x in res.x_hist]
    return next((k + 1 for k, e in enumerate(errs) if e <= tol), None), min(errs)


@pytest.mark.parametrize("gen", CASES)
def test_mixed_reaches_plain_accuracy_with_more_rqis(gen):
    A, b, ref = _problem(gen)
    plain = rqi.rqi_pcgtls(A, b, rqi.cholesky_R(A), patience=3, kmax=60)
    mixed = rqi.rqi_pcgtls(A, b, _mp_factor(A), prec_p=np.float32, patience=3, kmax=60)
    kp, ep = _first_within(plain, ref)
    km, em = _first_within(mixed, ref)
    assert kp is not None and km is not None, (kp, km, ep, em)
    assert km >= kp
    assert em <= 100 * max(ep, 1e-15)


def test_bjorck_with_clamp_plain_converges():
    A, b, ref = _problem("paper_bjorck")
    sn = np.linalg.svd(A, compute_uv=False)[-1]
    plain = rqi.rqi_pcgtls(A, b, rqi.cholesky_R(A), patience=3, kmax=60, shift_clamp=0.9 * sn * sn)
    k, e = _first_within(plain, ref)
    assert k is not None and abs(plain.sigma - ref.sigma) / ref.sigma < 1e-12


@pytest.mark.parametrize("gen", ["paper_random", "paper_vanhuffel"])
def test_half_precision_pcgtls_limits_accuracy(gen):
    A, b, ref = _problem(gen)
    R = _mp_factor(A)
    single = rqi.rqi_pcgtls(A, b, R, prec_p=np.float32, patience=3, kmax=60)
    half = rqi.rqi_pcgtls(A, b, R, prec_p=np.float16, patience=3, kmax=60)
    _, e32 = _first_within(single, ref)
    _, e16 = _first_within(half, ref)
    assert e32 < 1e-12
    assert 1e-7 < e16 < 1e-2          # u_p = half stalls far above the FP32 limit


def test_ge_rule_stops_no_later():
    A, b, ref = _problem("paper_delta")
    R = _mp_factor(A)
    gt = rqi.rqi_pcgtls(A, b, R, prec_p=np.float32, patience=1, kmax=60)
    ge = rqi.rqi_pcgtls(A, b, R, prec_p=np.float32, patience=1, kmax=60, stop_ge=True)
    assert ge.iters <= gt.iters


@pytest.mark.parametrize("gen", CASES)
def test_qr_factor_plain_equals_cholesky_and_mixed_converges(gen):
    """Section 3: for full-rank A the R-factor of A equals the Cholesky
    factor of A^T A, so the plain runs take the same iterations; the mixed
    run with the FP16 QR factor reaches the plain accuracy with at least as
    many RQIs. On Van Huffel's problem the Cholesky factor needs no more RQIs
    than the QR factor (the paper sees Cholesky ahead there)."""
    A, b, ref = _problem(gen)
    chol = rqi.rqi_pcgtls(A, b, rqi.cholesky_R(A), patience=3, kmax=60)
    plain = rqi.rqi_pcgtls(A, b, qr.householder_r(A), patience=3, kmax=60)
    Rh, d = qr.scaled_qr_factor(A, "fp16")
    mixed = rqi.rqi_pcgtls(A, b, Rh * d[None, :], prec_p=np.float32, patience=3, kmax=60)
    kc, _ = _first_within(chol, ref)
    kp, ep = _first_within(plain, ref)
    km, em = _first_within(mixed, ref)
    assert kp == kc
    assert km is not None and km >= kp and em <= 100 * max(ep, 1e-15)
    if gen == "paper_vanhuffel":
        kmc, _ = _first_within(rqi.rqi_pcgtls(A, b, _mp_factor(A), prec_p=np.float32, patience=3,
                                              kmax=60), ref)
        assert kmc <= km
