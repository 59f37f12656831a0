"""GPU parity of the full RQI-PCGTLS solve (tls_rqi_solve) against the
oracle's definition of the answer (SVD of [A, b], long-double Rayleigh
quotient)."""
import numpy as np
import pytest

import tlsgen
from oracle import exact, certify, polish, rqi

pytestmark = pytest.mark.gpu


def _tls():
    from paper_2305_19028_amd import tls
    return tls


def _errs(x, sigma, ref):
    return abs(sigma - ref.sigma) / ref.sigma, np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)


@pytest.mark.parametrize("gen,kw", [
    ("dense_gaussian", {}),
    ("paper_random", {}),
    ("paper_vanhuffel", {}),
    ("paper_delta", {"stop_patience": 3}),
    ("paper_toeplitz", {"stop_patience": 3}),
])
def test_rqi_fp64_small(gen, kw):
    tls = _tls()
    print(f"rqi fp64 {gen}", flush=True)
    out = getattr(tlsgen, gen)()
    A, b = out[0], out[1]
    ref = exact.svd_tls(A, b)
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    x, sigma, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(**kw))
    es, ex = _errs(x.cpu().numpy(), sigma, ref)
    bs, bx = certify.attainable(ref.sigma_1_Ab, ref.sigma, ref.kappa_tls)
    assert es < max(1e-10, 100 * bs), (es, st)
    assert ex < max(1e-10, 100 * bx), (ex, st)


def test_rqi_fp64_matches_oracle_iterates():
    # same algorithm, same readings: the psi sequences agree
    tls = _tls()
    A, b, _ = tlsgen.dense_gaussian()
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    x, sigma, st = tls.tls_rqi_solve(Ad, b, P)
    o = rqi.rqi_pcgtls(A, b)
    assert st["iters"] == o.iters and st["k_best"] == o.k_best
    for a, c in zip(st["psi"][:2], o.psi[:2]):
        assert abs(a - c) <= 1e-6 * c


def test_rqi_sparse_small():
    tls = _tls()
    A, b, _, _ = tlsgen.sparse_scaled(4000, 300, density=0.01, seed=77)
    ref_rqi = rqi.rqi_pcgtls(A, b, patience=2)
    sig_ref = polish.rayleigh_ld(A, b, ref_rqi.x)
    Ad = tls.from_tlsgen(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    x, sigma, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(stop_patience=2))
    x = x.cpu().numpy()
    assert abs(sigma - sig_ref) / sig_ref < 1e-10
    assert np.linalg.norm(x - ref_rqi.x) / np.linalg.norm(ref_rqi.x) < 1e-10
