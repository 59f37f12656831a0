"""Dense path on the matrix cores: the MFMA Gram (FP64, FP32, FP16, BF16
inputs) against the oracle, and full-size dense solves (65536 x 4096) with
answers fixed by a planted SVD and by the normal-equation identity."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import tlsgen
from oracle import lowprec

pytestmark = pytest.mark.gpu


def _tls():
    from paper_2305_19028_amd import tls
    return tls


@pytest.mark.parametrize("u_q", ["fp64", "fp32", "fp16", "bf16"])
@pytest.mark.parametrize("shape", [(3000, 300), (4097, 129), (300, 64), (20000, 200)])
def test_gram_tiles_against_oracle(u_q, shape):
    """Several 128 x 128 Gram tiles, ragged m (partial K chunk) and ragged n
    (partial tile): R^T R of the stored factor against the Gram matrix of the
    oracle's rounding of A D^{-1}."""
    tls = _tls()
    m, n = shape
    print(f"gram {u_q} {shape}", flush=True)
    A, b, _ = tlsgen.dense_gaussian(m, n, seed=31 + n)
    P, rep = tls.tls_factor_precond(tls.dense(A), u_q)
    Rh, d = tls.tls_precond_export(P)
    Ah = A / d if u_q == "fp64" else lowprec.round_to(A * (1.0 / d), u_q)
    H = Ah.T @ Ah
    if u_q == "fp64":
        assert np.max(np.abs(Rh - sla.cholesky(H, lower=False))) < 1e-11
        return
    u = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}[u_q]
    # FP32 products; FP32 sums over 32-row chunks folded into FP64 (FP32
    # inputs) or over 8192-row segments added in FP64 (FP16 / BF16 inputs;
    # 20000 rows: three segments, the last ragged); Cholesky in FP32, factor
    # stored in u_q: the storage rounding dominates
    err = np.linalg.norm(Rh.T @ Rh - H, 2) / np.linalg.norm(H, 2)
    assert err < 30 * u, err
    assert np.array_equal(Rh, np.triu(lowprec.round_to(Rh, u_q)))


@pytest.mark.parametrize("u_q", ["fp64", "fp32", "fp16", "bf16", "bf16x3"])
@pytest.mark.parametrize("shape", [(70, 3), (300, 64), (3000, 300), (4097, 129), (9000, 520),
                                   (20000, 200), (40000, 700)])
def test_gram_elementwise_against_oracle(u_q, shape):
    """The Gram step alone (tls_gram) against the oracle's Gram matrix of its
    own rounding of A D^{-1}, entry by entry. The 16-bit products are exact
    in FP32; what remains is the FP32 accumulation (the matrix cores' sums
    restarted every 128 rows, at most a few dozen FP32 additions per entry
    over a segment) and the final FP32 rounding, so every entry is within
    100 u_32 of the oracle's, relative to (|Ahat|^T |Ahat|)_ij. Shapes cover
    ragged m (partial 64-row chunks), ragged n (partial 128-column tiles), an
    odd number of tile columns (a pair whose second tile is below the
    diagonal or past the last column) and several row segments."""
    tls = _tls()
    m, n = shape
    print(f"gram elementwise {u_q} {shape}", flush=True)
    A, _, _ = tlsgen.dense_gaussian(m, n, seed=7 + n)
    A = A * np.exp(np.random.default_rng(n).uniform(-3, 3, n))      # spread column scales
    G, d = tls.tls_gram(tls.dense(A), u_q)
    G = G.cpu().numpy()
    d = d.cpu().numpy()
    d_or = np.linalg.norm(A, axis=0)
    assert np.allclose(d, d_or, rtol=1e-14, atol=0)
    if u_q == "bf16x3":
        # the split pair: hi^T hi + hi^T lo + lo^T hi in three BF16 products
        hi, lo = lowprec.split_bf16(A * (1.0 / d_or))
        H = lowprec.split_gram(hi, lo)
        W = lowprec.split_gram(np.abs(hi), np.abs(lo))
        # and within 3 2^-16 of the Gram matrix of A D^{-1} itself
        As = A * (1.0 / d_or)
        Wa = np.abs(As).T @ np.abs(As)
        iu = np.triu_indices(n)
        assert np.all(np.abs(G[iu] - (As.T @ As)[iu]) <= (3 * 2.0 ** -16 + 200 * 2.0 ** -24) * Wa[iu])
    else:
        Ah = A * (1.0 / d_or) if u_q == "fp64" else lowprec.round_to(A * (1.0 / d_or), u_q)
        H = Ah.T @ Ah
        W = np.abs(Ah).T @ np.abs(Ah)
    iu = np.triu_indices(n)
    u = 2.0 ** -53 if u_q == "fp64" else 2.0 ** -24
    k = 4 * np.sqrt(m) if u_q == "fp64" else 100.0
    err = np.abs(G[iu] - H[iu]) / W[iu]
    assert np.max(err) <= k * u, (np.max(err) / u, np.unravel_index(np.argmax(err), err.shape))
    assert np.all(np.tril(G, -1) == 0)


def _planted_c3(seed=3100):
    # the configuration's spectrum: sigma'_i geometric from 1 to 1e-3, and a
    # planted smallest singular value of [A, b] at 3.9e-5
    m, n = 65536, 4096
    s = np.concatenate([1e-3 ** (np.arange(n) / (n - 1)), [3.9e-5]])
    A, b, sig, w = tlsgen.planted_svd(m, n, s, seed=seed)
    x = 2 * w[n] * w[:n] / (1 - 2 * w[n] ** 2)    # x_TLS = -v_{1:n}/v_{n+1}, v = (I - 2ww^T) e_{n+1}
    return A, b, float(s[n]), x


@pytest.fixture(scope="module")
def planted():
    print("planted 65536 x 4096: generating", flush=True)
    return _planted_c3()


def test_c3_planted_fp64(planted):
    tls = _tls()
    A, b, sig, x = planted
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    xs, s, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(stop_patience=2))
    es = abs(s - sig) / sig
    ex = np.linalg.norm(xs.cpu().numpy() - x) / np.linalg.norm(x)
    print(f"fp64: sigma {es:.2e} x {ex:.2e} iters {st['iters']}", flush=True)
    # attainable: u sigma_1 / sigma_{n+1} ~ 3e-12, u kappa_TLS ~ 1e-13
    assert es < 1e-10 and ex < 1e-10


@pytest.mark.parametrize("u_q", ["fp16", "bf16"])
def test_c3_planted_mixed_gate_escalates(planted, u_q):
    """FP16 or BF16 requested with the gate on: the factor that is used
    carries the a-posteriori certificate (Ritz values of R^{-T} A^T A R^{-1}
    within [1/2, 3/2]; escalation if the requested one had failed), and the
    answer meets 1e-10."""
    tls = _tls()
    A, b, sig, x = planted
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, u_q)
    opts = tls.default_opts(u_p="fp32", gate_enforce=1, allow_escalate=1, stop_patience=2,
                            refine_sweeps=1)
    xs, s, st = tls.tls_rqi_solve(Ad, b, P, opts)
    g = P.info()["gate"]
    es = abs(s - sig) / sig
    ex = np.linalg.norm(xs.cpu().numpy() - x) / np.linalg.norm(x)
    print(f"mixed: used {g['used']} escalations {g['escalations']} quality "
          f"[{g['quality_lo']:.3g}, {g['quality_hi']:.3g}] sigma {es:.2e} x {ex:.2e}", flush=True)
    if g["used"] != tls.PREC["fp64"]:
        assert g["verdict"] & 16 and 0.5 <= g["quality_lo"] and g["quality_hi"] <= 1.5
    assert g["used"] == tls.PREC[u_q] or g["escalations"] >= 1
    assert es < 1e-10 and ex < 1e-10


def test_c3_reflector_fp64_normal_equations():
    """The configuration's own generator (with the 1e-5 perturbation, no
    closed form): the FP64 answer satisfies (A^T A - sigma^2 I) x = A^T b and
    sigma^2 = ||b - A x||^2 / (1 + ||x||^2) to rounding."""
    tls = _tls()
    print("reflector 65536 x 4096: generating", flush=True)
    A, b, _, _ = tlsgen.reflector_dense(65536, 4096)
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    xs, s, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(stop_patience=2))
    x = xs.cpu().numpy()
    r = b - A @ x
    res = A.T @ (A @ x) - s * s * x - A.T @ b
    scale = np.linalg.norm(A.T @ (A @ x)) + np.linalg.norm(A.T @ b)
    assert np.linalg.norm(res) / scale < 1e-11
    assert abs(s * s - (r @ r) / (1 + x @ x)) / (s * s) < 1e-9


@pytest.fixture(scope="module")
def reflector():
    import json
    import os
    print("reflector 65536 x 4096 (seed 3000): generating", flush=True)
    A, b, _, _ = tlsgen.reflector_dense(65536, 4096, seed=3000)
    with open(os.path.join(os.path.dirname(__file__), "golden", "dense_c3_ref.json")) as f:
        ref = json.load(f)
    return A, b, ref


@pytest.mark.parametrize("u_q", ["fp64", "bf16", "fp16", "bf16x3"])
def test_c3_reflector_against_oracle(reflector, u_q):
    """The configured dense workload (its own generator, with the 1e-5
    perturbation of A) through the paths the benchmark times: FP64, and the
    BF16, FP16 and split-BF16 factors with FP32 PCGTLS, the gate and the
    refinement. Against the stored oracle answer (plain float64 RQI-PCGTLS
    with long-double Newton polish): x and sigma within 1e-10 relative (the
    attainable float64 accuracy is u kappa_TLS = 1.2e-13 for x and
    u sigma_1([A,b]) / sigma = 4.8e-11 for sigma, both recorded with the
    reference); the factor that was used carries the certificate."""
    tls = _tls()
    A, b, ref = reflector
    print(f"c3 reflector {u_q}", flush=True)
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, u_q)
    if u_q == "fp64":
        opts = tls.default_opts(stop_patience=2)
    else:
        opts = tls.default_opts(u_p="fp32", gate_enforce=1, allow_escalate=1, stop_patience=2,
                                refine_sweeps=1)
    xs, s, st = tls.tls_rqi_solve(Ad, tls.device_vector(b), P, opts)
    xr = np.array(ref["x"])
    ex = np.linalg.norm(xs.cpu().numpy() - xr) / np.linalg.norm(xr)
    es = abs(s - ref["sigma"]) / ref["sigma"]
    g = P.info()["gate"]
    print(f"{u_q}: iters {st['iters']} sigma {es:.2e} x {ex:.2e} used {g['used']} "
          f"quality [{g['quality_lo']:.4g}, {g['quality_hi']:.4g}]", flush=True)
    assert ref["bounds"]["attainable_x"] < 1e-11 and ref["bounds"]["attainable_sigma"] < 1e-10
    assert ex < 1e-10 and es < 1e-10
    if u_q != "fp64":
        assert g["used"] == tls.PREC[u_q]
        assert g["verdict"] & 16 and 0.5 <= g["quality_lo"] and g["quality_hi"] <= 1.5
