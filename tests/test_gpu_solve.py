"""GPU parity of the full RQI-PCGTLS solve (tls_rqi_solve) against the
oracle's definition of the answer (SVD of [A, b], long-double Rayleigh
quotient)."""
import math

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
    # psi_1 is far above the rounding floor: both implementations agree on it;
    # later psi sit at the float64 floor (~1e-14) where the stop iteration is
    # decided by rounding noise
    assert abs(st["psi"][0] - o.psi[0]) <= 1e-2 * o.psi[0]
    assert abs(st["iters"] - o.iters) <= 2
    assert max(st["psi"][1:]) < 1e-12 and max(o.psi[1:]) < 1e-12


def _iterate_cases():
    return {
        "dense_200x20": lambda: tlsgen.dense_gaussian(200, 20, seed=1000)[:2],
        "dense_2000x150": lambda: tlsgen.dense_gaussian(2000, 150, seed=31)[:2],
        "sparse_4000x300": lambda: tlsgen.sparse_scaled(4000, 300, density=0.01, seed=77)[:2],
        "paper_random": lambda: tlsgen.paper_random()[:2],
        "paper_vanhuffel": lambda: tlsgen.paper_vanhuffel()[:2],
    }


@pytest.mark.parametrize("case", list(_iterate_cases()))
def test_rqi_fp64_iterates_match_oracle(case):
    """The plain FP64 path and the oracle run the same algorithm (Algorithms
    2 and 3 with l = k, the same x_LS, the same initial step) on the same
    data, so their iterates differ only by rounding: x_k agrees element by
    element to 1e-11 relative to ||x_k|| at every iterate both computed.
    sigma_k and psi_k come from r = b - A x, whose float64 rounding error is
    about u (||b|| + ||A||_F ||x||) (the Rayleigh quotient's attainable
    accuracy, u sigma_1 / sigma): sigma_k agrees to 30 times that relative
    to ||r_k|| (and to 1e-12 at least), psi_k to 1e-6 relative or ten times
    its own rounding level u ||A||_F (||b|| + ||A||_F ||x||)."""
    import torch
    tls = _tls()
    A, b = _iterate_cases()[case]()
    print(f"iterates {case}", flush=True)
    Ad = tls.from_tlsgen(A)
    n = Ad.n
    snaps = torch.zeros((40, n), dtype=torch.float64, device="cuda")
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    x, sigma, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(stop_patience=2, kmax=40, x_snapshots=snaps))
    o = rqi.rqi_pcgtls(A, b, patience=2, kmax=40)
    xs = snaps[: st["iters"]].cpu().numpy()
    kk = min(st["iters"], o.iters)
    nA = math.sqrt(float(np.sum(A.val ** 2)) if hasattr(A, "val") else float(np.sum(A * A)))
    nb = float(np.linalg.norm(b))
    u = 2.0 ** -53
    for k in range(kk):
        xo = o.x_hist[k]
        nx = float(np.linalg.norm(xo))
        dx = np.linalg.norm(xs[k] - xo) / nx
        ds = abs(st["sigma"][k] - o.sigma_hist[k]) / o.sigma_hist[k]
        rnorm = o.sigma_hist[k] * math.sqrt(1 + nx * nx)
        tol_s = max(1e-12, 30 * u * (nb + nA * nx) / rnorm)
        psi_floor = u * nA * (nb + nA * nx)
        print(f"k={k + 1}: x {dx:.2e} sigma {ds:.2e} (tol {tol_s:.1e}) psi {st['psi'][k]:.3e} / "
              f"{o.psi[k]:.3e} (floor {psi_floor:.1e})", flush=True)
        assert dx <= 1e-11, (k, dx)
        assert ds <= tol_s, (k, ds, tol_s)
        assert abs(st["psi"][k] - o.psi[k]) <= max(1e-6 * o.psi[k], 10 * psi_floor), (k, st["psi"][k], o.psi[k])
    assert kk >= 2


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


@pytest.mark.parametrize("u_q", ["fp32", "fp16", "bf16"])
def test_rqi_mixed_small(u_q):
    # RQI-PCGTLS-MP: factor in u_q, PCGTLS in FP32, outer loop in FP64; the
    # fixed point is the FP64 TLS solution
    tls = _tls()
    print(f"rqi mixed {u_q}", flush=True)
    A, b, _ = tlsgen.dense_gaussian(2000, 150, seed=31)
    ref = exact.svd_tls(A, b)
    Ad = tls.dense(A)
    P, rep = tls.tls_factor_precond(Ad, u_q)
    x, sigma, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(u_p="fp32", stop_patience=2))
    es, ex = _errs(x.cpu().numpy(), sigma, ref)
    assert es < 1e-10 and ex < 1e-10, (es, ex, st["iters"])
