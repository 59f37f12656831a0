"""GPU parity of the warm-start network kernels and of the warm start in the
solve, against the float64 oracle (oracle.mlp, oracle.features)."""
import math

import numpy as np
import pytest

import tlsgen
from oracle import exact, features, mlp, rqi

pytestmark = pytest.mark.gpu


def _tls():
    from paper_2305_19028_amd import tls
    return tls


def _dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("B", [1, 37, 300])
def test_forward_matches_oracle(B):
    tls = _tls()
    print(f"mlp forward B={B}", flush=True)
    th = tlsgen.mlp_init(1)
    X, _, norm = tlsgen.mlp_batch(B, seed=2)
    y = tls.tls_mlp_forward(_dev(th), _dev(norm), _dev(X)).cpu().numpy()
    yo, _ = mlp.forward(th.astype(np.float64), X, norm)
    # FP32 through four layers of at most 256-term dot products
    assert np.max(np.abs(y - yo)) <= 2e-5 * (1 + np.max(np.abs(yo)))


@pytest.mark.parametrize("B", [2, 37, 300])
def test_loss_and_gradient_match_oracle(B):
    tls = _tls()
    print(f"mlp grad B={B}", flush=True)
    th = tlsgen.mlp_init(3)
    X, t, norm = tlsgen.mlp_batch(B, seed=4)
    loss, g = tls.tls_mlp_loss_grad(_dev(th), _dev(norm), _dev(X), _dev(t))
    lo, go = mlp.loss_grad(th.astype(np.float64), X, t, norm)
    g = g.cpu().numpy().astype(np.float64)
    assert abs(float(loss.cpu()) - lo) <= 1e-5 * lo
    # every layer's weight and bias block agrees in the relative 2-norm
    off = 0
    for i, o in mlp.LAYERS:
        for size in (i * o, o):
            a, b = g[off:off + size], go[off:off + size]
            assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b) + 1e-12, (i, o, size)
            off += size
    assert off == g.size


def test_gradient_is_bitwise_reproducible():
    tls = _tls()
    th = _dev(tlsgen.mlp_init(3))
    X, t, norm = tlsgen.mlp_batch(300, seed=4)
    Xd, td, nd = _dev(X), _dev(t), _dev(norm)
    _, g1 = tls.tls_mlp_loss_grad(th, nd, Xd, td)
    _, g2 = tls.tls_mlp_loss_grad(th, nd, Xd, td)
    assert bool((g1 == g2).all())


def test_adam_matches_oracle():
    tls = _tls()
    rng = np.random.default_rng(5)
    th = tlsgen.mlp_init(6)
    m = (1e-3 * rng.standard_normal(th.size)).astype(np.float32)
    v = (1e-6 * rng.random(th.size)).astype(np.float32)
    g = (1e-2 * rng.standard_normal(th.size)).astype(np.float32)
    thd, md, vd = _dev(th), _dev(m), _dev(v)
    lr, b1, b2, eps, step = 1e-3, 0.9, 0.999, 1e-8, 7
    tls.tls_mlp_adam(thd, md, vd, _dev(g), step, lr, b1, b2, eps)
    # the oracle takes the FP32 values of the hyper-parameters the kernel receives
    f = lambda z: float(np.float32(z))
    m64, v64, g64 = m.astype(np.float64), v.astype(np.float64), g.astype(np.float64)
    tho, mo, vo = mlp.adam(th.astype(np.float64), m64, v64, g64, step, f(lr), f(b1), f(b2), f(eps))
    # FP32 rounding of the two-term moment updates: |err| <= 2u (|b m| + |(1-b) g|)
    u = 2.0 ** -24
    dm = 4 * u * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64))
    dv = 4 * u * (b2 * v64 + (1 - b2) * g64 * g64)
    assert np.all(np.abs(md.cpu().numpy() - mo) <= dm + 1e-30)
    assert np.all(np.abs(vd.cpu().numpy() - vo) <= dv + 1e-30)
    # the step lr m_hat / (sqrt(v_hat) + eps) inherits the moment error (the
    # update of m can cancel) plus a few roundings; theta adds its own rounding
    c1 = 1 / (1 - b1 ** step)
    c2 = 1 / (1 - b2 ** step)
    den = np.sqrt(vo * c2) + eps
    step_o = tho - th.astype(np.float64)
    bound = lr * c1 * dm / den + 1e-6 * np.abs(step_o) + 2 * u * np.abs(tho) + 1e-15
    assert np.all(np.abs(thd.cpu().numpy() - tho) <= bound)


def test_training_trajectory_follows_oracle():
    """30 Adam steps on one batch from the same initial parameters: the
    device (FP32) and oracle (FP64) losses stay together."""
    import torch
    tls = _tls()
    th0 = tlsgen.mlp_init(8)
    X, t, norm = tlsgen.mlp_batch(256, seed=9)
    thd = _dev(th0)
    md, vd = torch.zeros_like(thd), torch.zeros_like(thd)
    Xd, td, nd = _dev(X), _dev(t), _dev(norm)
    tho = th0.astype(np.float64)
    mo, vo = np.zeros_like(tho), np.zeros_like(tho)
    for s in range(1, 31):
        loss, g = tls.tls_mlp_loss_grad(thd, nd, Xd, td)
        tls.tls_mlp_adam(thd, md, vd, g, s, 1e-3)
        lo, go = mlp.loss_grad(tho, X, t, norm)
        tho, mo, vo = mlp.adam(tho, mo, vo, go, s, 1e-3)
        assert abs(float(loss.cpu()) - lo) <= 2e-3 * lo + 1e-7, (s, float(loss.cpu()), lo)
    assert lo < 0.5 * mlp.loss_grad(th0.astype(np.float64), X, t, norm)[0]


@pytest.mark.parametrize("gen", ["dense_gaussian", "sparse_small"])
def test_solver_features_match_oracle(gen):
    tls = _tls()
    print(f"features {gen}", flush=True)
    if gen == "dense_gaussian":
        A, b, _ = tlsgen.dense_gaussian(200, 20, seed=1000)
        Ad, Ah = tls.dense(A), A
    else:
        A, b, _, _ = tlsgen.sparse_scaled(3000, 150, 0.02, 2.0, 1e-3, seed=2100)
        Ad, Ah = tls.from_tlsgen(A), A.to_dense()
    fo, _ = features.warm_features(Ah, b)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    _, _, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(features=1, stop_patience=2))
    f = np.array(st["features"], dtype=np.float64)
    # features 22, 23 and 26 are logarithms of ratios near 1 formed from
    # products of dot products; the others are plain logs of FP64 quantities
    for i in range(32):
        tol = 1e-4 if i in (22, 23, 26, 12, 31) else 2e-6 * max(1.0, abs(fo[i]))
        assert abs(f[i] - fo[i]) <= tol, (i, f[i], fo[i])


def test_warm_start_with_exact_shift_keeps_the_answer_and_helps():
    """sigma0_hint = the exact sigma_{n+1} (noise 0.1, sigma_{n+1}/sigma'_n =
    0.04): the warm candidate is taken, it reaches 1e-10 no later than the
    plain start, and the answer is the plain solve's answer."""
    import torch
    tls = _tls()
    A, b, _ = tlsgen.dense_gaussian(200, 20, seed=1000, noise_A=1e-3, noise_b=0.1)
    ref = exact.svd_tls(A, b)
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    k_tol = {}
    for name, kw in (("plain", {}), ("warm", {"sigma0_hint": ref.sigma})):
        snaps = torch.zeros((60, 20), dtype=torch.float64, device="cuda")
        x, s, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(stop_patience=2, x_snapshots=snaps,
                                                                    **kw))
        xs = snaps.cpu().numpy()
        k_tol[name] = next(k for k in range(st["iters"])
                           if np.linalg.norm(xs[k] - ref.x) <= 1e-10 * np.linalg.norm(ref.x))
        assert abs(s - ref.sigma) / ref.sigma < 1e-10
        assert np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x) < 1e-10
        if name == "warm":
            assert st["warm_used"] == 1 and st["psi_warm"] < 0.1 * st["psi_plain"]
    assert k_tol["warm"] <= k_tol["plain"]


def test_network_warm_start_in_solve():
    """The solver's single-sample inference agrees with the oracle network on
    the solver's own features, and a warm solve returns the plain answer."""
    import torch
    tls = _tls()
    A, b, _ = tlsgen.dense_gaussian(200, 20, seed=1000)
    ref = exact.svd_tls(A, b)
    th = tlsgen.mlp_init(12)
    norm = np.concatenate([np.zeros(32), np.full(32, 0.1)]).astype(np.float32)
    thd, nd = _dev(th), _dev(norm)
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    x, s, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(stop_patience=2, mlp=(thd, nd)))
    yo, _ = mlp.forward(th.astype(np.float64), np.array([st["features"]], dtype=np.float32), norm)
    base = st["features"][31]
    want = st["sigma_ls"] * math.sqrt(-math.expm1(min(base + float(yo[0]), 0.0)))
    assert st["sigma_hat"] == pytest.approx(want, rel=2e-5)
    assert abs(s - ref.sigma) / ref.sigma < 1e-10
    assert np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x) < 1e-10
    del torch


@pytest.mark.parametrize("hint", ["exact", "half_sigma0", "above_sigma0"])
def test_warm_step_matches_oracle(hint):
    """The warm candidate x_1w = x_0 + lam u_0 + lam^2 u_1 and the psi-based
    choice between it and the plain x_1, against oracle.rqi.warm_candidate on
    the oracle's own x_LS and factor: the capped shift, both psi values and
    the choice agree."""
    tls = _tls()
    A, b, _ = tlsgen.dense_gaussian(200, 20, seed=1000, noise_A=1e-3, noise_b=0.1)
    ref = exact.svd_tls(A, b)
    R = rqi.cholesky_R(A)
    x0 = rqi.x_ls(A, b, R, 1)
    r0 = b - A @ x0
    s0 = math.sqrt(float(r0 @ r0) / (1 + x0 @ x0))
    sh = {"exact": ref.sigma, "half_sigma0": 0.5 * s0, "above_sigma0": 2.0 * s0}[hint]
    xk, taken, pw, pp, used = rqi.warm_candidate(A, b, R, x0, sh)
    Ad = tls.dense(A)
    P, _ = tls.tls_factor_precond(Ad, "fp64")
    x, s, st = tls.tls_rqi_solve(Ad, b, P, tls.default_opts(stop_patience=2, sigma0_hint=sh))
    print(f"warm {hint}: sigma_hat {st['sigma_hat']:.6e} / {used:.6e} psi_w {st['psi_warm']:.6e} / {pw:.6e} "
          f"psi_p {st['psi_plain']:.6e} / {pp:.6e} used {st['warm_used']} / {taken}", flush=True)
    assert st["sigma_ls"] == pytest.approx(s0, rel=1e-12)
    assert st["sigma_hat"] == pytest.approx(used, rel=1e-12)
    assert st["psi_warm"] == pytest.approx(pw, rel=1e-7)
    assert st["psi_plain"] == pytest.approx(pp, rel=1e-7)
    assert bool(st["warm_used"]) == taken
    assert abs(s - ref.sigma) / ref.sigma < 1e-10
