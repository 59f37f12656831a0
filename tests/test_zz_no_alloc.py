"""The allocation-free PCGTLS entry point (tls_pcg_step_noalloc) against
tls_pcg_step, through the C ABI: the same kernels on the same inputs, so the
results agree bit for bit; two calls in a row on one device, the second with
a smaller problem (the static scratch keeps the first call's contents)."""
import numpy as np
import pytest

import tlsgen
from oracle import rqi

pytestmark = pytest.mark.gpu


def _case(n, seed):
    A, _, _ = tlsgen.dense_gaussian(3 * n, n, seed=seed)
    R = rqi.cholesky_R(A)
    s_n = np.linalg.svd(A, compute_uv=False)[-1]
    F = np.random.default_rng(seed).standard_normal((2, n))
    return R, (0.7 * s_n) ** 2, F


@pytest.mark.parametrize("mode", ["inverse", "substitution"])
def test_noalloc_pcg_matches_workspace_entry(mode):
    from paper_2305_19028_amd import tls
    for n, l, u_p, nrhs in [(700, 8, "fp64", 2), (130, 5, "fp32", 1)]:
        print(f"noalloc pcg n={n} l={l} {u_p} nrhs={nrhs} {mode}", flush=True)
        R, sig2, F = _case(n, n)
        P = tls.tls_precond_import(R, None, "fp64")
        P.set_apply(mode)
        rhs = F[:nrhs]
        ref, tref = tls.tls_pcg_step(P, sig2, rhs, l, u_p, trace=True)
        got, tgot = tls.tls_pcg_step_noalloc(P, sig2, rhs, l, u_p, trace=True)
        ref, got = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(ref.view(np.uint64), got.view(np.uint64))
        for k in ("eta", "delta", "alpha", "beta"):
            assert np.array_equal(np.nan_to_num(tref[k], nan=-7.0), np.nan_to_num(tgot[k], nan=-7.0)), k
        # against Algorithm 3 itself
        sR, sRT = rqi._tri_solvers(R)
        for r in range(nrhs):
            w = rqi.pcgtls(sR, sRT, sig2, rhs[r], l, dtype=np.float64 if u_p == "fp64" else np.float32)
            tol = 1e-11 if u_p == "fp64" else 1e-4
            assert np.linalg.norm(got[r] - w) <= tol * np.linalg.norm(w)


def test_noalloc_rejects_sizes_beyond_the_scratch():
    from paper_2305_19028_amd import tls
    # n = 5600 (N = 88 block rows) with l = 4096 needs more than 16 MiB
    # (the per-step partials alone are 4098 * 3 * 2 * 88 doubles); the size
    # check comes before any device work
    n = 5600
    P = tls.tls_precond_import(np.eye(n), None, "fp64")
    F = np.ones((2, n))
    assert tls.lib().tls_pcg_workspace_size(P.handle, 2, 4096) > 16 << 20
    with pytest.raises(tls.TLSError) as e:
        tls.tls_pcg_step_noalloc(P, 0.0, F, 4096, "fp64")
    assert e.value.status == -8 and "static" in str(e.value)
    # a size that fits runs: R = I, sigma = 0 gives omega = f after one step
    out, _ = tls.tls_pcg_step_noalloc(P, 0.0, F, 3, "fp64")
    assert np.array_equal(out.cpu().numpy(), F)
