"""The device-side problem generator (tlsgen.device) run on the CPU: the
sizes are the host generator's, the matrices follow the stated recipe."""
import numpy as np
import pytest

import tlsgen
from tlsgen import device


@pytest.mark.parametrize("seed", range(4))
def test_sizes_match_host_generator(seed):
    h = tlsgen.warmstart_problem(seed, m_range=(300, 900), n_range=(20, 80))
    d = device.warmstart_problem(seed, m_range=(300, 900), n_range=(20, 80), device="cpu")
    assert (h["kind"], h["m"], h["n"], h["noise"]) == (d["kind"], d["m"], d["n"], d["noise"])


def _first(kind, lo=(2000, 6000), n=(100, 400)):
    for s in range(200):
        p = device.warmstart_problem(s, m_range=lo, n_range=n, device="cpu")
        if p["kind"] == kind:
            return p
    raise AssertionError("no problem of that kind")


def test_sparse_recipe():
    p = _first("sparse")
    m, n = p["m"], p["n"]
    rp, ci, va = p["row_ptr"].numpy(), p["col_idx"].numpy(), p["val"].numpy()
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == ci.size == va.size
    assert abs(ci.size / (m * n) - 0.005) < 0.0005                 # 0.5% nonzeros
    assert np.unique(ci).size == n                                  # every column covered
    for i in range(0, m, max(1, m // 50)):                          # distinct, sorted positions
        assert np.all(np.diff(ci[rp[i]:rp[i + 1]]) > 0)
    A = tlsgen.CSR(m, n, rp, ci, va)
    r = p["b"].numpy() - A.matvec(p["x_true"].numpy())
    assert 0.8 < r.std() / p["noise"] < 1.2                          # b = A x + noise N(0,1)
    scales = np.sqrt(np.bincount(ci, weights=va * va, minlength=n) / np.bincount(ci, minlength=n))
    assert 0.3 < scales.min() and scales.max() < 3e4                # N(0,1) x 10^U(0,4)


def test_dense_recipe():
    p = _first("dense")
    m, n = p["m"], p["n"]
    At = p["At"].numpy()
    assert At.shape == (n, m)
    assert abs(At.std() - 1.0) < 0.02 and abs(At.mean()) < 0.02
    # b = A_clean x + noise: the residual against the observed A is about
    # noise (sqrt(1 + ||x||^2)) in size
    r = p["b"].numpy() - At.T @ p["x_true"].numpy()
    x = p["x_true"].numpy()
    assert r.std() < 3 * p["noise"] * np.sqrt(1 + x @ x)
