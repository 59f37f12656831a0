"""Edge shapes through the whole path: one column, exactly one 64-wide tile,
a ragged second tile, the minimal row count m = n + 1, and a CSR matrix with
empty rows. Answers against the SVD of [A, b]."""
import numpy as np
import pytest

import tlsgen
from oracle import certify, exact

pytestmark = pytest.mark.gpu


def _tls():
    from paper_2305_19028_amd import tls
    return tls


CASES = [
    ("n1", 50, 1),
    ("tile64_min_rows", 65, 64),
    ("ragged65", 200, 65),
    ("two_tiles_exact", 500, 128),
]


@pytest.mark.parametrize("name,m,n", CASES)
@pytest.mark.parametrize("path", ["fp64", "mixed"])
def test_edge_shapes_dense(name, m, n, path):
    tls = _tls()
    print(f"edge {name} {path}", flush=True)
    A, b, _ = tlsgen.dense_gaussian(m, n, seed=40 + n, noise_A=1e-3, noise_b=1e-2)
    ref = exact.svd_tls(A, b)
    assert ref.unique
    Ad = tls.dense(A)
    if path == "fp64":
        P, _ = tls.tls_factor_precond(Ad, "fp64")
        opts = tls.default_opts(stop_patience=2)
    else:
        P, _ = tls.tls_factor_precond(Ad, "fp16")
        opts = tls.default_opts(u_p="fp32", stop_patience=2, gate_enforce=1, allow_escalate=1,
                                refine_sweeps=1)
    x, s, st = tls.tls_rqi_solve(Ad, b, P, opts)
    x = x.cpu().numpy()
    bs, bx = certify.attainable(ref.sigma_1_Ab, ref.sigma, ref.kappa_tls)
    assert abs(s - ref.sigma) / ref.sigma < max(1e-10, 100 * bs)
    assert np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x) < max(1e-10, 100 * bx)


def test_csr_with_empty_rows_and_columns_of_one_entry():
    tls = _tls()
    # 0.2% density on 3000 x 120: most rows are empty, some columns hold one entry
    A, b, _, _ = tlsgen.sparse_scaled(3000, 120, 0.002, 1.0, 1e-3, seed=2400)
    D = A.to_dense()
    assert (np.count_nonzero(D, axis=1) == 0).sum() > 2000
    ref = exact.svd_tls(D, b)
    Ad = tls.from_tlsgen(A)
    for uq, up in (("fp64", "fp64"), ("fp16", "fp32")):
        P, _ = tls.tls_factor_precond(Ad, uq)
        opts = tls.default_opts(u_p=up, stop_patience=2, gate_enforce=int(uq != "fp64"),
                                allow_escalate=1, refine_sweeps=int(uq != "fp64"))
        x, s, st = tls.tls_rqi_solve(Ad, b, P, opts)
        bs, bx = certify.attainable(ref.sigma_1_Ab, ref.sigma, ref.kappa_tls)
        assert abs(s - ref.sigma) / ref.sigma < max(1e-10, 100 * bs), uq
        assert np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x) < max(1e-10, 100 * bx), uq
