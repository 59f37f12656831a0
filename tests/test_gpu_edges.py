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


@pytest.mark.parametrize("defect", ["col_out_of_range", "col_negative", "row_ptr_decreasing",
                                    "row_ptr_end", "row_ptr_start", "unsorted_row", "duplicate_col"])
def test_invalid_csr_structure_is_an_argument_error(defect):
    """A malformed CSR matrix is rejected by the factorization with
    TLS_ERR_ARG: the device check reads only row_ptr[0..m] and, for rows whose
    pointers lie inside [0, nnz], their entries of col_idx, and it runs before
    any kernel uses the indices. A solve with other index arrays than the
    factor's is rejected as well."""
    import scipy.sparse as sp
    tls = _tls()
    g = np.random.default_rng(8)
    S = sp.random(400, 30, density=0.2, random_state=4, format="csr") + sp.eye(400, 30, format="csr")
    S.sort_indices()
    rp, ci, val = S.indptr.astype(np.int32).copy(), S.indices.astype(np.int32).copy(), S.data.copy()
    r = 7                                             # a row with at least two entries
    while rp[r + 1] - rp[r] < 2:
        r += 1
    e = rp[r]
    if defect == "col_out_of_range":
        ci[e + 1] = 30
    elif defect == "col_negative":
        ci[e] = -1
    elif defect == "row_ptr_decreasing":
        rp[r + 1] = rp[r] - 1
    elif defect == "row_ptr_end":
        rp[-1] = rp[-1] - 1
    elif defect == "row_ptr_start":
        rp[0] = 1
    elif defect == "unsorted_row":
        ci[e], ci[e + 1] = ci[e + 1], ci[e]
    else:
        ci[e + 1] = ci[e]
    print(f"invalid csr {defect}", flush=True)
    Ad = tls.csr(rp, ci, val, 400, 30)
    with pytest.raises(tls.TLSError) as ex:
        tls.tls_factor_precond(Ad, "fp64")
    assert ex.value.status == -1 and "CSR structure" in str(ex.value)
    # the valid matrix factors; a solve handed a copy of it (other arrays) is refused
    good = tls.csr(S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data, 400, 30)
    P, _ = tls.tls_factor_precond(good, "fp64")
    other = tls.csr(S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data, 400, 30)
    b = g.standard_normal(400)
    with pytest.raises(tls.TLSError) as ex2:
        tls.tls_rqi_solve(other, b, P)
    assert ex2.value.status == -1
    x, s, st = tls.tls_rqi_solve(good, b, P)
    assert np.isfinite(s)
