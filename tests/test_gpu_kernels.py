"""GPU parity of the individual kernels through the C ABI against the CPU
oracle / plain NumPy on the same seeded inputs."""
import numpy as np
import pytest
import scipy.linalg as sla

import tlsgen
from oracle import lowprec, rqi

pytestmark = pytest.mark.gpu


def _tls():
    from paper_2305_19028_amd import tls
    return tls


@pytest.mark.parametrize("fmt", ["fp16", "bf16", "fp32"])
def test_round_bit_exact(fmt):
    tls = _tls()
    g = np.random.default_rng(5)
    x = np.concatenate([
        g.standard_normal(50000) * 10.0 ** g.uniform(-40, 40, 50000),
        (np.arange(1, 3000) + 0.5) * 2.0 ** -10,          # fp16 ties
        1.0 + (np.arange(0, 3000) + 0.5) * 2.0 ** -7,     # bf16 ties
        np.array([0.0, -0.0, 65504.0, 65519.99, 65520.0, 6.0e-8, 2.98e-8, 1e-45, 3.4e38, 3.5e38]),
    ])
    got = _tls().tls_round(x, fmt).cpu().numpy()
    ref = lowprec.round_to(x, fmt)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


@pytest.mark.parametrize("kind", ["dense", "csr"])
@pytest.mark.parametrize("m,n", [(70, 3), (1000, 65), (4097, 130)])
def test_matvec(kind, m, n):
    tls = _tls()
    print(f"matvec {kind} {m}x{n}", flush=True)
    if kind == "dense":
        A, b, _ = tlsgen.dense_gaussian(m, n, seed=m + n)
        Ad = tls.dense(A)
        P = None
        Af = A
    else:
        A, b, _, _ = tlsgen.sparse_scaled(m, n, density=0.05, seed=m + n)
        Ad = tls.from_tlsgen(A)
        P, _ = tls.tls_factor_precond(Ad, "fp64")
        Af = A.to_dense()
    x = np.random.default_rng(1).standard_normal(n)
    y = tls.tls_matvec(Ad, P, 0, x).cpu().numpy()
    assert np.allclose(y, Af @ x, rtol=1e-12, atol=1e-12 * np.abs(Af).max() * np.abs(x).sum())
    if P is None and kind == "csr":
        return
    if kind == "dense":
        P = None
    z = tls.tls_matvec(Ad, P, 1, b).cpu().numpy()
    ref = Af.T @ b
    assert np.allclose(z, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def _csr_case(kind):
    import scipy.sparse as sp
    g = np.random.default_rng(11)
    if kind == "workload":            # row blocks of 1024, ~5 entries per block and column
        m, n, k = 20000, 2000, 200000
    elif kind == "ragged":            # ragged last block, empty rows, one full column
        m, n, k = 3001, 300, 18000
    else:                             # more row blocks x columns than the segmented build takes
        m, n, k = 1_100_000, 1000, 22000
    rows, cols = g.integers(0, m, k), g.integers(0, n, k)
    if kind == "ragged":
        keep = (rows < 100) | (rows >= 500)
        rows, cols = rows[keep], cols[keep]
        rows, cols = np.concatenate([rows, np.arange(m)]), np.concatenate([cols, np.full(m, 11)])
    A = sp.coo_matrix((g.standard_normal(rows.size), (rows, cols)), shape=(m, n)).tocsr()
    A = (A + sp.eye(m, n, format="csr")).tocsr()     # full column rank
    A.sum_duplicates()
    A.sort_indices()
    return A


@pytest.mark.parametrize("kind", ["workload", "ragged", "fallback"])
def test_csc_copy_rmatvec(kind):
    """A^T b through the CSC copy a factorization builds (row-block segments
    with LDS slot counters, or the global-atomic build past its size limit):
    equal to SciPy's product to rounding, and bit-identical across two
    factorizations (rows sorted inside each column, so the summation order is
    fixed)."""
    tls = _tls()
    A = _csr_case(kind)
    m, n = A.shape
    print(f"csc {kind} {m}x{n} nnz {A.nnz}", flush=True)
    Ad = tls.csr(A.indptr, A.indices, A.data, m, n)
    b = np.random.default_rng(3).standard_normal(m)
    ref = A.T @ b
    zs = []
    for _ in range(2):
        P, _ = tls.tls_factor_precond(Ad, "fp64")
        zs.append(tls.tls_matvec(Ad, P, 1, b).cpu().numpy())
    # both sums err by at most (column count) u |A|^T |b| each
    kmax = int(np.diff(A.tocsc().indptr).max())
    scale = abs(A).T @ np.abs(b)
    assert np.all(np.abs(zs[0] - ref) <= 2 * kmax * 2.0 ** -53 * scale), np.max(np.abs(zs[0] - ref) / scale)
    assert np.array_equal(zs[0].view(np.uint64), zs[1].view(np.uint64))


def _tri(n, seed, cond=10.0):
    g = np.random.default_rng(seed)
    A = g.standard_normal((n + 20, n))
    R = np.linalg.qr(A, mode="r")
    R = R * np.sign(np.diag(R))[:, None]
    return R


@pytest.mark.parametrize("mode", ["inverse", "inverse_rows", "substitution"])
@pytest.mark.parametrize("n", [5, 64, 100, 257, 1000, 3100])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_triangular_solves_fp64(n, nrhs, mode):
    tls = _tls()
    print(f"trsv n={n} nrhs={nrhs} {mode}", flush=True)
    R = _tri(n, n)
    d = np.exp(np.random.default_rng(2).uniform(-2, 2, n))
    P = tls.tls_precond_import(R, d, "fp64")
    P.set_apply(mode)
    V = np.random.default_rng(3).standard_normal((nrhs, n))
    Rfull = R * d[None, :]          # R = R_hat diag(d)
    for trans in (0, 1):
        out = tls.tls_apply_precond(P, trans, V).cpu().numpy()
        for r in range(nrhs):
            ref = sla.solve_triangular(Rfull, V[r], lower=False, trans="T" if trans else "N")
            assert np.linalg.norm(out[r] - ref) <= 1e-12 * np.linalg.norm(ref), (trans, r)


@pytest.mark.parametrize("mode", ["inverse", "inverse_rows", "substitution"])
@pytest.mark.parametrize("storage", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("u_p", ["fp64", "fp32"])
def test_triangular_solves_low_storage(storage, u_p, mode):
    tls = _tls()
    n = 300
    R = _tri(n, 7)
    R = R / np.abs(R).max()
    P = tls.tls_precond_import(R, None, storage)
    P.set_apply(mode)
    Rq = np.triu(lowprec.round_to(R, storage))      # what the library stores
    V = np.random.default_rng(4).standard_normal((2, n))
    # the explicit inverse of a low-precision factor is held in FP32
    tol = 1e-12 if (u_p == "fp64" and mode == "substitution") else (1e-6 if u_p == "fp64" else 1e-4)
    for trans in (0, 1):
        out = tls.tls_apply_precond(P, trans, V, u_p).cpu().numpy()
        for r in range(2):
            ref = sla.solve_triangular(Rq, V[r], lower=False, trans="T" if trans else "N")
            assert np.linalg.norm(out[r] - ref) <= tol * np.linalg.norm(ref) * 10, (trans, r)


@pytest.mark.parametrize("mode", ["inverse", "inverse_rows", "substitution"])
@pytest.mark.parametrize("n,l", [(20, 0), (20, 3), (130, 5), (700, 8), (3100, 3)])
def test_pcg_step_matches_algorithm3(n, l, mode):
    tls = _tls()
    print(f"pcg n={n} l={l} {mode}", flush=True)
    A, b, _ = tlsgen.dense_gaussian(3 * n, n, seed=n)
    R = rqi.cholesky_R(A)
    P = tls.tls_precond_import(R, None, "fp64")
    P.set_apply(mode)
    sR, sRT = rqi._tri_solvers(R)
    s_n = np.linalg.svd(A, compute_uv=False)[-1]
    sig2 = (0.7 * s_n) ** 2
    F = np.random.default_rng(n).standard_normal((2, n))
    out, tr = tls.tls_pcg_step(P, sig2, F, l, "fp64", trace=True)
    out = out.cpu().numpy()
    for r in range(2):
        w, t = rqi.pcgtls(sR, sRT, sig2, F[r], l, trace=True)
        assert np.linalg.norm(out[r] - w) <= 1e-11 * np.linalg.norm(w)
        k = len(t.delta)
        assert np.allclose(tr["delta"][r][:k], t.delta, rtol=1e-10)
        assert np.allclose(tr["eta"][r][:k], t.eta[:k], rtol=1e-10)
    # FP32 arithmetic: same iteration to single precision
    out32, _ = tls.tls_pcg_step(P, sig2, F, l, "fp32")
    out32 = out32.cpu().numpy()
    for r in range(2):
        w = rqi.pcgtls(sR, sRT, sig2, F[r], l)
        assert np.linalg.norm(out32[r] - w) <= 1e-4 * np.linalg.norm(w)


@pytest.mark.parametrize("mode", ["inverse", "inverse_rows", "substitution"])
def test_pcg_sigma_zero_and_single_rhs(mode):
    tls = _tls()
    A, b, _ = tlsgen.dense_gaussian(90, 30, seed=3)
    R = rqi.cholesky_R(A)
    P = tls.tls_precond_import(R, None, "fp64")
    P.set_apply(mode)
    f = np.random.default_rng(9).standard_normal(30)
    out, tr = tls.tls_pcg_step(P, 0.0, f, 4, trace=True)
    ref = sla.solve_triangular(R, sla.solve_triangular(R, f, trans="T"))
    assert np.allclose(out.cpu().numpy()[0], ref, rtol=1e-12)
    # alpha_0 = 1 exactly (C = I), so eta_1 = 0 ends the loop before step 1:
    # delta_1 is never formed
    assert tr["eta"][0][1] == 0.0 and np.isnan(tr["delta"][0][1])


@pytest.mark.parametrize("mode", ["inverse", "inverse_rows", "substitution"])
def test_pcg_eta_underflow_ends_cleanly(mode):
    # the oracle's float32 case: R = 1e-3 I, f = 1e-27. s_0 = 1e-24 squares
    # below the smallest float32 subnormal, so eta_0 = 0 while s_0 != 0. Run
    # as printed, the next beta is 0/0 and omega turns NaN; with the eta check
    # the loop ends before step 0 and omega stays 0 (the oracle's result)
    tls = _tls()
    n = 8
    R = 1e-3 * np.eye(n)
    P = tls.tls_precond_import(R, None, "fp64")
    P.set_apply(mode)
    f = np.full((2, n), 1e-27)
    sR, sRT = rqi._tri_solvers(R, np.float32)
    with np.errstate(divide="raise", invalid="raise"):
        w_ref, t_ref = rqi.pcgtls(sR, sRT, 0.5, f[0], l=4, dtype=np.float32, trace=True)
    out, tr = tls.tls_pcg_step(P, 0.5, f, 4, "fp32", trace=True)
    out = out.cpu().numpy()
    assert t_ref.steps == 0 and np.all(w_ref == 0)
    assert np.all(out == 0.0), out
    for r in range(2):
        assert tr["eta"][r][0] == 0.0 and np.all(np.isnan(tr["delta"][r]))
        assert np.all(np.isnan(tr["alpha"][r]))


@pytest.mark.parametrize("u_q", ["fp64", "bf16"])
def test_tall_dense_column_norms(u_q):
    """A dense A taller than 64 slabs of 2048 rows (140001 rows: the norm
    pass's slab sums are reduced in two levels, the last slab ragged), with
    leading dimension > m: the scaling d matches the column norms to 1e-14,
    the FP64 factor the LAPACK Cholesky of the scaled Gram matrix, the solve
    (over the row-major copy made from the padded buffer) the SVD answer to
    1e-10, and a NaN in the padding rows between columns (not part of A) is
    ignored while one inside A is reported."""
    tls = _tls()
    import torch
    m, n, ld = 140001, 40, 140003
    print(f"tall dense {u_q}", flush=True)
    A, b, _ = tlsgen.dense_gaussian(m, n, seed=17)
    A = A * np.exp(np.random.default_rng(2).uniform(-2, 2, n))
    buf = np.full((n, ld), np.nan)            # column-major with NaN padding rows
    buf[:, :m] = A.T
    dev = torch.from_numpy(buf).cuda()
    Ad = tls.dense_t(dev, m)
    P, _ = tls.tls_factor_precond(Ad, u_q)
    Rh, d = tls.tls_precond_export(P)
    dref = np.linalg.norm(A, axis=0)
    assert np.allclose(d, dref, rtol=1e-14, atol=0)
    if u_q == "fp64":
        H = (A / dref).T @ (A / dref)
        assert np.max(np.abs(Rh - sla.cholesky(H, lower=False))) < 1e-11
    # the solve reads the row-major copy made from the padded buffer
    from oracle import exact
    ref = exact.svd_tls(A, b)
    opts = tls.default_opts(stop_patience=2) if u_q == "fp64" else \
        tls.default_opts(u_p="fp32", gate_enforce=1, allow_escalate=1, stop_patience=2, refine_sweeps=1)
    x, sigma, st = tls.tls_rqi_solve(Ad, b, P, opts)
    es = abs(sigma - ref.sigma) / ref.sigma
    ex = np.linalg.norm(x.cpu().numpy() - ref.x) / np.linalg.norm(ref.x)
    print(f"solve: sigma {es:.2e} x {ex:.2e} iters {st['iters']}", flush=True)
    assert es < 1e-10 and ex < 1e-10
    buf[5, 1000] = np.nan                     # inside A: column 5, row 1000
    dev2 = torch.from_numpy(buf).cuda()
    with pytest.raises(tls.TLSError) as e:
        tls.tls_factor_precond(tls.dense_t(dev2, m), u_q)
    assert e.value.status == -9


@pytest.mark.parametrize("case", ["dense_small", "dense_ragged", "sparse"])
@pytest.mark.parametrize("u_q", ["fp64"])
def test_factor_matches_cholesky(case, u_q):
    tls = _tls()
    print(f"factor {case} {u_q}", flush=True)
    if case == "dense_small":
        A, b, _ = tlsgen.dense_gaussian(200, 20, seed=1000)
        Ad = tls.dense(A)
        Af = A
    elif case == "dense_ragged":
        A, b, _ = tlsgen.dense_gaussian(700, 150, seed=12)
        Ad = tls.dense(A)
        Af = A
    else:
        A, b, _, _ = tlsgen.sparse_scaled(3000, 200, density=0.02, seed=7)
        Ad = tls.from_tlsgen(A)
        Af = A.to_dense()
    P, rep = tls.tls_factor_precond(Ad, u_q)
    Rh, d = tls.tls_precond_export(P)
    dref = np.linalg.norm(Af, axis=0)
    assert np.allclose(d, dref, rtol=1e-14)
    H = (Af / dref).T @ (Af / dref)
    Rref = sla.cholesky(H, lower=False)
    assert np.max(np.abs(Rh - Rref)) < 1e-12 * 10


@pytest.mark.parametrize("case", ["dense", "sparse"])
@pytest.mark.parametrize("u_q", ["fp32", "fp16", "bf16", "bf16x3"])
def test_low_precision_factor_and_gate(case, u_q):
    from oracle import constraints
    tls = _tls()
    print(f"factor {case} {u_q}", flush=True)
    if case == "dense":
        A, b, _ = tlsgen.dense_gaussian(700, 150, seed=12)
        Ad = tls.dense(A)
        Af = A
    else:
        A, b, _, _ = tlsgen.sparse_scaled(3000, 200, density=0.02, seed=7)
        Ad = tls.from_tlsgen(A)
        Af = A.to_dense()
    P, rep = tls.tls_factor_precond(Ad, u_q)
    Rh, d = tls.tls_precond_export(P)
    u = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8, "bf16x3": 2.0 ** -16}[u_q]
    # the stored factor is a u_q-accurate Cholesky factor of the scaled Gram matrix
    H = (Af / d).T @ (Af / d)
    err = np.linalg.norm(Rh.T @ Rh - H, 2) / np.linalg.norm(H, 2)
    assert err < 30 * u, err
    # stored values are representable in the storage format (the split BF16
    # factor is computed and stored in FP32)
    store = "fp32" if u_q == "bf16x3" else u_q
    assert np.array_equal(Rh, np.triu(lowprec.round_to(Rh, store)))
    assert rep["used"] == tls.PREC[u_q]
    # Lanczos estimates against the exact singular values
    ex = constraints.bounds(Af, b, scaled=True)
    assert abs(rep["sigma_n_est"] - ex.sigma_n_A) / ex.sigma_n_A < 0.2
    assert 0.5 < rep["kappa_est"] / ex.kappa < 1.0 + 1e-6 + 50 * u
    assert abs(rep["bound5"] - ex.bound5) / ex.bound5 < 1.0
    # the Cholesky kappa^-2 and the HP bound from the same estimates: the
    # Lanczos Ritz values lie inside the spectrum, so kappa_hat <= kappa and
    # lambda_min_hat >= lambda_min(H): both bounds come out at or above the
    # exact ones, within the estimates' accuracy (kappa to a factor 2)
    assert 1.0 - 1e-6 <= rep["bound_chol"] / ex.chol < 4.0, (rep["bound_chol"], ex.chol)
    assert 1.0 - 1e-6 <= rep["bound_hp"] / ex.hp < 4.0, (rep["bound_hp"], ex.hp)
    # the verdict bits follow the printed comparisons u_q < bound
    uq = rep["u_q"]
    assert bool(rep["verdict"] & 1) == (uq < rep["bound5"])
    assert bool(rep["verdict"] & 2) == (uq < rep["bound_chol"])
    assert bool(rep["verdict"] & 4) == (uq < rep["bound_hp"])
