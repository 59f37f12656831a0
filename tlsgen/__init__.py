"""Seeded synthetic inputs for total least squares (TLS) problems.

This module only draws random data and assembles matrices; it contains no
part of the solver's arithmetic (no Rayleigh quotients, no conjugate
gradients, no factorizations used by the method). Both the CPU oracle and
the GPU path take their inputs from here.

Every generator uses ``numpy.random.Generator(PCG64(seed))`` so that an
instance is a pure function of its arguments. Dense matrices are returned
in column-major (Fortran) order; sparse matrices as a :class:`CSR` triple
with int32 indices, rows in order and column indices sorted within a row.

Workloads (the paper's own test problems are in Section 4; the large
synthetic configurations are this project's):

* ``dense_gaussian``   dense N(0,1) A with an errors-in-variables
  perturbation, b from the clean A plus noise (small dense case).
* ``sparse_scaled``    CSR A at uniform random positions, N(0,1) values
  times log-uniform column scales, b = A x_true + noise.
* ``reflector_dense``  A = Y diag(s) Z^T with single Householder
  reflectors Y, Z and geometric s, plus a spectral-size perturbation.
* ``planted_gap``      CSR A with noise orthogonal to range(A), scaled so
  that sigma_{n+1}([A,b]) sits a chosen relative gap below sigma_n(A).
* ``planted_svd``      [A,b] = Y [diag(sigma); 0] W^T with a prescribed
  spectrum, so sigma_{n+1} and the TLS solution are known in closed form.
* ``paper_*``          the five model problems of Section 4 (random,
  delta, Bjorck, Toeplitz, Van Huffel) built from their descriptions.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "CSR", "rng", "dense_gaussian", "sparse_scaled", "reflector_dense",
    "planted_gap", "planted_svd", "paper_random", "paper_delta",
    "paper_bjorck", "paper_toeplitz", "paper_vanhuffel", "warmstart_problem",
    "CONFIG_SEED",
]

# seed rule: 1000 * config index + instance
CONFIG_SEED = {"dense_small": 1000, "sparse_c2": 2000, "dense_c3": 3000,
               "sparse_c4": 4000}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclasses.dataclass
class CSR:
    """Compressed sparse row matrix, int32 indices, float64 values."""
    m: int
    n: int
    row_ptr: np.ndarray   # int32, m+1
    col_idx: np.ndarray   # int32, nnz
    val: np.ndarray       # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col_idx, self.row_ptr),
                             shape=(self.m, self.n))

    def to_dense(self) -> np.ndarray:
        out = np.zeros((self.m, self.n), order="F")
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        out[rows, self.col_idx] = self.val
        return out

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """Plain y = A x (used by generators to build b)."""
        prod = self.val * x[self.col_idx]
        y = np.zeros(self.m)
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        np.add.at(y, rows, prod)
        return y


def _csr_from_positions(m: int, n: int, pos: np.ndarray, val: np.ndarray) -> CSR:
    order = np.argsort(pos, kind="stable")
    pos = pos[order]
    val = val[order]
    rows = (pos // n).astype(np.int64)
    cols = (pos % n).astype(np.int32)
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds int32 range")
    return CSR(m, n, row_ptr.astype(np.int32), cols, np.ascontiguousarray(val, dtype=np.float64))


def _uniform_positions(g: np.random.Generator, m: int, n: int, nnz: int) -> np.ndarray:
    """``nnz`` distinct positions drawn uniformly from the m*n grid."""
    total = m * n
    if nnz > total:
        raise ValueError("nnz larger than m*n")
    if nnz > total // 4:
        return np.sort(g.permutation(total)[:nnz])
    pos = np.unique(g.integers(0, total, size=int(nnz * 1.05) + 16))
    while pos.size < nnz:
        extra = g.integers(0, total, size=nnz - pos.size + 16)
        pos = np.unique(np.concatenate([pos, extra]))
    # keep a uniform random subset of exactly nnz distinct positions
    keep = g.permutation(pos.size)[:nnz]
    return np.sort(pos[keep])


def _ensure_column_coverage(g, m, n, pos):
    """Add one entry to any empty column (a zero column makes A rank deficient)."""
    cols = pos % n
    present = np.zeros(n, dtype=bool)
    present[cols] = True
    missing = np.nonzero(~present)[0]
    if missing.size:
        rows = g.integers(0, m, size=missing.size)
        extra = rows.astype(np.int64) * n + missing
        pos = np.unique(np.concatenate([pos, extra]))
    return pos


# ----------------------------------------------------------------------------
# project workloads
# ----------------------------------------------------------------------------

def dense_gaussian(m: int = 200, n: int = 20, seed: int = 1000,
                   noise_A: float = 1e-3, noise_b: float = 1e-3):
    """Dense A with i.i.d. N(0,1) entries observed with an N(0,1)*noise_A
    perturbation; b = A_clean x_true + noise_b*N(0,1), x_true ~ N(0,1).

    Returns (A_obs column-major, b, x_true)."""
    g = rng(seed)
    A = g.standard_normal((m, n))
    x = g.standard_normal(n)
    b = A @ x + noise_b * g.standard_normal(m)
    A_obs = A + noise_A * g.standard_normal((m, n))
    return np.asfortranarray(A_obs), b, x


def sparse_scaled(m: int = 20000, n: int = 2000, density: float = 0.005,
                  scale_decades: float = 4.0, noise_b: float = 1e-4,
                  seed: int = 2000):
    """CSR A with round(density*m*n) distinct uniformly random positions,
    values N(0,1) * s_j where s_j = 10**U(0, scale_decades) per column;
    b = A x_true + noise_b*N(0,1).

    Returns (CSR, b, x_true, column_scales)."""
    g = rng(seed)
    nnz = int(round(density * m * n))
    pos = _uniform_positions(g, m, n, nnz)
    pos = _ensure_column_coverage(g, m, n, pos)
    scales = 10.0 ** g.uniform(0.0, scale_decades, size=n)
    val = g.standard_normal(pos.size) * scales[pos % n]
    A = _csr_from_positions(m, n, pos, val)
    x = g.standard_normal(n)
    b = A.matvec(x) + noise_b * g.standard_normal(m)
    return A, b, x, scales


def reflector_dense(m: int = 65536, n: int = 4096, s_min: float = 1e-3,
                    noise_A: float = 1e-5, noise_b: float = 1e-5,
                    seed: int = 3000, dtype=np.float64):
    """A = Y [diag(s); 0] Z^T + E with single Householder reflectors
    Y = I - 2 y y^T / y^T y (m x m) and Z = I - 2 z z^T / z^T z (n x n),
    s_i = s_min**((i-1)/(n-1)) (geometric from 1 to s_min).

    The perturbation E = noise_A * G / (sqrt(m) + sqrt(n)) has spectral
    norm about noise_A (entrywise noise_A*N(0,1) would have norm about
    noise_A*(sqrt(m)+sqrt(n)) and swamp the designed spectrum).
    b = A_clean x_true + noise_b*N(0,1).

    Returns (A column-major, b, x_true, s)."""
    g = rng(seed)
    y = g.standard_normal(m)
    z = g.standard_normal(n)
    x = g.standard_normal(n)
    s = s_min ** (np.arange(n) / max(n - 1, 1))
    yy = float(y @ y)
    zz = float(z @ z)
    # S Z^T = diag(s) (I - 2 z z^T / zz)
    SZt = np.diag(s) - (2.0 / zz) * np.outer(s * z, z)          # n x n
    # A_clean = Y [SZ^T; 0] = [SZ^T; 0] - (2/yy) y (y[:n]^T SZ^T)
    w = (2.0 / yy) * (y[:n] @ SZt)                                # n
    # -y w^T built as the transpose of the C-ordered (n, m) product: one
    # allocation, already column-major (the same values as -outer(y, w))
    A = np.multiply.outer(-w, y).T
    A[:n, :] += SZt
    b = A @ x + noise_b * g.standard_normal(m)
    scale = noise_A / (math.sqrt(m) + math.sqrt(n))
    chunk = max(1, (1 << 24) // m)
    buf = np.empty((chunk, m))                  # reused for every column block
    for j0 in range(0, n, chunk):
        j1 = min(n, j0 + chunk)
        blk = buf[: j1 - j0]
        g.standard_normal(out=blk)
        blk *= scale
        A[:, j0:j1] += blk.T
    return A.astype(dtype, copy=False), b, x, s


def planted_gap(m: int = 100000, n: int = 8000, density: float = 0.001,
                scale_decades: float = 6.0, rel_gap: float = 1e-3,
                seed: int = 4000):
    """CSR A (as in ``sparse_scaled`` with wider column scales) and
    b = A x_true + e with e orthogonal to range(A), its norm chosen so that
    the smallest singular value of [A, b] equals sqrt(lam) with
    lam = ((1 - rel_gap) * sigma_n)**2, sigma_n an estimate of sigma_n(A).

    Instance construction (not the solver). With A^T e = 0, the smallest root
    of the TLS secular equation is lam when
    ||e||^2 = lam (1 + ||x||^2 + lam x^T (A^T A - lam I)^{-1} x).
    The projection and the quadratic form are evaluated through the
    column-equilibrated Gram matrix G_s = D^{-1} A^T A D^{-1} (well
    conditioned even for widely scaled columns); sigma_n comes from the
    eigenvalues of A^T A and only needs to be accurate enough to keep lam
    below sigma_n(A)^2.

    Returns (CSR, b, x_true, lam, sigma_n estimate)."""
    import scipy.linalg as sla
    import scipy.sparse as sp
    g = rng(seed)
    nnz = int(round(density * m * n))
    pos = _uniform_positions(g, m, n, nnz)
    pos = _ensure_column_coverage(g, m, n, pos)
    scales = 10.0 ** g.uniform(0.0, scale_decades, size=n)
    val = g.standard_normal(pos.size) * scales[pos % n]
    A = _csr_from_positions(m, n, pos, val)
    x = g.standard_normal(n)
    S = A.to_scipy()
    d = np.sqrt(np.asarray(S.multiply(S).sum(axis=0)).ravel())
    Ss = S @ sp.diags(1.0 / d)
    Gs = (Ss.T @ Ss).toarray()
    cf = sla.cho_factor(Gs, lower=False)
    G = (S.T @ S).toarray()
    sig_n = math.sqrt(max(sla.eigvalsh(G, subset_by_index=[0, 0])[0], 0.0))
    lam = ((1.0 - rel_gap) * sig_n) ** 2
    # projected noise direction: e = h - A_s G_s^{-1} A_s^T h, applied twice
    h = g.standard_normal(m)
    e = h - Ss @ sla.cho_solve(cf, Ss.T @ h)
    e = e - Ss @ sla.cho_solve(cf, Ss.T @ e)
    # q = x^T (A^T A - lam I)^{-1} x = (x/d)^T (G_s - lam D^{-2})^{-1} (x/d)
    Msh = Gs - lam * np.diag(1.0 / (d * d))
    xs = x / d
    q = float(xs @ sla.cho_solve(sla.cho_factor(Msh, lower=False), xs))
    e_norm2 = lam * (1.0 + float(x @ x) + lam * q)
    e *= math.sqrt(e_norm2) / np.linalg.norm(e)
    b = S @ x + e
    return A, np.asarray(b), x, lam, sig_n


def planted_svd(m: int, n: int, sigmas, seed: int = 0):
    """[A, b] = C = Y [diag(sigmas); 0] W^T with Y = I - 2 y y^T / y^T y
    (m x m) and W = I - 2 w w^T, ||w|| = 1 ((n+1) x (n+1)).

    ``sigmas`` (length n+1, any order) are exactly the singular values of C
    and the right singular vectors are the columns of W. Returns
    (A column-major, b, sigmas, w)."""
    sig = np.asarray(sigmas, dtype=np.float64)
    if sig.shape != (n + 1,):
        raise ValueError("need n+1 singular values")
    if m < n + 1:
        raise ValueError("need m >= n+1")
    g = rng(seed)
    y = g.standard_normal(m)
    w = g.standard_normal(n + 1)
    w /= np.linalg.norm(w)
    Wt = np.eye(n + 1) - 2.0 * np.outer(w, w)                  # symmetric
    top = sig[:, None] * Wt                                     # diag(s) W^T
    C = np.zeros((m, n + 1), order="F")
    C[: n + 1, :] = top
    C -= (2.0 / float(y @ y)) * np.outer(y, y[: n + 1] @ top)
    return np.asfortranarray(C[:, :n]), np.ascontiguousarray(C[:, n]), sig, w


# ----------------------------------------------------------------------------
# the paper's model problems (Section 4), built from their descriptions
# ----------------------------------------------------------------------------

def paper_random(m: int = 100, n: int = 60, eps: float = 1e-6, seed: int = 0):
    """Example 1: A uniform on [0,1], b = ones; E = eps*U[0,1], e = eps*U[0,1].
    Returns (A+E, b+e)."""
    g = rng(seed)
    A = g.uniform(size=(m, n))
    b = np.ones(m)
    E = eps * g.uniform(size=(m, n))
    e = eps * g.uniform(size=m)
    return np.asfortranarray(A + E), b + e


def paper_delta(delta: float = 1e-2, eps: float = 1e-1, seed: int = 1):
    """Example 2 (the delta matrix). The displayed system is read as A 9x4
    with delta at (1,1) and (3,2) and ones at (7,3) and (9,4), x in R^4,
    b = ones(9). E = eps * Ebar .* A and e = eps * ebar .* b with Ebar, ebar
    uniform on (-1,1) (elementwise products: the shapes exclude a matrix
    product). Returns (A+E, b+e)."""
    g = rng(seed)
    A = np.zeros((9, 4))
    A[0, 0] = delta
    A[2, 1] = delta
    A[6, 2] = 1.0
    A[8, 3] = 1.0
    b = np.ones(9)
    Ebar = g.uniform(-1.0, 1.0, size=A.shape)
    ebar = g.uniform(-1.0, 1.0, size=b.shape)
    return np.asfortranarray(A + eps * Ebar * A), b + eps * ebar * b


def _haar_orthogonal(g, k):
    Q, Rr = np.linalg.qr(g.standard_normal((k, k)))
    return Q * np.sign(np.diag(Rr))


def paper_bjorck(m: int = 30, n: int = 15, eps: float = 0.05, seed: int = 1):
    """Example 3: A = Y [D; 0] Z^T, D = diag(1, 2^-1, ..., 2^-(n-1)),
    Y, Z Haar-random orthogonal; b = A x, x = (1, 1/2, ..., 1/n);
    E = eps*U[0,1] (m x n), e = eps*U[0,1] (m). Returns (A+E, b+e)."""
    g = rng(seed)
    Y = _haar_orthogonal(g, m)
    Z = _haar_orthogonal(g, n)
    D = np.diag(2.0 ** -np.arange(n))
    A = Y[:, :n] @ D @ Z.T
    x = 1.0 / np.arange(1, n + 1)
    b = A @ x
    E = eps * g.uniform(size=(m, n))
    e = eps * g.uniform(size=m)
    return np.asfortranarray(A + E), b + e


def _toeplitz(col, row):
    from scipy.linalg import toeplitz
    return toeplitz(col, row)


def paper_toeplitz(n: int = 100, omega: int = 2, alpha: float = 1.25,
                   scale: float = 1e-3, seed: int = 1):
    """Example 4 (signal restoration). T is n x (n - 2 omega) lower banded
    Toeplitz whose first column is c_i = exp(-(omega-i+1)^2/(2 alpha^2)) /
    sqrt(2 pi alpha^2) for i = 1..2 omega + 1 (zero below) and whose first
    row is (c_1, 0, ..., 0) (the printed row/column labels are read
    swapped: a first row of 2 omega + 1 nonzeros would not give a lower
    Toeplitz matrix). E is a random Toeplitz matrix of the same shape built
    the same way from a uniform first column, scaled by ``scale``;
    b = ones + scale * uniform. Returns (T+E, b)."""
    g = rng(seed)
    k = n - 2 * omega
    i = np.arange(1, 2 * omega + 2)
    c = np.zeros(n)
    c[: 2 * omega + 1] = np.exp(-((omega - i + 1) ** 2) / (2 * alpha ** 2)) / math.sqrt(2 * math.pi * alpha ** 2)
    r = np.zeros(k)
    r[0] = c[0]
    T = _toeplitz(c, r)
    ec = g.uniform(size=n)
    er = np.zeros(k)
    er[0] = ec[0]
    E = _toeplitz(ec, er)
    b = np.ones(n) + scale * g.uniform(size=n)
    return np.asfortranarray(T + scale * E), b


def paper_vanhuffel(n: int = 100, eps: float = 1e-6, seed: int = 1):
    """Example 5: A is n x (n-2): (n I - 1 1^T) of order n-2 on top of two
    rows of -1; b = -1 everywhere except b_{n-1} = n - 1. E = eps*U[0,1],
    e = eps*U[0,1]. Returns (A+E, b+e)."""
    g = rng(seed)
    k = n - 2
    A = np.vstack([n * np.eye(k) - np.ones((k, k)), -np.ones((2, k))])
    b = -np.ones(n)
    b[n - 2] = n - 1
    E = eps * g.uniform(size=(n, k))
    e = eps * g.uniform(size=n)
    return np.asfortranarray(A + E), b + e


# ----------------------------------------------------------------------------
# warm-start training distribution
# ----------------------------------------------------------------------------

def warmstart_problem(seed: int, m_range=(5000, 50000), n_range=(500, 5000),
                      noise_range=(1e-6, 1e-2)):
    """One training / evaluation problem for the learned warm start:
    m ~ logU(m_range), n ~ logU(n_lo, min(n_hi, m/2)), noise ~ logU, and the
    dense-Gaussian or sparse-scaled generator with probability 1/2 each.

    Returns a dict with kind, m, n, noise, and the generator output."""
    g = rng(seed)
    lm = g.uniform(math.log(m_range[0]), math.log(m_range[1]))
    m = int(round(math.exp(lm)))
    n_hi = min(n_range[1], m // 2)
    ln = g.uniform(math.log(n_range[0]), math.log(n_hi))
    n = int(round(math.exp(ln)))
    noise = math.exp(g.uniform(math.log(noise_range[0]), math.log(noise_range[1])))
    kind = "dense" if g.uniform() < 0.5 else "sparse"
    sub = int(g.integers(0, 2**31 - 1))
    if kind == "dense":
        A, b, x = dense_gaussian(m, n, seed=sub, noise_A=noise, noise_b=noise)
    else:
        A, b, x, _ = sparse_scaled(m, n, seed=sub, noise_b=noise)
    return {"kind": kind, "m": m, "n": n, "noise": noise, "A": A, "b": b, "x_true": x}


# ----------------------------------------------------------------------------
# warm-start network: initial parameters and synthetic batches
# ----------------------------------------------------------------------------

MLP_LAYERS = [(32, 256), (256, 256), (256, 256), (256, 1)]   # (in, out)


def mlp_init(seed: int = 7) -> np.ndarray:
    """Initial parameters (float32): for each layer W (out x in, row-major)
    then its bias, both uniform on [-1/sqrt(in), 1/sqrt(in)]."""
    g = rng(seed)
    parts = []
    for i, o in MLP_LAYERS:
        a = 1.0 / math.sqrt(i)
        parts.append(g.uniform(-a, a, size=i * o))
        parts.append(g.uniform(-a, a, size=o))
    return np.concatenate(parts).astype(np.float32)


def mlp_batch(batch: int, seed: int = 11):
    """Synthetic (features, targets, norm) for network tests: features
    N(1, 2^2), targets a smooth function of them, norm = [mean, 1/std]."""
    g = rng(seed)
    X = (1.0 + 2.0 * g.standard_normal((batch, 32))).astype(np.float32)
    t = (np.tanh(X[:, :8].astype(np.float64) @ g.standard_normal(8) / 8.0)
         - 0.1 * X[:, 8].astype(np.float64) ** 2 / 4.0).astype(np.float32)
    norm = np.concatenate([np.full(32, 1.0), np.full(32, 0.5)]).astype(np.float32)
    return X, t, norm
