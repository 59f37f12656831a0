"""Pins of oracle.constraints, oracle.lowprec, oracle.costmodel, oracle.polish."""
import math

import numpy as np
import pytest

import tlsgen
from oracle import constraints, lowprec, costmodel, polish, exact, rqi


# values printed in Section 4 for constraints (5) and (6) on the model problems
PRINTED = {
    "paper_random": (2e-2, 4e-3),
    "paper_delta": (9e-3, 1e-3),
    "paper_bjorck": (4e-2, None),      # (6) depends on the instance's gap
    "paper_vanhuffel": (2e-1, 5e-3),
}


@pytest.mark.parametrize("gen", sorted(PRINTED))
def test_constraint_magnitudes_match_printed(gen):
    A, b = getattr(tlsgen, gen)()
    bd = constraints.bounds(A, b)
    p5, p6 = PRINTED[gen]
    assert abs(math.log10(bd.bound5 / p5)) < math.log10(3.0)
    if p6 is not None:
        assert abs(math.log10(bd.bound6 / p6)) < math.log10(3.0)
    # (6) is never looser than (5)'s kappa_F analogue
    assert bd.bound6 <= 1.0 / bd.kappa_F * (1 + 1e-12)
    # half precision passes both constraints on these problems (Section 4)
    if p6 is not None:
        assert constraints.UNIT_ROUNDOFF["fp16"] < bd.bound6


def _diag_problem(s, beta, m):
    # A = [diag(s); 0] (m x n) and b = beta e_{n+1}, orthogonal to range(A):
    # the singular values of [A, b] are those of A plus beta, so with
    # beta < min(s), sigma_{n+1} = beta and sigma'_n = min(s) in closed form
    n = len(s)
    A = np.zeros((m, n))
    A[np.arange(n), np.arange(n)] = s
    b = np.zeros(m)
    b[n] = beta
    return A, b


def test_constraint_bounds_closed_form_diagonal():
    # every bound of Section 3.1 on a diagonal A, where kappa = s_max/s_min,
    # kappa_F = ||s||/s_min and H = D^{-1} A^T A D^{-1} = I (lambda_min = 1)
    s = np.array([4.0, 2.0, 1.0, 0.5, 0.25])
    m, n, beta = 9, 5, 0.1
    A, b = _diag_problem(s, beta, m)
    bd = constraints.bounds(A, b)
    kap, kapF = 16.0, math.sqrt(float(s @ s)) / 0.25
    gap = 1.0 - (beta / 0.25) ** 2
    want = dict(kappa=kap, kappa_F=kapF, sigma_n_A=0.25, sigma=beta,
                qr_nonsingular=1.0 / (m * n ** 1.5 * kap),
                qr_probabilistic=1.0 / (math.sqrt(m) * n ** 0.75 * kap),
                bound5=1.0 / kap, wilkinson=1.0 / (20.0 * n ** 1.5 * kap ** 2),
                chol=kap ** -2.0, hp=1.0 / ((2.0 + n) * (n + 1)), bound6=gap / kapF)
    for key, v in want.items():
        assert getattr(bd, key) == pytest.approx(v, rel=1e-13), key
    # scaled: A D^{-1} = [I; 0] has kappa = 1 and kappa_F = sqrt(n); sigma'_n
    # and sigma_{n+1} stay those of (A, b)
    sc = constraints.bounds(A, b, scaled=True)
    assert sc.kappa == pytest.approx(1.0, rel=1e-14) and sc.kappa_F == pytest.approx(math.sqrt(n), rel=1e-14)
    assert sc.sigma_n_A == pytest.approx(0.25, rel=1e-14) and sc.bound6 == pytest.approx(gap / math.sqrt(n), rel=1e-13)


@pytest.mark.parametrize("c", [0.3, 0.9, -0.99])
def test_constraint_hp_closed_form_two_columns(c):
    # columns e_1 and (c, sqrt(1 - c^2), 0...): A^T A = [[1, c], [c, 1]] is
    # already scaled, lambda_min(H) = 1 - |c|, kappa(A)^2 = (1 + |c|)/(1 - |c|)
    m = 6
    A = np.zeros((m, 2))
    A[0, 0] = 1.0
    A[0, 1], A[1, 1] = c, math.sqrt(1 - c * c)
    b = np.zeros(m)
    b[3] = 0.01
    bd = constraints.bounds(A, b)
    lam = 1.0 - abs(c)
    k2 = (1.0 + abs(c)) / (1.0 - abs(c))
    assert bd.hp == pytest.approx(lam / ((2 * lam + 2) * 3), rel=1e-10)
    assert bd.chol == pytest.approx(1.0 / k2, rel=1e-10)
    assert bd.wilkinson == pytest.approx(1.0 / (20 * 2 ** 1.5 * k2), rel=1e-10)
    assert bd.kappa == pytest.approx(math.sqrt(k2), rel=1e-10)
    # sigma'_n = sqrt(1 - |c|), sigma_{n+1} = 0.01
    assert bd.sigma_n_A == pytest.approx(math.sqrt(lam), rel=1e-10) and bd.sigma == pytest.approx(0.01, rel=1e-12)


def test_unit_roundoffs_table2():
    u = constraints.UNIT_ROUNDOFF
    assert abs(u["fp16"] - 4.88e-4) < 0.01e-4
    assert abs(u["fp32"] - 5.96e-8) < 0.01e-8
    assert abs(u["fp64"] - 1.11e-16) < 0.01e-16
    assert abs(u["fp128"] - 9.63e-35) < 0.01e-35


def test_round_fp16_is_ieee_rne():
    g = np.random.default_rng(0)
    x = np.concatenate([g.standard_normal(20000) * 10.0 ** g.uniform(-9, 5, 20000),
                        np.array([-0.0, 0.0]),
                        # exact ties between fp16 neighbours
                        (np.arange(1, 2000) + 0.5) * 2.0 ** -10,
                        np.array([65504.0, 65519.0, 65520.0, 1e6, 5.96e-8, 2.98e-8, 2.99e-8])])
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    got = lowprec.round_to(x, "fp16")
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    # signed zeros survive rounding (IEEE 754)
    z = lowprec.round_to(np.array([-0.0, 0.0, -1e-30]), "fp16")
    assert np.array_equal(z.view(np.uint64), np.array([-0.0, 0.0, -0.0]).view(np.uint64))


def test_round_bf16_nearest_even():
    g = np.random.default_rng(1)
    x = g.standard_normal(20000) * 10.0 ** g.uniform(-30, 30, 20000)
    got = lowprec.round_to(x, "bf16")
    bits = got.astype(np.float32).view(np.uint32)
    assert np.all(bits & 0xFFFF == 0)                    # representable in bf16
    assert np.array_equal(got.astype(np.float32).astype(np.float64), got)
    up = (bits + 0x10000).view(np.float32).astype(np.float64)
    dn = (bits - 0x10000).view(np.float32).astype(np.float64)
    e = np.abs(got - x)
    assert np.all(e <= np.abs(up - x)) and np.all(e <= np.abs(dn - x))
    # ties go to the even significand
    t = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8])
    assert np.array_equal(lowprec.round_to(t, "bf16"), [1.0, 1.0 + 2.0 ** -6])


def test_scaled_factor_backward_error():
    A, b, _, _ = tlsgen.sparse_scaled(2000, 100, seed=3)
    for fmt, u in (("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)):
        Rh, d = lowprec.scaled_factor(A, fmt)
        Ad = A.to_dense() / d
        H = Ad.T @ Ad
        err = np.linalg.norm(Rh.T @ Rh - H, 2)
        # input rounding, float32 Cholesky and storage rounding: a few u
        assert err < 20 * u * np.linalg.norm(H, 2)
        assert err > 0.01 * u * np.linalg.norm(H, 2)     # really is low precision


def test_costmodel_sums_algorithm4_lines():
    # per-line counts annotated in Algorithm 4, built from Table 1
    m, n, r = 5000, 300, 7
    T = costmodel.TABLE1
    line_r = T["matvec"](m, n) + 2 * m                  # r = b - A x
    line_sigma = T["vecmul"](m) + T["vecmul"](n)        # sigma^2
    init = line_r + line_sigma + 2 * T["subs"](n) + T["vecupdate"](n)
    line_f = 2 * m * n + 2 * n
    line_g = T["vecmul"](m)
    line_z = n
    line_beta = 2 * T["vecmul"](n)
    line_x = T["vecupdate"](n)
    per = line_r + line_sigma + line_f + line_g + line_z + line_beta + line_x
    pcg_setup = T["subs"](n) + T["vecmul"](n)
    # two substitutions, three inner products, four vector updates
    pcg_iter = 2 * T["subs"](n) + 3 * T["vecmul"](n) + 4 * T["vecupdate"](n) - 2 * n + 2 * n
    assert pcg_iter == 2 * n * n + 14 * n - 3
    steps = sum(2 * (k + 1) for k in range(1, r + 1))
    assert steps == r * r + 3 * r
    total = init + r * per + 2 * r * pcg_setup + steps * pcg_iter + T["qr"](m, n)
    assert abs(total - costmodel.cost(m, n, r)) / total < 1e-12


def test_costmodel_speedup_limits():
    assert costmodel.speedup(10 ** 12, 10 ** 7, 5) > 3.99
    assert costmodel.speedup(10 ** 12, 10 ** 7, 5) < 4.0
    for m, n, r in [(200, 20, 50), (10 ** 4, 10, 1000), (10 ** 6, 10 ** 3, 2000)]:
        assert costmodel.speedup(m, n, r) >= 1.0
        assert costmodel.speedup(m, n, r, 1.0, 1.0, 1.0) == 1.0
    # tall-skinny: more than 2x at a moderate number of RQIs
    assert costmodel.speedup(10 ** 6, 500, 5) > 2.0


def test_polish_rayleigh_quotient_is_stationary():
    A, b, _ = tlsgen.dense_gaussian(200, 20, seed=7)
    s = exact.svd_tls(A, b)
    mp = exact.mp_svd_tls(A[:30, :4], b[:30])
    sig = polish.rayleigh_ld(A[:30, :4], b[:30], mp.x)
    assert abs(sig - mp.sigma) / mp.sigma < 1e-15
    # a perturbation eps of x changes sigma only at second order:
    # ten times the perturbation gives a hundred times the change
    d = np.random.default_rng(2).standard_normal(20)
    d /= np.linalg.norm(d)
    ch = [polish.rayleigh_ld(A, b, s.x + e * d * np.linalg.norm(s.x)) - s.sigma for e in (1e-6, 1e-5)]
    assert ch[0] > 0 and ch[1] > 0
    assert 80 < ch[1] / ch[0] < 120


def test_polish_refines_x():
    A, b = tlsgen.paper_vanhuffel()
    sol = exact.svd_tls(A, b)
    x0 = sol.x * (1 + 1e-7)
    x1, sig = polish.polish(A, b, x0)
    assert np.linalg.norm(x1 - sol.x) / np.linalg.norm(sol.x) < 1e-13
    assert abs(sig - sol.sigma) / sol.sigma < 1e-14


def test_split_bf16_pair_bounds():
    # the split pair by its definition: hi is x rounded to bf16 (8
    # significant bits, unit roundoff 2^-8), lo is the remainder rounded to
    # bf16, so |x - hi| <= 2^-8 |x| and |x - hi - lo| <= 2^-8 |x - hi| (normal range)
    g = np.random.default_rng(3)
    x = g.standard_normal(20000) * 10.0 ** g.uniform(-20, 20, 20000)
    hi, lo = lowprec.split_bf16(x)
    assert np.array_equal(hi, lowprec.round_to(x, "bf16"))
    assert np.array_equal(lo, lowprec.round_to(lo, "bf16"))
    assert np.all(np.abs(x - hi) <= 2.0 ** -8 * np.abs(x))
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -8 * np.abs(x - hi))
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -16 * np.abs(x))
    # a worked case: 1 + 3 2^-9 lies between the bf16 neighbours 1 and
    # 1 + 2^-7, nearer the upper; the remainder -2^-9 is a bf16 number
    h1, l1 = lowprec.split_bf16(np.array([1.0 + 3 * 2.0 ** -9]))
    assert h1[0] == 1.0 + 2.0 ** -7 and l1[0] == -(2.0 ** -9) and h1[0] + l1[0] == 1.0 + 3 * 2.0 ** -9


def test_split_gram_drops_only_lo_lo():
    g = np.random.default_rng(5)
    A = g.standard_normal((300, 7))
    hi, lo = lowprec.split_bf16(A)
    full = (hi + lo).T @ (hi + lo)
    assert np.allclose(lowprec.split_gram(hi, lo) + lo.T @ lo, full, rtol=0, atol=1e-12 * np.abs(full).max())
    # and the pair's Gram matrix is within 3 2^-16 (relative to |A|^T |A|) of
    # A^T A: twice the representation error and the dropped lo^T lo
    W = np.abs(A).T @ np.abs(A)
    assert np.all(np.abs(lowprec.split_gram(hi, lo) - A.T @ A) <= 3 * 2.0 ** -16 * W)
