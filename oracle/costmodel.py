"""Operation-count performance model (Section 3.2, Table 1).

cost(m, n, r, c, c_p, c_q) =
    c   (2mn + 3m + 4n + 2n^2 - 2 + r (4mn + 5m + 11n - 5))
  + c_p (2r (n^2 + 2n - 1) + (r^2 + 3r)(2n^2 + 14n - 3))
  + c_q (2mn^2 - 2n^3/3)

with (c, c_p, c_q) the per-precision weights (1 double, 0.5 single,
0.25 half). The paper prints the speedup as cost(MP)/cost(plain); it is
read as cost(plain)/cost(MP), the only orientation under which "up to 4x"
holds.

Pins: tests/test_oracle_misc.py (the formula equals the sum of the
Table 1 counts over the lines of Algorithm 4; the supremum 4 for
(1, 0.5, 0.25); speedup >= 1 whenever the weights are <= 1).
"""
from __future__ import annotations

TABLE1 = {
    "qr": lambda m, n: 2 * m * n * n - 2 * n ** 3 / 3,
    "subs": lambda n: n * n,
    "matvec": lambda m, n: 2 * m * n - m,
    "vecmul": lambda n: 2 * n - 1,
    "vecupdate": lambda n: 2 * n,
}

WEIGHTS = {"fp64": 1.0, "fp32": 0.5, "fp16": 0.25}


def cost(m, n, r, c=1.0, c_p=1.0, c_q=1.0) -> float:
    outer = 2 * m * n + 3 * m + 4 * n + 2 * n * n - 2 + r * (4 * m * n + 5 * m + 11 * n - 5)
    inner = 2 * r * (n * n + 2 * n - 1) + (r * r + 3 * r) * (2 * n * n + 14 * n - 3)
    fact = 2 * m * n * n - 2 * n ** 3 / 3
    return c * outer + c_p * inner + c_q * fact


def speedup(m, n, r, c=1.0, c_p=0.5, c_q=0.25) -> float:
    """cost(plain) / cost(mixed) at the same number r of RQIs."""
    return cost(m, n, r) / cost(m, n, r, c, c_p, c_q)
