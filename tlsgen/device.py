"""Seeded inputs drawn on the device, for data sets too large to draw on the
host (the learned warm start's 20000 training problems up to 50000 x 5000).

The recipes are those of the host generators in this package: a dense
N(0,1) matrix observed with an N(0,1) * noise perturbation and
b = A_clean x_true + noise N(0,1) (dense_gaussian), or a CSR matrix with
0.5% nonzeros at uniformly random distinct positions, every column covered,
values N(0,1) times column scales 10^U(0, 4), and b = A x_true +
noise N(0,1) (sparse_scaled). The problem's sizes, noise level and kind are
drawn on the host exactly as warmstart_problem draws them; the entries come
from torch's device generator seeded with the same sub-seed, so they differ
from the host version's values while following the same distributions.
No arithmetic of the method is here.
"""
from __future__ import annotations

import math

from . import rng


def _torch():
    import torch
    return torch


def _sizes(seed, m_range, n_range, noise_range):
    # the same draws, in the same order, as warmstart_problem on the host
    g = rng(seed)
    m = int(round(math.exp(g.uniform(math.log(m_range[0]), math.log(m_range[1])))))
    n_hi = min(n_range[1], m // 2)
    n = int(round(math.exp(g.uniform(math.log(n_range[0]), math.log(n_hi)))))
    noise = math.exp(g.uniform(math.log(noise_range[0]), math.log(noise_range[1])))
    kind = "dense" if g.uniform() < 0.5 else "sparse"
    sub = int(g.integers(0, 2**31 - 1))
    return m, n, noise, kind, sub


def dense_gaussian(m, n, noise_A, noise_b, gen, device="cuda"):
    """(A_obs as its transpose At (n x m row-major, i.e. A column-major), b,
    x_true), all float64 on the device."""
    torch = _torch()
    At = torch.randn((n, m), generator=gen, device=device, dtype=torch.float64)
    x = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
    b = At.t() @ x + noise_b * torch.randn(m, generator=gen, device=device, dtype=torch.float64)
    At.add_(torch.randn((n, m), generator=gen, device=device, dtype=torch.float64), alpha=noise_A)
    return At, b, x


def sparse_scaled(m, n, noise_b, gen, density=0.005, scale_decades=4.0, device="cuda"):
    """(row_ptr int32, col_idx int32, val float64, b, x_true) on the device."""
    torch = _torch()
    total = m * n
    nnz = int(round(density * total))
    kw = dict(generator=gen, device=device)
    pos = torch.unique(torch.randint(0, total, (int(nnz * 1.05) + 16,), dtype=torch.int64, **kw))
    while pos.numel() < nnz:
        extra = torch.randint(0, total, (nnz - pos.numel() + 16,), dtype=torch.int64, **kw)
        pos = torch.unique(torch.cat([pos, extra]))
    keep = torch.randperm(pos.numel(), **kw)[:nnz]
    pos = torch.sort(pos[keep]).values
    # one entry in every empty column
    present = torch.zeros(n, dtype=torch.bool, device=device)
    present[pos % n] = True
    missing = torch.nonzero(~present).flatten()
    if missing.numel():
        rows = torch.randint(0, m, (missing.numel(),), dtype=torch.int64, **kw)
        pos = torch.unique(torch.cat([pos, rows * n + missing]))
    scales = 10.0 ** (scale_decades * torch.rand(n, dtype=torch.float64, **kw))
    cols = pos % n
    rows = pos // n
    val = torch.randn(pos.numel(), dtype=torch.float64, **kw) * scales[cols]
    counts = torch.bincount(rows, minlength=m)
    row_ptr = torch.zeros(m + 1, dtype=torch.int64, device=device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    x = torch.randn(n, dtype=torch.float64, **kw)
    b = torch.zeros(m, dtype=torch.float64, device=device).index_add_(0, rows, val * x[cols])
    b += noise_b * torch.randn(m, dtype=torch.float64, **kw)
    return row_ptr.to(torch.int32), cols.to(torch.int32), val, b, x


def warmstart_problem(seed: int, m_range=(5000, 50000), n_range=(500, 5000), noise_range=(1e-6, 1e-2),
                      device="cuda"):
    """One warm-start problem drawn on the device: a dict with kind, m, n,
    noise and the device arrays (dense: At, the transpose of A; sparse:
    row_ptr, col_idx, val), b and x_true."""
    torch = _torch()
    m, n, noise, kind, sub = _sizes(seed, m_range, n_range, noise_range)
    gen = torch.Generator(device=device)
    gen.manual_seed(sub)
    out = {"kind": kind, "m": m, "n": n, "noise": noise}
    if kind == "dense":
        out["At"], out["b"], out["x_true"] = dense_gaussian(m, n, noise, noise, gen, device)
    else:
        out["row_ptr"], out["col_idx"], out["val"], out["b"], out["x_true"] = sparse_scaled(m, n, noise, gen,
                                                                                          device=device)
    return out
