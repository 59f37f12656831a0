"""Pins of the float64 warm-start network (oracle.mlp)."""
import math

import numpy as np
import pytest

import tlsgen
from oracle import mlp


def test_param_count():
    # 32*256+256 + 2*(256*256+256) + 256+1
    assert mlp.param_count() == 140289
    assert tlsgen.mlp_init(0).size == 140289


def test_gelu_tabulated_normal_cdf():
    # GELU(z) = z Phi(z); Phi(1) = 0.8413447460685429, Phi(2) = 0.9772498680518208
    # (standard normal table)
    z = np.array([0.0, 1.0, -1.0, 2.0, -2.0])
    want = np.array([0.0, 0.8413447460685429, -(1 - 0.8413447460685429),
                     2 * 0.9772498680518208, -2 * (1 - 0.9772498680518208)])
    assert np.allclose(mlp.gelu(z), want, rtol=0, atol=1e-15)
    # derivative: GELU'(0) = 1/2, GELU'(z) -> 1 for large z, -> 0 for very negative z
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5, abs=1e-15)
    assert mlp.gelu_grad(np.array([12.0]))[0] == pytest.approx(1.0, abs=1e-12)
    assert abs(mlp.gelu_grad(np.array([-12.0]))[0]) < 1e-12
    # and against a central difference of GELU itself
    zz = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(zz + h) - mlp.gelu(zz - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(zz), fd, rtol=0, atol=1e-8)


def test_zero_network_outputs_last_bias():
    th = np.zeros(mlp.param_count())
    th[-1] = 0.37
    X, _, norm = tlsgen.mlp_batch(5)
    y, _ = mlp.forward(th, X, norm)
    assert np.all(y == 0.37)


def test_gradient_matches_central_differences():
    th = tlsgen.mlp_init(3).astype(np.float64)
    X, t, norm = tlsgen.mlp_batch(6, seed=4)
    loss, g = mlp.loss_grad(th, X, t, norm)
    assert loss > 0
    rng = np.random.default_rng(0)
    # every layer's weights and biases are sampled
    offs, off = [], 0
    for i, o in mlp.LAYERS:
        offs.append((off, off + i * o)); off += i * o
        offs.append((off, off + o)); off += o
    idx = np.concatenate([rng.integers(a, b, size=6) for a, b in offs])
    h = 1e-6
    for k in idx:
        tp = th.copy(); tp[k] += h
        tm = th.copy(); tm[k] -= h
        fd = (mlp.loss_grad(tp, X, t, norm)[0] - mlp.loss_grad(tm, X, t, norm)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])) + 1e-9, (k, fd, g[k])


def test_adam_first_step_closed_form():
    # with m = v = 0 the bias-corrected moments are g and g^2, so the first
    # step is -lr g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-9, 0.0])
    th = np.array([1.0, 1.0, 1.0, 1.0])
    lr, eps = 1e-2, 1e-8
    th1, m, v = mlp.adam(th, np.zeros(4), np.zeros(4), g, 1, lr, eps=eps)
    assert np.allclose(th1, th - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_reduces_the_loss():
    th = tlsgen.mlp_init(5).astype(np.float64)
    X, t, norm = tlsgen.mlp_batch(64, seed=6)
    m = np.zeros_like(th); v = np.zeros_like(th)
    l0 = mlp.loss_grad(th, X, t, norm)[0]
    for s in range(1, 31):
        loss, g = mlp.loss_grad(th, X, t, norm)
        th, m, v = mlp.adam(th, m, v, g, s, 1e-3)
    assert mlp.loss_grad(th, X, t, norm)[0] < 0.5 * l0
