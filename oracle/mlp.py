"""Warm-start network in float64: forward pass, gradient of the loss, Adam.

A project addition (not in the paper): a multilayer perceptron maps 32
features of a problem (A, b) to y = ln(1 - sigma_{n+1}^2 / sigma_0^2), the
log of the relative gap between sigma_{n+1}^2 and the least-squares
estimate sigma_0^2 of Algorithm 2's initial step; the solver turns the
prediction into an initial shift.

Network: 32 -> 256 -> 256 -> 256 -> 1, affine layers W h + c with the exact
GELU, GELU(z) = z Phi(z) (Phi the standard normal CDF), after each hidden
layer. Inputs are standardised first, h0 = (x - mu) * s with fixed vectors
mu, s (``norm`` = [mu, s], 64 values). Loss: mean squared error over the
batch, L = (1/B) sum_b (y_b - t_b)^2. Adam as published by Kingma & Ba
(ICLR 2015, Algorithm 1), with bias-corrected moments.

Parameter vector theta (float32 on the device, float64 here): for each
layer in order, W (out x in, row-major) followed by c (out).

Pins (tests/test_oracle_mlp.py): GELU against tabulated values of the normal
CDF, the gradient against central finite differences, Adam's first step
against its closed form, the zero-network special case.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

LAYERS = [(32, 256), (256, 256), (256, 256), (256, 1)]   # (in, out)
N_IN = 32


def param_count() -> int:
    return sum(i * o + o for i, o in LAYERS)


def unpack(theta):
    """[(W, c)] views into theta, W of shape (out, in)."""
    out, off = [], 0
    for i, o in LAYERS:
        W = theta[off:off + i * o].reshape(o, i)
        off += i * o
        c = theta[off:off + o]
        off += o
        out.append((W, c))
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz z Phi(z) = Phi(z) + z phi(z)."""
    Phi = 0.5 * (1.0 + erf(z / math.sqrt(2.0)))
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


def forward(theta, X, norm):
    """y (B,) and the cache of pre-activations and activations."""
    theta = np.asarray(theta, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    norm = np.asarray(norm, dtype=np.float64)
    h = (X - norm[:N_IN]) * norm[N_IN:]
    hs, zs = [h], []
    layers = unpack(theta)
    for li, (W, c) in enumerate(layers):
        z = h @ W.T + c
        zs.append(z)
        h = gelu(z) if li < len(layers) - 1 else z
        hs.append(h)
    return hs[-1][:, 0], (hs, zs)


def loss_grad(theta, X, t, norm):
    """(L, dL/dtheta) for L = mean_b (y_b - t_b)^2, by the chain rule."""
    theta = np.asarray(theta, dtype=np.float64)
    y, (hs, zs) = forward(theta, X, norm)
    t = np.asarray(t, dtype=np.float64)
    B = y.shape[0]
    loss = float(np.mean((y - t) ** 2))
    layers = unpack(theta)
    grads = [None] * len(layers)
    dz = (2.0 / B * (y - t))[:, None]                 # dL/dz of the output layer
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        h_in = hs[li]
        grads[li] = (dz.T @ h_in, dz.sum(axis=0))     # dW (out x in), dc (out)
        if li > 0:
            dz = (dz @ W) * gelu_grad(zs[li - 1])
    g = np.concatenate([np.concatenate([gW.ravel(), gc]) for gW, gc in grads])
    return loss, g


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step = 1, 2, ...): returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
