"""The 512-256-256-1 GELU surrogate of log pi, its backward pass and Adam, FP64.

Test infrastructure only (see ``oracle/__init__.py``).

The paper has no surrogate; this is the learned-part extension.  Layout:
inputs are standardised, xs = (x - in_mean) * in_scale, then
h1 = gelu(W1 xs + b1), h2 = gelu(W2 h1 + b2), out = W3 h2 + b3, and the
surrogate log-density is out * out_std + out_mean.  Weights Wk are
(fan_out, fan_in); batches are columns (d x n).  GELU is exact,
gelu(a) = a Phi(a) with Phi the standard normal CDF via erf.  The loss is
the mean squared error over the batch, L = mean_j (out_j - t_j)^2.
Pinned by central finite differences (gradients), by scipy's normal CDF
(GELU) and by the closed form of Adam's first step.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT1_2 = 1.0 / math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)

LAYERS = (512, 256, 256, 1)


def gelu(a):
    return a * 0.5 * (1.0 + erf(a * SQRT1_2))


def gelu_grad(a):
    return 0.5 * (1.0 + erf(a * SQRT1_2)) + a * INV_SQRT_2PI * np.exp(-0.5 * a * a)


def forward(params, Xs):
    """params = [W1, b1, W2, b2, W3, b3]; Xs standardised inputs (d x n).
    Returns (out (n,), cache)."""
    W1, b1, W2, b2, W3, b3 = params
    a1 = W1 @ Xs + b1[:, None]
    h1 = gelu(a1)
    a2 = W2 @ h1 + b2[:, None]
    h2 = gelu(a2)
    out = (W3 @ h2 + b3[:, None])[0]
    return out, (Xs, a1, h1, a2, h2)


def loss_and_grad(params, Xs, t):
    """MSE loss and its gradient w.r.t. every parameter (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = params
    out, (Xs, a1, h1, a2, h2) = forward(params, Xs)
    n = out.size
    r = out - t
    loss = float(np.mean(r * r))
    g_out = (2.0 / n) * r[None, :]                  # 1 x n
    gW3 = g_out @ h2.T
    gb3 = g_out.sum(axis=1)
    g_h2 = W3.T @ g_out
    g_a2 = g_h2 * gelu_grad(a2)
    gW2 = g_a2 @ h1.T
    gb2 = g_a2.sum(axis=1)
    g_h1 = W2.T @ g_a2
    g_a1 = g_h1 * gelu_grad(a1)
    gW1 = g_a1 @ Xs.T
    gb1 = g_a1.sum(axis=1)
    return loss, [gW1, gb1, gW2, gb2, gW3, gb3]


def adam_step(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba 2015), bias-corrected; step counts from 1."""
    out_p, out_m, out_v = [], [], []
    c1 = 1.0 - b1 ** step
    c2 = 1.0 - b2 ** step
    for p, g, mm, vv in zip(params, grads, m, v):
        mm = b1 * mm + (1.0 - b1) * g
        vv = b2 * vv + (1.0 - b2) * g * g
        p = p - lr * (mm / c1) / (np.sqrt(vv / c2) + eps)
        out_p.append(p)
        out_m.append(mm)
        out_v.append(vv)
    return out_p, out_m, out_v


def he_init(seed, layers=LAYERS):
    """He-normal weights N(0, 2/fan_in), zero biases (the surrogate's init)."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(layers[:-1], layers[1:]):
        params.append(rng.standard_normal((fo, fi)) * math.sqrt(2.0 / fi))
        params.append(np.zeros(fo))
    return params


def round_bf16(a):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
