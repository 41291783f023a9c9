"""Plain float64 reference of the learned chunk predictor and its training step.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The predictor proposes the whole chunk's initial Newton iterate.  It is a
fully connected network x -> GELU(W1 x + b1) -> GELU(W2 . + b2) -> W3 . + b3
with x = [y_s, t_s, log dt] (standardised by fixed input statistics) and
output the m x n average slopes s_j, from which dy0_j = (t_{s+j} - t_s) s_j.
GELU is the exact form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.

Training minimises the mean squared error between predicted and observed
slopes with Adam (Kingma and Ba, 2015: bias-corrected first and second
moment estimates).  Parameters are packed as W1[H][n_in], b1[H], W2[H][H],
b2[H], W3[n_out][H], b3[n_out].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def sizes(n_in, hidden, n_out):
    return [hidden * n_in, hidden, hidden * hidden, hidden, n_out * hidden, n_out]


def unpack(theta, n_in, hidden, n_out):
    parts = np.split(np.asarray(theta, dtype=np.float64), np.cumsum(sizes(n_in, hidden, n_out))[:-1])
    W1, b1, W2, b2, W3, b3 = parts
    return W1.reshape(hidden, n_in), b1, W2.reshape(hidden, hidden), b2, W3.reshape(n_out, hidden), b3


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(theta, x, n_in, hidden, n_out):
    """Outputs [M, n_out] and the pre-activations needed by the backward pass."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    a1 = gelu(z1)
    z2 = a1 @ W2.T + b2
    a2 = gelu(z2)
    out = a2 @ W3.T + b3
    return out, (x, z1, a1, z2, a2)


def loss_and_grad(theta, x, target, n_in, hidden, n_out):
    """L = mean over samples and outputs of (out - target)^2 and dL/dtheta."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, hidden, n_out)
    out, (x, z1, a1, z2, a2) = forward(theta, x, n_in, hidden, n_out)
    M = x.shape[0]
    diff = out - np.asarray(target, dtype=np.float64)
    L = np.mean(diff ** 2)
    d3 = 2.0 * diff / (M * n_out)
    gW3 = d3.T @ a2
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3) * gelu_grad(z2)
    gW2 = d2.T @ a1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * gelu_grad(z1)
    gW1 = d1.T @ x
    gb1 = d1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, grad


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
