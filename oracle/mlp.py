"""Two-layer GELU network used as a warm start for CG on the normal equations.

Test infrastructure only (see the package docstring).

The paper has no learned component; this is the float64 reference for the
network the library trains on the GPU.  Shapes (row-major batches):
    X  : B x d_in          input rows
    W1 : h x d_in, b1 : h  first layer
    W2 : d_out x h, b2 : d_out
    A  = X W1^T + b1       pre-activation
    H  = gelu(A)           gelu(a) = a * Phi(a) = a/2 * (1 + erf(a / sqrt 2))
    Yh = H W2^T + b2
Loss (relative mean squared error, averaged over the batch):
    loss = (1/B) sum_b ||Yh_b - T_b||^2 / ||T_b||^2
Adam (Kingma & Ba 2015) with bias correction.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

_SQRT1_2 = 1.0 / math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(a):
    return 0.5 * a * (1.0 + erf(a * _SQRT1_2))


def gelu_grad(a):
    """d gelu / da = Phi(a) + a * phi(a)."""
    return 0.5 * (1.0 + erf(a * _SQRT1_2)) + a * _INV_SQRT_2PI * np.exp(-0.5 * a * a)


def forward(params, X):
    W1, b1, W2, b2 = params
    A = X @ W1.T + b1[None, :]
    H = gelu(A)
    Y = H @ W2.T + b2[None, :]
    return Y, (X, A, H)


def loss(Y, T):
    """Relative MSE averaged over rows."""
    num = np.sum((Y - T) ** 2, axis=1)
    den = np.sum(T * T, axis=1)
    return float(np.mean(num / den))


def backward(params, cache, Y, T):
    """Gradients of `loss` w.r.t. (W1, b1, W2, b2)."""
    W1, b1, W2, b2 = params
    X, A, H = cache
    B = X.shape[0]
    den = np.sum(T * T, axis=1)
    dY = (2.0 / B) * (Y - T) / den[:, None]
    dW2 = dY.T @ H
    db2 = dY.sum(axis=0)
    dH = dY @ W2
    dA = dH * gelu_grad(A)
    dW1 = dA.T @ X
    db1 = dA.sum(axis=0)
    return dW1, db1, dW2, db2


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
