"""Plain FP64 reference of the surrogate network (test infrastructure).

A fully connected network x -> W_L gelu(... gelu(W_0 x + b_0) ...) + b_L with
the exact GELU, z Phi(z) = z/2 (1 + erf(z / sqrt 2)), evaluated on normalized
inputs and producing normalized outputs; the loss is the weighted mean squared
error L = (1/B) sum_r sum_j w_j (yhat_rj - t_rj)^2. Backward is the chain rule
written out layer by layer. Pinned by central finite differences of L.
"""
import math

import numpy as np
from scipy.special import erf

SQ2 = math.sqrt(2.0)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQ2))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / SQ2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params, x):
    """params: list of (W [out, in], b [out]); x: (B, in). Returns output and the
    pre-activations of every layer."""
    a = x
    zs = []
    for i, (W, b) in enumerate(params):
        z = a @ W.T + b
        zs.append(z)
        a = gelu(z) if i < len(params) - 1 else z
    return a, zs


def loss(params, x, t, w):
    y, _ = forward(params, x)
    return float((w[None, :] * (y - t) ** 2).sum() / x.shape[0])


def gradients(params, x, t, w):
    """dL/dW, dL/db for every layer, and L."""
    y, zs = forward(params, x)
    B = x.shape[0]
    L = float((w[None, :] * (y - t) ** 2).sum() / B)
    dz = 2.0 * w[None, :] * (y - t) / B
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        a_in = x if i == 0 else gelu(zs[i - 1])
        grads[i] = (dz.T @ a_in, dz.sum(axis=0))
        if i > 0:
            da = dz @ W
            dz = da * gelu_prime(zs[i - 1])
    return grads, L
