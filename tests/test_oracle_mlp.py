"""Pins of the oracle network: GELU against its definition through the normal
CDF, and backward against central finite differences of the loss."""
import math

import numpy as np
from scipy.stats import norm

from oracle import mlp


def small_net(rng, sizes=(5, 7, 6, 3)):
    return [(rng.normal(size=(o, i)) / math.sqrt(i), rng.normal(size=o) * 0.1)
            for i, o in zip(sizes[:-1], sizes[1:])]


def test_gelu_is_z_times_normal_cdf():
    z = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(z), z * norm.cdf(z), rtol=1e-14, atol=1e-15)
    h = 1e-6
    assert np.allclose(mlp.gelu_prime(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), atol=1e-8)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    params = small_net(rng)
    x = rng.normal(size=(9, 5))
    t = rng.normal(size=(9, 3))
    w = np.array([1.0, 0.5, 2.0])
    grads, L = mlp.gradients(params, x, t, w)
    assert np.isclose(L, mlp.loss(params, x, t, w))
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, g in ((W, grads[li][0]), (b, grads[li][1])):
            fd = np.zeros_like(arr)
            for idx in np.ndindex(arr.shape):
                old = arr[idx]
                arr[idx] = old + h
                lp = mlp.loss(params, x, t, w)
                arr[idx] = old - h
                lm = mlp.loss(params, x, t, w)
                arr[idx] = old
                fd[idx] = (lp - lm) / (2 * h)
            assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)
