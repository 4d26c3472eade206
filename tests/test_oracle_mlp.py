"""Pins of the FP64 surrogate-network oracle (no GPU)."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_values_and_identities():
    """GELU(0) = 0, GELU(z) - GELU(-z) = z (odd part of z Phi(z)), GELU -> z
    for large z and -> 0 for very negative z; GELU(1) = Phi(1) = 0.8413447."""
    z = np.linspace(-6, 6, 101)
    assert mlp.gelu(0.0) == 0.0
    assert np.allclose(mlp.gelu(z) - mlp.gelu(-z), z, atol=1e-15)
    assert mlp.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-14)
    assert mlp.gelu(30.0) == pytest.approx(30.0, rel=1e-15)
    assert abs(mlp.gelu(-30.0)) < 1e-150


def test_gelu_grad_is_the_derivative():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-9)


def test_backward_matches_finite_differences():
    """Central differences on a narrow network: every parameter."""
    dims = [5, 7, 6, 4]
    rng = np.random.default_rng(3)
    p = mlp.init_params(dims, 1) + 0.1 * rng.standard_normal(mlp.flatten(mlp.unflatten(
        mlp.init_params(dims, 1), dims)).size)
    x = rng.standard_normal((9, 5))
    t = rng.standard_normal((9, 4))
    _, g = mlp.loss_and_grads(p, dims, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (mlp.loss_and_grads(p + e, dims, x, t)[0] - mlp.loss_and_grads(p - e, dims, x, t)[0]) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_adamw_first_step_closed_form():
    """At step 1 the bias-corrected moments are m = g and v = g^2, so the
    update is -lr (sign(g) g/(|g| + eps) + wd w) on weights, no decay on biases."""
    dims = [3, 2]
    w = np.array([0.5, -1.0, 2.0, 0.25, 0.0, -3.0, 0.1, 0.2])   # W (2x3) then b (2)
    g = np.array([0.3, -0.2, 1e-3, 5.0, -7.0, 0.0, -0.4, 0.6])
    new, m, v = mlp.adamw(w, g, np.zeros_like(w), np.zeros_like(w), 1, dims, lr=0.01, b1=0.9, b2=0.999,
                          eps=1e-8, wd=0.1)
    decay = np.array([0.1] * 6 + [0.0] * 2)
    want = w - 0.01 * (g / (np.abs(g) + 1e-8) + decay * w)
    assert np.allclose(new, want, rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_default_network_size():
    dims = [5, 512, 512, 512, 512, 258]
    n = sum(dims[l] * dims[l + 1] + dims[l + 1] for l in range(len(dims) - 1))
    assert n == 923394
    assert mlp.init_params(dims, 0).size == n
