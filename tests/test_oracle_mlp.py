"""Pins of the oracle MLP: bf16 rounding against torch's conversion, gelu and its
derivative, gradients against central differences, Adam's first step, and the
zero network."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-5, 5, 5000),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38])])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_gelu_and_derivative():
    z = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(z), 0.5 * z * (1 + np.array([math.erf(t / math.sqrt(2)) for t in z])), atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, atol=1e-8)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0 and abs(mlp.gelu(np.array([30.0]))[0] - 30.0) < 1e-12


def test_gradients_match_central_differences():
    p = mlp.init_params(12, 10, 6, seed=1)
    for k in p:
        if k.startswith("b"):
            p[k] = np.random.default_rng(2).standard_normal(p[k].shape) * 0.1
    rng = np.random.default_rng(3)
    X = rng.standard_normal((7, 12))
    T = rng.standard_normal((7, 6))
    y, cache = mlp.forward(p, X, emulate_bf16=False)
    g = mlp.backward(p, cache, y, T, emulate_bf16=False)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.mse(mlp.forward(p, X, False)[0], T)
            flat[idx] = old - h
            lm = mlp.mse(mlp.forward(p, X, False)[0], T)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(g[k].reshape(-1)[idx] - fd) <= 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_zero_network_returns_zero_guess():
    p = mlp.init_params(16, 8, 4, seed=0)
    for k in p:
        p[k][...] = 0.0
    y, _ = mlp.forward(p, np.random.default_rng(0).standard_normal((5, 16)))
    assert np.array_equal(y, np.zeros((5, 4)))
    stats_out = [(0.0, 1.0)] * 4
    assert np.array_equal(mlp.decode(np.zeros((3, 8)), stats_out, 0.1, 2), np.zeros((4, 3, 2)))


def test_adam_first_step_is_lr_sign():
    p = {"W": np.array([0.5, -0.2, 0.0])}
    g = {"W": np.array([2.0, -3.0, 1e-3])}
    mlp.adam_step(p, g, {}, lr=0.01)
    # first step: m_hat = g, v_hat = g^2 -> update lr * g / (|g| + eps)
    assert np.allclose(p["W"], [0.49, -0.19, -0.01 * 1e-3 / (1e-3 + 1e-8)], atol=1e-12)
