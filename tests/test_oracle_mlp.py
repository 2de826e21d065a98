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


def _fields(nel=3, Np=2, dt=0.5):
    """Entries that spell out their own position: field f, variable v, element e,
    point k -> 1000 f + 100 v + 10 e + k (Y fields stored times dt)."""
    U = np.empty((4, nel, Np))
    R = np.empty((4, nel, Np))
    Y1 = np.empty((4, nel, Np))
    Y2 = np.empty((4, nel, Np))
    for v in range(4):
        for e in range(nel):
            for k in range(Np):
                base = 100 * v + 10 * e + k
                U[v, e, k] = base
                R[v, e, k] = 1000 + base
                Y1[v, e, k] = (2000 + base) * dt
                Y2[v, e, k] = (3000 + base) * dt
    return U, R, Y1, Y2


def test_features_layout_hand_built():
    """Two elements (taken in the order 2, 0), two points each, identity statistics: row r
    lists field-major, then variable, then point, the raw entries of element elems[r] with
    the increments divided by dt."""
    dt = 0.5
    U, R, Y1, Y2 = _fields(dt=dt)
    ident = [[(0.0, 1.0)] * 4 for _ in range(4)]
    X = mlp.features(U, R, Y1, Y2, dt, np.array([2, 0]), ident)
    assert X.shape == (2, 32)
    row_e2 = [20, 21, 120, 121, 220, 221, 320, 321,
              1020, 1021, 1120, 1121, 1220, 1221, 1320, 1321,
              2020, 2021, 2120, 2121, 2220, 2221, 2320, 2321,
              3020, 3021, 3120, 3121, 3220, 3221, 3320, 3321]
    row_e0 = [0, 1, 100, 101, 200, 201, 300, 301,
              1000, 1001, 1100, 1101, 1200, 1201, 1300, 1301,
              2000, 2001, 2100, 2101, 2200, 2201, 2300, 2301,
              3000, 3001, 3100, 3101, 3200, 3201, 3300, 3301]
    assert np.array_equal(X[0], np.array(row_e2, dtype=float))
    assert np.array_equal(X[1], np.array(row_e0, dtype=float))


def test_features_standardisation_per_field_and_variable():
    """Each (field, variable) group takes its own mean and deviation; None for a previous
    increment means zero, which standardises to -mean/std."""
    dt = 0.25
    U, R, Y1, _ = _fields(nel=2, Np=1, dt=dt)
    stats = [[(10.0 * f + v, 2.0 + f + 0.5 * v) for v in range(4)] for f in range(4)]
    X = mlp.features(U, R, Y1, np.zeros_like(U), dt, np.array([1]), stats)
    # element 1, variable 2, field R: raw 1210, mean 12, std 4
    assert X[0, 4 + 2] == (1210.0 - 12.0) / 4.0
    # element 1, variable 3, field Y1/dt: raw 2310, mean 23, std 5.5
    assert X[0, 8 + 3] == (2310.0 - 23.0) / 5.5
    # field Y2 all zero: -mean/std
    assert X[0, 12 + 1] == -31.0 / 5.5


def test_decode_inverts_the_target_standardisation():
    """decode(y) places output v*Np + k of row b at [v, b, k] and undoes the target
    standardisation t = (Y/dt - mean_v)/std_v exactly for values representable without
    rounding; with unit statistics it is y times dt."""
    Np, dt = 3, 0.5
    stats_out = [(1.0, 2.0), (-3.0, 0.5), (0.0, 4.0), (8.0, 1.0)]
    Y = np.arange(4 * 2 * Np, dtype=float).reshape(4, 2, Np) * dt     # [v, b, k]
    t = np.empty((2, 4 * Np))
    for v in range(4):
        mean, std = stats_out[v]
        t[:, v * Np:(v + 1) * Np] = (Y[v] / dt - mean) / std
    assert np.array_equal(mlp.decode(t, stats_out, dt, Np), Y)
    y = np.array([[1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0, 8.0, 9.0, 10.0, 11.0, 12.0]])
    out = mlp.decode(y, [(0.0, 1.0)] * 4, dt, Np)
    assert out.shape == (4, 1, 3)
    assert np.array_equal(out[:, 0, :], np.array([[0.5, 1.0, 1.5], [2.0, 2.5, 3.0], [3.5, 4.0, 4.5], [5.0, 5.5, 6.0]]))
