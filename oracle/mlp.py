"""Oracle (test infrastructure only): the per-element MLP that predicts the GMRES
initial guess of a stage increment (a learned warm start added on top of the
paper's method; the paper's own initial guess is zero).

Input per element: the element's entries of [U, R(U), Y_{i-1}/dt, Y_{i-2}/dt]
(field-major, then variable, then solution point), each (field, variable)
standardised with training-set mean and deviation; output: the element's
entries of Y_i/dt, standardised per variable.

Network: h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2), y = W3 h2 + b3 with the
exact gelu(z) = z (1 + erf(z/sqrt 2)) / 2.  Precision model of the kernels:
weights, layer inputs and hidden activations rounded to bfloat16
(round-to-nearest-even), products accumulated exactly here (FP32 on the GPU),
biases and the output in FP32.  Loss: mean squared error.  Optimiser: Adam.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through float32, returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init_params(n_in, n_hidden, n_out, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, (o, i) in (("1", (n_hidden, n_in)), ("2", (n_hidden, n_hidden)), ("3", (n_out, n_hidden))):
        lim = 1.0 / math.sqrt(i)
        p["W" + name] = rng.uniform(-lim, lim, size=(o, i))
        p["b" + name] = np.zeros(o)
    return p


def forward(p, X, emulate_bf16=True):
    """X: [batch, n_in] standardised features.  Returns (y, cache)."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    rf32 = (lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)) if emulate_bf16 else r
    x = r(X)
    z1 = rf32(x @ r(p["W1"]).T + rf32(p["b1"]))
    h1 = r(gelu(z1))
    z2 = rf32(h1 @ r(p["W2"]).T + rf32(p["b2"]))
    h2 = r(gelu(z2))
    y = rf32(h2 @ r(p["W3"]).T + rf32(p["b3"]))
    return y, (x, z1, h1, z2, h2)


def mse(y, t):
    return float(np.mean((y - t) ** 2))


def backward(p, cache, y, t, emulate_bf16=True):
    """Gradients of the mean squared error; the backward operands are rounded to
    bfloat16 where the kernels round them (the output error and the hidden-layer
    gradients as operands of the weight-gradient and back-propagation products).  The
    bias gradients are sums of the same gradients before that rounding."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x, z1, h1, z2, h2 = cache
    B = y.shape[0]
    dy = 2.0 * (y - t) / y.size
    g = {}
    dyr = r(dy)
    g["W3"] = dyr.T @ h2
    g["b3"] = dy.sum(axis=0)
    dh2 = dyr @ r(p["W3"])
    dz2 = r(dh2 * gelu_grad(z2))
    g["W2"] = dz2.T @ h1
    g["b2"] = (dh2 * gelu_grad(z2)).sum(axis=0)
    dh1 = dz2 @ r(p["W2"])
    dz1 = r(dh1 * gelu_grad(z1))
    g["W1"] = dz1.T @ x
    g["b1"] = (dh1 * gelu_grad(z1)).sum(axis=0)
    return g


def adam_step(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of every parameter in place; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m" + k, np.zeros_like(p[k]))
        v = state.setdefault("v" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def features(U, R, Y1, Y2, dt, elems, stats_in):
    """Standardised [len(elems), 4 * 4 * Np] features; fields in [v, e, k] layout."""
    cols = []
    for f, a in enumerate((U, R, np.asarray(Y1) / dt, np.asarray(Y2) / dt)):
        for v in range(4):
            mean, std = stats_in[f][v]
            cols.append((np.asarray(a)[v][elems] - mean) / std)
    return np.concatenate(cols, axis=1)


def decode(y, stats_out, dt, Np):
    """Network output [batch, 4 * Np] -> increments [4, batch, Np] (times dt)."""
    out = np.empty((4, y.shape[0], Np))
    for v in range(4):
        mean, std = stats_out[v]
        out[v] = (y[:, v * Np:(v + 1) * Np] * std + mean) * dt
    return out
