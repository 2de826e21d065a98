"""Oracle (test infrastructure only): 1D reference-element basis of FR (Section 3).

Solution points are the P+1 Gauss-Legendre nodes of [-1, 1] (the paper does not
name the point set; Gauss points are the reading taken here).  The correction
functions are the left/right Radau polynomials, the choice that makes FR
reproduce nodal DG (Section 3, text after the correction-flux equation).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss_points(P: int):
    """Nodes and weights of the (P+1)-point Gauss-Legendre rule on [-1, 1]."""
    x, w = npleg.leggauss(P + 1)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def lagrange(xs: np.ndarray, t) -> np.ndarray:
    """ell_b(t) for the Lagrange basis on nodes xs: shape (len(t), len(xs))."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(xs)
    out = np.ones((len(t), n))
    for b in range(n):
        for c in range(n):
            if c != b:
                out[:, b] *= (t - xs[c]) / (xs[b] - xs[c])
    return out


def lagrange_deriv(xs: np.ndarray, t) -> np.ndarray:
    """ell_b'(t): product rule on the Lagrange product, shape (len(t), len(xs))."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    n = len(xs)
    out = np.zeros((len(t), n))
    for b in range(n):
        for m in range(n):
            if m == b:
                continue
            term = np.full(len(t), 1.0 / (xs[b] - xs[m]))
            for c in range(n):
                if c != b and c != m:
                    term *= (t - xs[c]) / (xs[b] - xs[c])
            out[:, b] += term
    return out


def diff_matrix(xs: np.ndarray) -> np.ndarray:
    """D[a, b] = ell_b'(x_a): derivative of the interpolant at the nodes."""
    return lagrange_deriv(xs, xs)


def radau_right(P: int, t) -> np.ndarray:
    """g_R(t) = (L_{P+1}(t) + L_P(t)) / 2: g_R(1) = 1, g_R(-1) = 0."""
    c = np.zeros(P + 2)
    c[P + 1] = 0.5
    c[P] += 0.5
    return npleg.legval(np.asarray(t, dtype=np.float64), c)


def radau_right_deriv(P: int, t) -> np.ndarray:
    c = np.zeros(P + 2)
    c[P + 1] = 0.5
    c[P] += 0.5
    return npleg.legval(np.asarray(t, dtype=np.float64), npleg.legder(c))


def radau_left_deriv(P: int, t) -> np.ndarray:
    """g_L(t) = g_R(-t), hence g_L'(t) = -g_R'(-t)."""
    return -radau_right_deriv(P, -np.asarray(t, dtype=np.float64))


class Basis:
    """Everything the 2D tensor-product FR scheme needs from the 1D basis."""

    def __init__(self, P: int):
        self.P = P
        self.n = P + 1
        self.x, self.w = gauss_points(P)
        self.D = diff_matrix(self.x)
        self.lm = lagrange(self.x, -1.0)[0]     # ell_b(-1): extrapolation to the left face
        self.lp = lagrange(self.x, 1.0)[0]      # ell_b(+1): extrapolation to the right face
        self.gLp = radau_left_deriv(P, self.x)  # g_L'(x_a)
        self.gRp = radau_right_deriv(P, self.x)  # g_R'(x_a)
