"""Oracle (test infrastructure only): the matrix-free LU-SGS preconditioner that Section
4.5 names beside element-Jacobi (the paper's results use element-Jacobi only).

A = shift I - dR/dq is split by element blocks into D + L + U, the elements ordered by
colour: on the doubly periodic structured mesh with even nx and ny the checkerboard
colouring (ex + ey even: colour 0, "red"; odd: colour 1, "black") leaves no two
elements of one colour coupled, because the Euler FR residual of an element depends on
its own state and its four face neighbours' only.  Red first, then black: L holds the
black rows' couplings to red elements, U the red rows' couplings to black ones.  The
symmetric Gauss-Seidel preconditioner M = (D + L) D^{-1} (D + U) is applied as

    forward   y_R = D_R^{-1} r_R,            y_B = D_B^{-1} (r_B - A_BR y_R),
    backward  z_B = y_B,                     z_R = y_R - D_R^{-1} A_RB z_B,

with D the element blocks (the element-Jacobi blocks) and the off-diagonal products
matrix-free: A_BR y_R is the black part of A applied to y with its black part zero,
i.e. of the Jacobian-free product [Section 4.5] of that vector.
"""
from __future__ import annotations

import numpy as np

from . import linear


def colours(mesh):
    """Colour of every element: (ex + ey) mod 2."""
    e = np.arange(mesh.nel)
    return ((e % mesh.nx) + (e // mesh.nx)) % 2


class LUSGS:
    """Matrix-free LU-SGS preconditioner at state U with shift s (apply(r) = M^{-1} r)."""

    def __init__(self, op, U, shift, residual=None, eps=linear.JF_EPS, eps_mode="rms"):
        m = op.mesh
        if m.nx % 2 or m.ny % 2:
            raise ValueError("LU-SGS with two colours needs even nx and ny")
        self.op = op
        self.U = U
        self.shift = shift
        self.R = residual if residual is not None else op.residual
        self.R0 = self.R(U)
        self.eps, self.eps_mode = eps, eps_mode
        self.blocks = linear.ejacobi_blocks(op, U, shift)
        c = colours(m)
        Np = op.n * op.n
        # masks over the [v, e, k] layout
        self.red = np.broadcast_to((c == 0)[None, :, None], (4, op.nel, Np)).reshape(np.shape(U))
        self.black = ~self.red

    def _A(self, v):
        return linear.jf_matvec(self.R, self.U, self.R0, v, self.shift, self.eps, self.eps_mode)

    def _Dinv(self, r, mask):
        """D^{-1} r on the elements of one colour, zero elsewhere."""
        return np.where(mask, linear.ejacobi_apply(self.op, self.blocks, np.where(mask, r, 0.0)), 0.0)

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64)
        red, black = self.red, self.black
        y = self._Dinv(r, red)                                  # y_R, y_B = 0
        y = y + self._Dinv(r - self._A(y), black)               # y_B = D_B^{-1}(r_B - A_BR y_R)
        zB = np.where(black, y, 0.0)
        return np.where(red, y - self._Dinv(self._A(zB), red), y)   # z_R = y_R - D_R^{-1} A_RB z_B


def lusgs_dense(A, blocks, order_red, nb):
    """The same preconditioner from an explicit matrix (tests): A in the [v, e, k] ordering,
    blocks[e] the element blocks, order_red[e] True for red elements; returns M^{-1} as a
    function.  M = (D + L) D^{-1} (D + U) with L / U the couplings of black rows to red
    columns / red rows to black columns."""
    n = A.shape[0]
    nel = len(order_red)
    Np = nb // 4
    # element of every dof in the [v, e, k] ordering
    el = (np.arange(n) // Np) % nel
    red = order_red[el]
    D = np.zeros_like(A)
    for e in range(nel):
        idx = np.array([v * nel * Np + e * Np + k for v in range(4) for k in range(Np)])
        D[np.ix_(idx, idx)] = blocks[e]
    Off = A - D
    L = np.where(np.outer(~red, red), Off, 0.0)
    U = np.where(np.outer(red, ~red), Off, 0.0)
    M = (D + L) @ np.linalg.solve(D, D + U)
    return lambda r: np.linalg.solve(M, np.asarray(r).reshape(-1)).reshape(np.shape(r))
