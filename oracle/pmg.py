"""Oracle (test infrastructure only): the p-multigrid preconditioner that Section 4.5
names beside element-Jacobi (the paper's results use element-Jacobi only).

Two levels on one mesh: the fine discretisation of degree P and a coarse one of degree
Pc < P, each with its own FR residual (rediscretisation) and element-Jacobi blocks.
Transfers between the nodal (Gauss-point) bases, per element and variable, as tensor
products of 1D operators:
  restriction  Pi = L2 projection onto degree Pc: (Pi f)_a = (1/w^c_a) sum_b w_b l^c_a(x_b) f_b,
               exact with the fine Gauss rule (degree Pc + P <= 2P + 1);
  prolongation I  = interpolation of the coarse polynomial at the fine points: I_ba = l^c_a(x_b).
The coarse state is Pi U, the coarse shift the fine one.  One application of the
preconditioner (a V-cycle, smoothers: block Jacobi with the element blocks):
  z  = D^{-1} r,                       then nu1 - 1 more sweeps z += D^{-1}(r - A z);
  rc = Pi (r - A z);  zc = Dc^{-1} rc, then nc - 1 sweeps zc += Dc^{-1}(rc - Ac zc);
  z += I zc;                           then nu2 sweeps z += D^{-1}(r - A z).
A and Ac are the Jacobian-free products (Section 4.5) of the two levels.
"""
from __future__ import annotations

import numpy as np

from . import linear
from .basis import gauss_points, lagrange


def transfer_1d(P, Pc):
    """(Pi, I): the 1D restriction ((Pc+1) x (P+1)) and prolongation ((P+1) x (Pc+1))."""
    xf, wf = gauss_points(P)
    xc, wc = gauss_points(Pc)
    Lc = lagrange(xc, xf)                 # Lc[b, a] = l^c_a(x_b)
    Pi = (Lc * wf[:, None]).T / wc[:, None]
    return Pi, Lc


def apply_2d(T, v, nel, n_in):
    """Per element and variable, the tensor product T (x) T on a [v, e, k] vector
    (k = b n + a, a along xi)."""
    q = np.asarray(v).reshape(4, nel, n_in, n_in)          # [v, e, b, a]
    out = np.einsum("ib,jc,vebc->veij", T, T, q)
    n_out = T.shape[0]
    return out.reshape(4, nel, n_out * n_out)


class PMultigrid:
    """Two-level p-multigrid preconditioner at state U with shift s (apply(r) = M^{-1} r)."""

    def __init__(self, op, op_c, U, shift, nu1=1, nu2=1, nc=2, eps=linear.JF_EPS, eps_mode="rms"):
        self.op, self.op_c = op, op_c
        self.P, self.Pc = op.n - 1, op_c.n - 1
        if not self.Pc < self.P:
            raise ValueError("the coarse degree must be below the fine one")
        self.Pi, self.I = transfer_1d(self.P, self.Pc)
        self.nel = op.nel
        self.shape_f = np.shape(U)
        self.U = np.asarray(U, dtype=np.float64)
        self.Uc = self.restrict(self.U)
        self.shift = shift
        self.nu1, self.nu2, self.nc = nu1, nu2, nc
        self.eps, self.eps_mode = eps, eps_mode
        self.R0 = op.residual(self.U)
        self.R0c = op_c.residual(self.Uc)
        self.D = linear.ElementJacobi(op, self.U, shift)
        self.Dc = linear.ElementJacobi(op_c, self.Uc, shift)

    def restrict(self, v):
        return apply_2d(self.Pi, v, self.nel, self.P + 1)

    def prolong(self, vc):
        return apply_2d(self.I, vc, self.nel, self.Pc + 1).reshape(self.shape_f)

    def A(self, v):
        return linear.jf_matvec(self.op.residual, self.U, self.R0, v, self.shift, self.eps, self.eps_mode)

    def Ac(self, v):
        return linear.jf_matvec(self.op_c.residual, self.Uc, self.R0c, v, self.shift, self.eps, self.eps_mode)

    def apply(self, r):
        r = np.asarray(r, dtype=np.float64).reshape(self.shape_f)
        z = self.D.apply(r)
        for _ in range(self.nu1 - 1):
            z = z + self.D.apply(r - self.A(z))
        rc = self.restrict(r - self.A(z))
        zc = self.Dc.apply(rc)
        for _ in range(self.nc - 1):
            zc = zc + self.Dc.apply(rc - self.Ac(zc))
        z = z + self.prolong(zc)
        for _ in range(self.nu2):
            z = z + self.D.apply(r - self.A(z))
        return z
