"""Oracle (test infrastructure only): FR/CPR residual R(q) of the 2D Euler
equations, dq/dt = R(q) (Section 3 and Section 4, eq. simplified_ode).

Per element, in reference coordinates:

  R = -(1/|J|) [ dF^l/dxi + (F^num - F^l)|_{xi=-1} g_L'(xi) + (F^num - F^l)|_{xi=+1} g_R'(xi)
                 + the same in eta with G ]

(eq. discrete_ns with the correction flux of Section 3), where F^l is the
Lagrange interpolant of the transformed flux F = |J|(f xi_x + g xi_y) through
the solution points, F^l at a face is that interpolant evaluated there, and
F^num = |J||grad xi| f_n^com (eq. norm_num_f) is the common flux in the face's
+xi (or +eta) direction.  The common flux f_n^com is either the Roe flux
(eq. invis_com) or the Rusanov flux (used by the 2D Euler workloads).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry


# ---------------------------------------------------------------- physics (Section 2)

def pressure(q, gamma):
    """Ideal gas: E = p/(gamma-1) + rho |u|^2 / 2."""
    rho, mx, my, E = q
    return (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / rho)


def physical_flux(q, gamma):
    """Inviscid fluxes f (x) and g (y) of q = (rho, rho u, rho v, E) (Section 2)."""
    rho, mx, my, E = q
    u = mx / rho
    v = my / rho
    p = pressure(q, gamma)
    f = np.stack([mx, mx * u + p, my * u, u * (E + p)])
    g = np.stack([my, mx * v, my * v + p, v * (E + p)])
    return f, g


def normal_flux(q, nx, ny, gamma):
    f, g = physical_flux(q, gamma)
    return f * nx + g * ny


def rusanov(qL, qR, nx, ny, gamma):
    """Local Lax-Friedrichs flux along the unit normal (nx, ny):
    (f_n(L) + f_n(R))/2 - lambda (qR - qL)/2 with lambda = max(|u_n| + c) over both sides."""
    fL = normal_flux(qL, nx, ny, gamma)
    fR = normal_flux(qR, nx, ny, gamma)
    lam = np.maximum(_speed(qL, nx, ny, gamma), _speed(qR, nx, ny, gamma))
    return 0.5 * (fL + fR) - 0.5 * lam * (qR - qL)


def _speed(q, nx, ny, gamma):
    rho = q[0]
    un = (q[1] * nx + q[2] * ny) / rho
    c = np.sqrt(gamma * pressure(q, gamma) / rho)
    return np.abs(un) + c


def roe(qL, qR, nx, ny, gamma):
    """Roe flux (eq. invis_com): (f_n(L) + f_n(R))/2 - R|Lambda|R^{-1}(qR - qL)/2,
    eigen-system of d f_n / d q at the Roe average; no entropy fix (none is stated)."""
    fL = normal_flux(qL, nx, ny, gamma)
    fR = normal_flux(qR, nx, ny, gamma)
    rL, rR = qL[0], qR[0]
    uL, vL, uR, vR = qL[1] / rL, qL[2] / rL, qR[1] / rR, qR[2] / rR
    pL, pR = pressure(qL, gamma), pressure(qR, gamma)
    HL, HR = (qL[3] + pL) / rL, (qR[3] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    rho = sL * sR
    u = (sL * uL + sR * uR) / (sL + sR)
    v = (sL * vL + sR * vR) / (sL + sR)
    H = (sL * HL + sR * HR) / (sL + sR)
    q2 = u * u + v * v
    c = np.sqrt((gamma - 1.0) * (H - 0.5 * q2))
    un = u * nx + v * ny
    ut = -u * ny + v * nx
    dr = rR - rL
    dp = pR - pL
    dun = (uR - uL) * nx + (vR - vL) * ny
    dut = -(uR - uL) * ny + (vR - vL) * nx
    # wave strengths and right eigenvectors: acoustic (un -+ c), entropy, shear (un)
    a1 = (dp - rho * c * dun) / (2.0 * c * c)
    a2 = dr - dp / (c * c)
    a3 = rho * dut
    a4 = (dp + rho * c * dun) / (2.0 * c * c)
    one = np.ones_like(u)
    zero = np.zeros_like(u)
    r1 = np.stack([one, u - c * nx, v - c * ny, H - un * c])
    r2 = np.stack([one, u, v, 0.5 * q2])
    r3 = np.stack([zero, -ny * one, nx * one, ut])
    r4 = np.stack([one, u + c * nx, v + c * ny, H + un * c])
    diss = (np.abs(un - c) * a1 * r1 + np.abs(un) * a2 * r2 + np.abs(un) * a3 * r3
            + np.abs(un + c) * a4 * r4)
    return 0.5 * (fL + fR) - 0.5 * diss


FLUXES = {"rusanov": rusanov, "roe": roe}


def face_flux(qL, qR, S, gamma, flux):
    """F^num = |S| f^com(qL, qR, S/|S|) for the area-weighted normal S (eq. norm_num_f);
    qL is the state on the side S points away from."""
    mag = np.sqrt(S[0] ** 2 + S[1] ** 2)
    return mag * FLUXES[flux](qL, qR, S[0] / mag, S[1] / mag, gamma)


# ---------------------------------------------------------------- FR residual (Section 3)

class EulerFR:
    def __init__(self, geo: Geometry, gamma: float = 1.4, flux: str = "rusanov"):
        self.geo = geo
        self.b = geo.basis
        self.mesh = geo.mesh
        self.gamma = gamma
        self.flux = flux
        self.n = self.b.n
        self.nel = self.mesh.nel
        self.ndof = 4 * self.nel * self.n * self.n

    def shape(self, U):
        return np.asarray(U, dtype=np.float64).reshape(4, self.nel, self.n, self.n)

    def transformed_flux(self, q):
        """F = y_eta f - x_eta g and G = -y_xi f + x_xi g at solution points."""
        geo = self.geo
        f, g = physical_flux(q, self.gamma)
        F = geo.y_eta * f - geo.x_eta * g
        G = -geo.y_xi * f + geo.x_xi * g
        return F, G

    def traces(self, q):
        """Solution traces on the four faces: W, E indexed [v, e, b]; S, N indexed [v, e, a]."""
        lm, lp = self.b.lm, self.b.lp
        return {"W": np.einsum("a,veba->veb", lm, q), "E": np.einsum("a,veba->veb", lp, q),
                "S": np.einsum("b,veba->vea", lm, q), "N": np.einsum("b,veba->vea", lp, q)}

    def neighbour_traces(self, tr):
        """For each element, the neighbour's trace on each shared face."""
        m = self.mesh
        return {"W": tr["E"][:, m.west], "E": tr["W"][:, m.east],
                "S": tr["N"][:, m.south], "N": tr["S"][:, m.north]}

    def residual_given_neighbours(self, q, nbr):
        """Element-local residual: own state q, neighbours' face traces nbr held fixed."""
        b, geo, gam = self.b, self.geo, self.gamma
        F, G = self.transformed_flux(q)
        tr = self.traces(q)
        FW = np.einsum("a,veba->veb", b.lm, F)
        FE = np.einsum("a,veba->veb", b.lp, F)
        GS = np.einsum("b,veba->vea", b.lm, G)
        GN = np.einsum("b,veba->vea", b.lp, G)
        # common fluxes; left/lower state first, normal pointing to +xi / +eta
        FnW = face_flux(nbr["W"], tr["W"], geo.SW, gam, self.flux)
        FnE = face_flux(tr["E"], nbr["E"], geo.SE, gam, self.flux)
        GnS = face_flux(nbr["S"], tr["S"], geo.SS, gam, self.flux)
        GnN = face_flux(tr["N"], nbr["N"], geo.SN, gam, self.flux)
        div = (np.einsum("ac,vebc->veba", b.D, F)
               + (FnW - FW)[:, :, :, None] * b.gLp[None, None, None, :]
               + (FnE - FE)[:, :, :, None] * b.gRp[None, None, None, :]
               + np.einsum("bc,veca->veba", b.D, G)
               + (GnS - GS)[:, :, None, :] * b.gLp[None, None, :, None]
               + (GnN - GN)[:, :, None, :] * b.gRp[None, None, :, None])
        return -div / geo.J[None]

    def local_residual_factory(self, U):
        """R_e as a function of the element's own state, the neighbours held at U: for the
        Euler residual they enter only through their solution traces on the shared faces."""
        nbr = self.neighbour_traces(self.traces(self.shape(U)))
        return lambda q: self.residual_given_neighbours(q, nbr)

    def residual(self, U):
        """R(q) for the whole mesh; U and the result in [v, e, k] layout (flattened)."""
        q = self.shape(U)
        nbr = self.neighbour_traces(self.traces(q))
        return self.residual_given_neighbours(q, nbr).reshape(np.shape(U))
