"""Oracle (test infrastructure only): FR on hexahedra (Section 3, the hexahedral forms of
the transformed fluxes and correction fluxes) for the 3D compressible Navier-Stokes
equations, restricted to uniform Cartesian elements of a triply periodic box (the
Taylor-Green vortex of Section 5.3), with the BR2 common gradient of the paper.

Element e = (ez ny + ey) nx + ex of size hx x hy x hz, solution points on the tensor
Gauss grid, point k = (c n + b) n + a (a along x, b along y, c along z); state
q = (rho, rho u, rho v, rho w, E) in [v, e, c, b, a] layout.  The map is affine, so
xi_x = 2/hx etc. are constant and the FR residual is, per direction d with h_d:

  R = -sum_d (2/h_d) [ D f_d + (f^com_- - f^l_-) g_L' + (f^com_+ - f^l_+) g_R' ]

with f_d = f_inv,d - f_vis,d at the solution points, f^l_+- its interpolant at the two
faces normal to d and f^com the common normal flux there (the Riemann solver between
the two traces minus the viscous flux at the common state and common gradient).

Gradients: inside the element (for the viscous flux at the solution points) the
FR-corrected gradient dq/dx_d = (2/h_d)[D q + (q^com_- - q_-) g_L' + (q^com_+ - q_+) g_R'];
on a face the BR2 common gradient ((grad q^- + r^-) + (grad q^+ + r^+)) / 2 with the raw
gradient of each side's polynomial extrapolated to the face and r = c_P (q^com - q_local)
(2/h_d) n_out, c_P = (P+1)(P+2)/2 (the readings of the 2D module, oracle/ns_bc.py).
"""
from __future__ import annotations

import numpy as np

from .basis import Basis


def pressure(q, gamma):
    rho, mx, my, mz, E = q
    return (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / rho)


def inviscid_flux(q, d, gamma):
    """Flux along axis d (0, 1, 2) of q = (rho, rho u, rho v, rho w, E)."""
    rho = q[0]
    vel = q[1 + d] / rho
    p = pressure(q, gamma)
    f = [q[1 + d], q[1] * vel, q[2] * vel, q[3] * vel, vel * (q[4] + p)]
    f[1 + d] = f[1 + d] + p
    return np.stack(f)


def viscous_flux(q, grad, d, gamma, rgas, mu, prandtl):
    """Viscous flux along axis d (Section 2 in 3D): Stokes stress with zero bulk viscosity,
    Fourier heat flux kappa = mu Cp / Pr; grad[k] is dq/dx_k."""
    rho = q[0]
    u = [q[1 + i] / rho for i in range(3)]
    du = [[(grad[k][1 + i] - u[i] * grad[k][0]) / rho for k in range(3)] for i in range(3)]   # du_i/dx_k
    ke = 0.5 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    p = (gamma - 1.0) * (q[4] - rho * ke)
    T = p / (rho * rgas)
    dp = [(gamma - 1.0) * (grad[k][4] - ke * grad[k][0] - rho * (u[0] * du[0][k] + u[1] * du[1][k] + u[2] * du[2][k]))
          for k in range(3)]
    dT = [(dp[k] - rgas * T * grad[k][0]) / (rho * rgas) for k in range(3)]
    div = du[0][0] + du[1][1] + du[2][2]
    tau = [mu * (du[i][d] + du[d][i] - (2.0 / 3.0 if i == d else 0.0) * div) for i in range(3)]
    kappa = mu * (gamma * rgas / (gamma - 1.0)) / prandtl
    energy = u[0] * tau[0] + u[1] * tau[1] + u[2] * tau[2] + kappa * dT[d]
    return np.stack([np.zeros_like(rho), tau[0], tau[1], tau[2], energy])


def rusanov(qL, qR, d, gamma):
    """Local Lax-Friedrichs flux along +axis d: (f(L) + f(R))/2 - lambda (qR - qL)/2,
    lambda = max(|u_d| + c) of the two sides."""
    def speed(q):
        return np.abs(q[1 + d] / q[0]) + np.sqrt(gamma * pressure(q, gamma) / q[0])
    lam = np.maximum(speed(qL), speed(qR))
    return 0.5 * (inviscid_flux(qL, d, gamma) + inviscid_flux(qR, d, gamma)) - 0.5 * lam * (qR - qL)


def roe(qL, qR, d, gamma):
    """Roe flux along +axis d (eq. invis_com in 3D): eigen-system of the flux Jacobian at the
    Roe average; acoustic waves u_d -+ c, entropy and two shear waves at u_d; no entropy fix."""
    fL, fR = inviscid_flux(qL, d, gamma), inviscid_flux(qR, d, gamma)
    rL, rR = qL[0], qR[0]
    uL = [qL[1 + i] / rL for i in range(3)]
    uR = [qR[1 + i] / rR for i in range(3)]
    pL, pR = pressure(qL, gamma), pressure(qR, gamma)
    HL, HR = (qL[4] + pL) / rL, (qR[4] + pR) / rR
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    rho = sL * sR
    u = [(sL * uL[i] + sR * uR[i]) / (sL + sR) for i in range(3)]
    H = (sL * HL + sR * HR) / (sL + sR)
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    c = np.sqrt((gamma - 1.0) * (H - 0.5 * q2))
    un = u[d]
    dr = rR - rL
    dp = pR - pL
    du = [uR[i] - uL[i] for i in range(3)]
    a1 = (dp - rho * c * du[d]) / (2.0 * c * c)
    a2 = dr - dp / (c * c)
    a4 = (dp + rho * c * du[d]) / (2.0 * c * c)
    one, zero = np.ones_like(un), np.zeros_like(un)
    e = [zero, zero, zero]
    e[d] = one

    def vec(r0, m, en):
        return np.stack([r0, m[0], m[1], m[2], en])
    r1 = vec(one, [u[i] - c * e[i] for i in range(3)], H - un * c)
    r4 = vec(one, [u[i] + c * e[i] for i in range(3)], H + un * c)
    r2 = vec(one, u, 0.5 * q2)
    diss = np.abs(un - c) * a1 * r1 + np.abs(un) * a2 * r2 + np.abs(un + c) * a4 * r4
    for t in range(3):          # shear waves: the tangential velocity jumps
        if t == d:
            continue
        m = [zero, zero, zero]
        m[t] = one
        diss = diss + np.abs(un) * rho * du[t] * vec(zero, m, u[t])
    return 0.5 * (fL + fR) - 0.5 * diss


FLUXES = {"rusanov": rusanov, "roe": roe}


class Box3D:
    """Triply periodic box of nx x ny x nz uniform hexahedra of size h = (hx, hy, hz)."""

    def __init__(self, nx, ny, nz, lo, L, P):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.nel = nx * ny * nz
        self.lo = np.asarray(lo, dtype=np.float64)
        self.L = np.asarray(L, dtype=np.float64)
        self.h = self.L / np.array([nx, ny, nz])
        self.b = Basis(P)
        self.n = P + 1
        e = np.arange(self.nel)
        self.ex, self.ey, self.ez = e % nx, (e // nx) % ny, e // (nx * ny)
        idx = lambda ex, ey, ez: ((ez % nz) * ny + (ey % ny)) * nx + (ex % nx)
        self.nbr = [(idx(self.ex - 1, self.ey, self.ez), idx(self.ex + 1, self.ey, self.ez)),
                    (idx(self.ex, self.ey - 1, self.ez), idx(self.ex, self.ey + 1, self.ez)),
                    (idx(self.ex, self.ey, self.ez - 1), idx(self.ex, self.ey, self.ez + 1))]

    def points(self):
        """x, y, z of every solution point, each [e, c, b, a]."""
        n, xs = self.n, self.b.x
        lo = self.lo[:, None] + self.h[:, None] * np.stack([self.ex, self.ey, self.ez])
        s = 0.5 * (xs + 1.0)
        x = lo[0][:, None, None, None] + self.h[0] * s[None, None, None, :] + 0 * s[None, :, None, None]
        y = lo[1][:, None, None, None] + self.h[1] * s[None, None, :, None] + 0 * s[None, :, None, None]
        z = lo[2][:, None, None, None] + self.h[2] * s[None, :, None, None] + 0 * s[None, None, :, None]
        sh = (self.nel, n, n, n)
        return np.broadcast_to(x, sh).copy(), np.broadcast_to(y, sh).copy(), np.broadcast_to(z, sh).copy()

    def weights(self):
        """Gauss weight times |J| of every point, [e, c, b, a] (sums to the box volume)."""
        w = self.b.w
        J = np.prod(self.h) / 8.0
        return np.broadcast_to(J * w[:, None, None] * w[None, :, None] * w[None, None, :],
                               (self.nel, self.n, self.n, self.n))


# axis of the [v, e, c, b, a] array that runs along direction d
AX = {0: 4, 1: 3, 2: 2}


def _apply(M, q, d):
    """Apply a 1D operator M[i, j] along direction d of a [v, e, c, b, a] array."""
    return np.moveaxis(np.tensordot(M, np.moveaxis(q, AX[d], 0), axes=(1, 0)), 0, AX[d])


def _face(q, vec, d):
    """Contract a [v, e, c, b, a] array with the row vector vec along direction d (a face trace)."""
    return np.tensordot(q, vec, axes=([AX[d]], [0]))


def _lift(face_vals, g, d):
    """face_vals (one face's values, the direction-d axis removed) times g along direction d."""
    return np.expand_dims(face_vals, AX[d]) * g.reshape([-1 if i == AX[d] else 1 for i in range(5)])


class NavierStokes3D:
    """FR residual on a Box3D; mu = 0 gives the Euler residual."""

    def __init__(self, box, gamma=1.4, rgas=1.0, mu=0.0, prandtl=0.71, flux="roe"):
        self.box, self.b = box, box.b
        self.gamma, self.rgas, self.mu, self.prandtl, self.flux = gamma, rgas, mu, prandtl, flux
        self.n = box.n
        self.nel = box.nel
        self.ndof = 5 * self.nel * self.n ** 3
        P = self.n - 1
        self.cP = (P + 1) * (P + 2) / 2.0

    def shape(self, U):
        n = self.n
        return np.asarray(U, dtype=np.float64).reshape(5, self.nel, n, n, n)

    def traces(self, q):
        """{(d, side)}: the solution trace on the face at -1 (side 0) / +1 (side 1) of direction d."""
        return {(d, s): _face(q, self.b.lm if s == 0 else self.b.lp, d) for d in range(3) for s in (0, 1)}

    def neighbour(self, arr, d, s):
        """For each element, the values `arr` of its neighbour across face (d, s)."""
        return arr[:, self.box.nbr[d][s]]

    def common_states(self, tr):
        return {(d, s): 0.5 * (tr[(d, s)] + self.neighbour(tr[(d, 1 - s)], d, s)) for d in range(3) for s in (0, 1)}

    def raw_gradient(self, q):
        return [(2.0 / self.box.h[k]) * _apply(self.b.D, q, k) for k in range(3)]

    def corrected_gradient(self, q, tr, qc):
        b = self.b
        out = []
        for k in range(3):
            g = _apply(b.D, q, k) + _lift(qc[(k, 0)] - tr[(k, 0)], b.gLp, k) + _lift(qc[(k, 1)] - tr[(k, 1)], b.gRp, k)
            out.append((2.0 / self.box.h[k]) * g)
        return out

    def face_gradients(self, q, tr, qc):
        """Each element's own BR2 gradient on each face: raw gradient extrapolated plus the
        face's lifting, {(d, s): [grad_x, grad_y, grad_z]}."""
        raw = self.raw_gradient(q)
        out = {}
        for d in range(3):
            for s in (0, 1):
                vec = self.b.lm if s == 0 else self.b.lp
                g = [_face(raw[k], vec, d) for k in range(3)]
                sign = -1.0 if s == 0 else 1.0
                g[d] = g[d] + self.cP * (qc[(d, s)] - tr[(d, s)]) * (2.0 / self.box.h[d]) * sign
                out[(d, s)] = g
        return out

    def _other_side(self, q):
        """For each face (d, s) of every element, the neighbour's trace there and, with
        viscosity, the neighbour's raw gradient extrapolated to that face."""
        tr = self.traces(q)
        other = {(d, s): self.neighbour(tr[(d, 1 - s)], d, s) for d in range(3) for s in (0, 1)}
        raw_other = None
        if self.mu != 0.0:
            raw = self.raw_gradient(q)
            raw_other = {}
            for d in range(3):
                for s in (0, 1):
                    vec = self.b.lp if s == 0 else self.b.lm      # the neighbour's face (d, 1 - s)
                    raw_other[(d, s)] = [self.neighbour(_face(raw[k], vec, d), d, s) for k in range(3)]
        return other, raw_other

    def residual(self, U):
        q = self.shape(U)
        other, raw_other = self._other_side(q)
        return self._residual(q, other, raw_other).reshape(np.shape(U))

    def local_residual_factory(self, U):
        """R as a function of each element's own state with every neighbour frozen at U,
        all elements at once (what the element-Jacobi blocks differentiate): the other
        side of each face (trace, raw gradient) comes from U; the common state and both
        sides' BR2 liftings use the element's own trace."""
        other, raw_other = self._other_side(self.shape(U))

        def local(V):
            q = self.shape(V)
            return self._residual(q, other, raw_other).reshape(np.shape(V))
        return local

    @property
    def nvar(self):
        return 5

    @property
    def npts(self):
        return self.n ** 3

    def _residual(self, q, other, raw_other):
        b, gam = self.b, self.gamma
        tr = self.traces(q)
        qc = {(d, s): 0.5 * (tr[(d, s)] + other[(d, s)]) for d in range(3) for s in (0, 1)}
        viscous = self.mu != 0.0
        if viscous:
            grad = self.corrected_gradient(q, tr, qc)
            fg = self.face_gradients(q, tr, qc)
        R = np.zeros_like(q)
        for d in range(3):
            f = inviscid_flux(q, d, gam)
            if viscous:
                f = f - viscous_flux(q, grad, d, gam, self.rgas, self.mu, self.prandtl)
            div = _apply(b.D, f, d)
            for s in (0, 1):
                fl = _face(f, b.lm if s == 0 else b.lp, d)
                mine = tr[(d, s)]
                qL, qR = (other[(d, s)], mine) if s == 0 else (mine, other[(d, s)])
                fc = FLUXES[self.flux](qL, qR, d, gam)
                if viscous:
                    # the neighbour's BR2 gradient on this face: its raw gradient plus its
                    # lifting (q^com - its trace) on its face (d, 1 - s)
                    gn = list(raw_other[(d, s)])
                    sign_nb = -1.0 if s == 1 else 1.0
                    gn[d] = gn[d] + self.cP * (qc[(d, s)] - other[(d, s)]) * (2.0 / self.box.h[d]) * sign_nb
                    gcom = [0.5 * (fg[(d, s)][k] + gn[k]) for k in range(3)]
                    fc = fc - viscous_flux(qc[(d, s)], gcom, d, gam, self.rgas, self.mu, self.prandtl)
                div = div + _lift(fc - fl, b.gLp if s == 0 else b.gRp, d)
            R -= (2.0 / self.box.h[d]) * div
        return R


def dissipation(op, U, rho0):
    """Kinetic energy E_k = (1/(rho0 V)) int rho |u|^2 / 2 dV and the dissipation rates of
    Section 5.3: eps1 = 2 mu / (rho0 V) int S^d : S^d dV and eps3 = -(1/(rho0 V)) int p div u dV
    (eps2 = 0: zero bulk viscosity), with the velocity gradient from the raw gradient of
    each element's solution polynomial (du_i = (d(rho u_i) - u_i d rho) / rho) and the
    solution-point Gauss rule.  On the periodic box int div u dV = 0 for the exact field, so
    eps3 takes the pressure about its volume mean, -(1/(rho0 V)) int (p - <p>) div u dV: the
    same number for a continuous field, without <p> times the sum of the velocity jumps
    between elements that the element-local gradient leaves in int div u dV (at M = 0.1
    <p> is about 71 rho0 V0^2 and that term would dominate)."""
    q = op.shape(U)
    box = op.box
    w = box.weights()
    V = float(np.sum(w))
    raw = op.raw_gradient(q)
    rho = q[0]
    u = [q[1 + i] / rho for i in range(3)]
    du = [[(raw[k][1 + i] - u[i] * raw[k][0]) / rho for k in range(3)] for i in range(3)]
    div = du[0][0] + du[1][1] + du[2][2]
    SdSd = np.zeros_like(rho)
    for i in range(3):
        for k in range(3):
            s = 0.5 * (du[i][k] + du[k][i]) - (div / 3.0 if i == k else 0.0)
            SdSd = SdSd + s * s
    p = pressure(q, op.gamma)
    ek = np.sum(w * 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)) / (rho0 * V)
    eps1 = 2.0 * op.mu / rho0 * np.sum(w * SdSd) / V
    pmean = np.sum(w * p) / V
    eps3 = -np.sum(w * (p - pmean) * div) / (rho0 * V)
    return float(ek), float(eps1), float(eps3)


def ssprk3_step(op, U, dt):
    """Three-stage strong-stability-preserving Runge-Kutta step (the paper's explicit reference
    integrator): U1 = U + dt R(U); U2 = 3/4 U + 1/4 (U1 + dt R(U1)); U+ = 1/3 U + 2/3 (U2 + dt R(U2))."""
    U = np.asarray(U, dtype=np.float64)
    U1 = U + dt * op.residual(U)
    U2 = 0.75 * U + 0.25 * (U1 + dt * op.residual(U1))
    return U / 3.0 + (2.0 / 3.0) * (U2 + dt * op.residual(U2))
