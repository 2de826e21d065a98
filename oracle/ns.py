"""Oracle (test infrastructure only): FR residual of the 2D compressible
Navier-Stokes equations with the BR1 common gradient.

Section 2 gives the viscous flux (Stokes stress, Fourier heat flux with
kappa = mu Cp / Pr, constant mu and Pr).  Section 3 gives the common state
q^com = (q+ + q-)/2 (eq. com_q) and the common gradient as the average of the
two sides' corrected gradients (eq. com_grad_q).  The workloads ask for the
first Bassi-Rebay scheme, in which the correction of a side's gradient is its
own FR-corrected gradient (the correction function lifts the jump
q^com - q_local); the paper's BR2 penalty (P+1)(P+2)/2 is not used here.

Per element, with the Radau correction derivatives g_L', g_R':
  dq/dxi~  = D q + (q^com - q)|_{xi=-1} g_L'(xi) + (q^com - q)|_{xi=+1} g_R'(xi)   (same in eta)
  grad q   = (1/|J|) [ y_eta dq/dxi~ - y_xi dq/deta~ ,  -x_eta dq/dxi~ + x_xi dq/deta~ ]
  face gradient of the element = its grad q extrapolated to the face
  common gradient = mean of the two sides' face gradients
The total flux f - f_v, g - g_v then goes through the FR residual of the
Euler module; at faces the viscous part of the common flux is evaluated at
(q^com, common gradient).
"""
from __future__ import annotations

import numpy as np

from .euler import EulerFR, face_flux, physical_flux


def viscous_flux(q, qx, qy, gamma, rgas, mu, prandtl):
    """f_v, g_v of Section 2 in 2D from the conservative state and its gradient."""
    rho, mx, my, E = q
    u = mx / rho
    v = my / rho
    ux = (qx[1] - u * qx[0]) / rho
    uy = (qy[1] - u * qy[0]) / rho
    vx = (qx[2] - v * qx[0]) / rho
    vy = (qy[2] - v * qy[0]) / rho
    p = (gamma - 1.0) * (E - 0.5 * rho * (u * u + v * v))
    T = p / (rho * rgas)
    px = (gamma - 1.0) * (qx[3] - 0.5 * (u * u + v * v) * qx[0] - rho * (u * ux + v * vx))
    py = (gamma - 1.0) * (qy[3] - 0.5 * (u * u + v * v) * qy[0] - rho * (u * uy + v * vy))
    Tx = (px - rgas * T * qx[0]) / (rho * rgas)
    Ty = (py - rgas * T * qy[0]) / (rho * rgas)
    div = ux + vy
    txx = mu * (2.0 * ux - 2.0 / 3.0 * div)
    tyy = mu * (2.0 * vy - 2.0 / 3.0 * div)
    txy = mu * (uy + vx)
    kappa = mu * (gamma * rgas / (gamma - 1.0)) / prandtl
    zero = np.zeros_like(rho)
    fv = np.stack([zero, txx, txy, u * txx + v * txy + kappa * Tx])
    gv = np.stack([zero, txy, tyy, u * txy + v * tyy + kappa * Ty])
    return fv, gv


class NavierStokesFR(EulerFR):
    def __init__(self, geo, gamma=1.4, flux="rusanov", rgas=1.0, mu=1e-4, prandtl=0.71):
        super().__init__(geo, gamma=gamma, flux=flux)
        self.rgas = rgas
        self.mu = mu
        self.prandtl = prandtl

    # ------------------------------------------------------------ gradients
    def corrected_gradient(self, q, qc):
        """Physical BR1 gradient at the solution points, given the element's common
        solution on its four faces qc = {W, E: [v, e, b], S, N: [v, e, a]}."""
        b, geo = self.b, self.geo
        tr = self.traces(q)
        dxi = (np.einsum("ac,vebc->veba", b.D, q)
               + (qc["W"] - tr["W"])[:, :, :, None] * b.gLp[None, None, None, :]
               + (qc["E"] - tr["E"])[:, :, :, None] * b.gRp[None, None, None, :])
        deta = (np.einsum("bc,veca->veba", b.D, q)
                + (qc["S"] - tr["S"])[:, :, None, :] * b.gLp[None, None, :, None]
                + (qc["N"] - tr["N"])[:, :, None, :] * b.gRp[None, None, :, None])
        qx = (geo.y_eta * dxi - geo.y_xi * deta) / geo.J
        qy = (-geo.x_eta * dxi + geo.x_xi * deta) / geo.J
        return qx, qy

    def face_values(self, a):
        """Traces of a [v, e, b, a] field on the four faces."""
        lm, lp = self.b.lm, self.b.lp
        return {"W": np.einsum("a,veba->veb", lm, a), "E": np.einsum("a,veba->veb", lp, a),
                "S": np.einsum("b,veba->vea", lm, a), "N": np.einsum("b,veba->vea", lp, a)}

    def common_solution(self, tr, nbr):
        return {f: 0.5 * (tr[f] + nbr[f]) for f in ("W", "E", "S", "N")}

    # ------------------------------------------------------------ residual
    def residual_parts(self, q, qc, gface_own, gface_nbr, nbr):
        """Element residual given the element's state q, its faces' common solution qc,
        its own face gradients and the neighbours' face gradients on the shared faces
        (each {face: (qx, qy)}), and the neighbours' solution traces nbr."""
        b, geo, gam = self.b, self.geo, self.gamma
        qx, qy = self.corrected_gradient(q, qc)
        f, g = physical_flux(q, gam)
        fv, gv = viscous_flux(q, qx, qy, gam, self.rgas, self.mu, self.prandtl)
        ft, gt = f - fv, g - gv
        F = geo.y_eta * ft - geo.x_eta * gt
        G = -geo.y_xi * ft + geo.x_xi * gt
        tr = self.traces(q)
        Fl = {"W": np.einsum("a,veba->veb", b.lm, F), "E": np.einsum("a,veba->veb", b.lp, F),
              "S": np.einsum("b,veba->vea", b.lm, G), "N": np.einsum("b,veba->vea", b.lp, G)}
        S = {"W": geo.SW, "E": geo.SE, "S": geo.SS, "N": geo.SN}
        Fn = {}
        for fc in ("W", "E", "S", "N"):
            left_nbr = fc in ("W", "S")
            qL, qR = (nbr[fc], tr[fc]) if left_nbr else (tr[fc], nbr[fc])
            inv = face_flux(qL, qR, S[fc], gam, self.flux)
            gx = 0.5 * (gface_own[fc][0] + gface_nbr[fc][0])
            gy = 0.5 * (gface_own[fc][1] + gface_nbr[fc][1])
            fvc, gvc = viscous_flux(qc[fc], gx, gy, gam, self.rgas, self.mu, self.prandtl)
            Fn[fc] = inv - (fvc * S[fc][0] + gvc * S[fc][1])
        div = (np.einsum("ac,vebc->veba", b.D, F)
               + (Fn["W"] - Fl["W"])[:, :, :, None] * b.gLp[None, None, None, :]
               + (Fn["E"] - Fl["E"])[:, :, :, None] * b.gRp[None, None, None, :]
               + np.einsum("bc,veca->veba", b.D, G)
               + (Fn["S"] - Fl["S"])[:, :, None, :] * b.gLp[None, None, :, None]
               + (Fn["N"] - Fl["N"])[:, :, None, :] * b.gRp[None, None, :, None])
        return -div / geo.J[None]

    def gradient_state(self, q):
        """Everything the BR1 residual needs from the whole mesh at state q."""
        m = self.mesh
        tr = self.traces(q)
        nbr = self.neighbour_traces(tr)
        qc = self.common_solution(tr, nbr)
        qx, qy = self.corrected_gradient(q, qc)
        gx, gy = self.face_values(qx), self.face_values(qy)
        own = {fc: (gx[fc], gy[fc]) for fc in ("W", "E", "S", "N")}
        opp = {"W": ("E", m.west), "E": ("W", m.east), "S": ("N", m.south), "N": ("S", m.north)}
        nb = {fc: (gx[o][:, idx], gy[o][:, idx]) for fc, (o, idx) in opp.items()}
        return tr, nbr, qc, own, nb

    def residual(self, U):
        q = self.shape(U)
        tr, nbr, qc, own, nb = self.gradient_state(q)
        return self.residual_parts(q, qc, own, nb, nbr).reshape(np.shape(U))

    # ------------------------------------------------------------ element-local form (element-Jacobi)
    def local_residual_factory(self, U):
        """R_e as a function of the element's own state only, every other element's state
        fixed at U.  Besides the element's own terms, R_e reaches a neighbour's state
        through that neighbour's corrected gradient on the shared face, which contains
        the shared face's common solution, hence the element's own trace."""
        q0 = self.shape(U)
        m = self.mesh
        tr0 = self.traces(q0)
        nbr = self.neighbour_traces(tr0)
        qc0 = self.common_solution(tr0, nbr)
        opp = {"W": ("E", m.west), "E": ("W", m.east), "S": ("N", m.south), "N": ("S", m.north)}
        # every neighbour's state, its geometry-dependent gradient and its frozen face commons
        nq = {fc: q0[:, idx] for fc, (o, idx) in opp.items()}
        nqc = {fc: {g: qc0[g][:, idx] for g in ("W", "E", "S", "N")} for fc, (o, idx) in opp.items()}
        geo = self.geo
        nmet = {fc: (geo.x_xi[idx], geo.x_eta[idx], geo.y_xi[idx], geo.y_eta[idx], geo.J[idx])
                for fc, (o, idx) in opp.items()}

        def nbr_face_gradient(fc, qc_shared):
            o, _ = opp[fc]
            qcn = dict(nqc[fc])
            qcn[o] = qc_shared
            qn = nq[fc]
            trn = self.traces(qn)
            b = self.b
            dxi = (np.einsum("ac,vebc->veba", b.D, qn)
                   + (qcn["W"] - trn["W"])[:, :, :, None] * b.gLp[None, None, None, :]
                   + (qcn["E"] - trn["E"])[:, :, :, None] * b.gRp[None, None, None, :])
            deta = (np.einsum("bc,veca->veba", b.D, qn)
                    + (qcn["S"] - trn["S"])[:, :, None, :] * b.gLp[None, None, :, None]
                    + (qcn["N"] - trn["N"])[:, :, None, :] * b.gRp[None, None, :, None])
            xx, xe, yx, ye, J = nmet[fc]
            qx = (ye * dxi - yx * deta) / J
            qy = (-xe * dxi + xx * deta) / J
            return self.face_values(qx)[o], self.face_values(qy)[o]

        def local(q):
            tr = self.traces(q)
            qc = self.common_solution(tr, nbr)
            qx, qy = self.corrected_gradient(q, qc)
            gx, gy = self.face_values(qx), self.face_values(qy)
            own = {fc: (gx[fc], gy[fc]) for fc in ("W", "E", "S", "N")}
            nb = {fc: nbr_face_gradient(fc, qc[fc]) for fc in ("W", "E", "S", "N")}
            return self.residual_parts(q, qc, own, nb, nbr)

        return local
