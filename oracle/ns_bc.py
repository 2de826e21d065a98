"""Oracle (test infrastructure only): the 2D Navier-Stokes FR residual with the
paper's BR2 common gradient and with wall / far-field boundaries on the eta = -1
side of the first element row and the eta = +1 side of the last one (xi stays
periodic: an O-grid around a body, or a channel).

BR2 (Section 3, eq. com_grad_q and the lifting that follows it): on a face,

  common gradient = ( (grad q^- + r^-) + (grad q^+ + r^+) ) / 2,
  r = gamma (q^com - q_local) n,   gamma = |grad w| g'(w) sign(n . grad w),  w in {xi, eta},

with g'(+-1) = +-(P+1)(P+2)/2 (the paper's stabilising value).  On either side,
whichever direction n is taken in, gamma n = c_P |grad w| n_out with c_P =
(P+1)(P+2)/2 and n_out the side's outward unit normal; |grad w| n_out = S_out / |J|,
S_out the outward area-weighted face normal and |J| taken at the face point.
Readings (the paper does not say more):
  * grad q^+- is the side's gradient without corrections: the physical gradient of its
    solution polynomial, J^{-T} (D q along xi, D q along eta), at the solution points,
    extrapolated to the face point;
  * the gradient inside the element (for the viscous flux at the solution points) is the
    FR-corrected one of the BR1 module (Radau g'), unchanged;
  * q^com = (q^+ + q^-)/2 as in BR1.

Boundaries (readings; the paper names the cylinder case's wall and far field but gives
no formulas):
  * far field: the outside trace is the given free-stream state q_far; the inviscid
    common flux is the interior Riemann solver between the trace and q_far; the common
    state is (q + q_far)/2; the common gradient is the side's own face gradient;
  * wall (no slip, adiabatic): the outside trace is (rho, -rho u, -rho v, E - rho |u|^2),
    so that q^com = (rho, 0, 0, E - rho |u|^2 / 2): zero velocity, the inside internal
    energy; the inviscid common flux is the pressure flux (0, p S_x, p S_y, 0) with p
    from the inside trace; the viscous flux is evaluated at q^com with the side's own
    face gradient, and its energy component is zero (no heat flux, zero velocity).
"""
from __future__ import annotations

import numpy as np

from .euler import face_flux, pressure
from .geometry import bilinear
from .ns import NavierStokesFR, viscous_flux

FACES = ("W", "E", "S", "N")


def wall_ghost(q):
    """Outside trace of a no-slip adiabatic wall: velocity reversed, kinetic energy removed twice."""
    rho, mx, my, E = q
    return np.stack([rho, -mx, -my, E - (mx * mx + my * my) / rho])


class NavierStokesBC(NavierStokesFR):
    """viscous: "br1" or "br2"; bc_south / bc_north: None (periodic), "wall" or "farfield"."""

    def __init__(self, geo, gamma=1.4, flux="rusanov", rgas=1.0, mu=1e-4, prandtl=0.71, viscous="br1",
                 bc_south=None, bc_north=None, q_far=None):
        super().__init__(geo, gamma=gamma, flux=flux, rgas=rgas, mu=mu, prandtl=prandtl)
        if viscous not in ("br1", "br2"):
            raise ValueError("viscous must be br1 or br2")
        for bc in (bc_south, bc_north):
            if bc not in (None, "wall", "farfield"):
                raise ValueError("bc must be None, wall or farfield")
        if "farfield" in (bc_south, bc_north) and q_far is None:
            raise ValueError("a far-field boundary needs q_far")
        self.viscous = viscous
        self.bc = {"S": bc_south, "N": bc_north}
        self.q_far = None if q_far is None else np.asarray(q_far, dtype=np.float64)
        m = self.mesh
        self.on_bnd = {"W": np.zeros(m.nel, bool), "E": np.zeros(m.nel, bool),
                       "S": (m.ey == 0) & (bc_south is not None), "N": (m.ey == m.ny - 1) & (bc_north is not None)}
        P = self.b.P
        self.cP = (P + 1) * (P + 2) / 2.0
        # |J| at the face points (W/E: [e, b] at xi = -+1; S/N: [e, a] at eta = -+1)
        xs = self.b.x
        one = np.ones_like(xs)
        self.Jf = {"W": bilinear(m, -one, xs)["J"], "E": bilinear(m, one, xs)["J"],
                   "S": bilinear(m, xs, -one)["J"], "N": bilinear(m, xs, one)["J"]}
        geo = self.geo
        S = {"W": geo.SW, "E": geo.SE, "S": geo.SS, "N": geo.SN}
        # outward area-weighted normals of every element's faces
        self.Sout = {f: (-S[f] if f in ("W", "S") else S[f]) for f in FACES}

    # ------------------------------------------------------------ boundary traces
    def ghost(self, f, q):
        if self.bc[f] == "wall":
            return wall_ghost(q)
        return np.broadcast_to(self.q_far.reshape((4,) + (1,) * (q.ndim - 1)), q.shape).copy()

    def neighbour_traces(self, tr):
        nbr = super().neighbour_traces(tr)
        for f in ("S", "N"):
            if self.bc[f] is not None:
                sel = self.on_bnd[f]
                nbr[f] = nbr[f].copy()
                nbr[f][:, sel] = self.ghost(f, tr[f][:, sel])
        return nbr

    # ------------------------------------------------------------ face gradients
    def raw_gradient(self, q):
        """Physical gradient of the solution polynomial at the solution points (no corrections)."""
        b, geo = self.b, self.geo
        dxi = np.einsum("ac,vebc->veba", b.D, q)
        deta = np.einsum("bc,veca->veba", b.D, q)
        return (geo.y_eta * dxi - geo.y_xi * deta) / geo.J, (-geo.x_eta * dxi + geo.x_xi * deta) / geo.J

    def own_face_gradients(self, q, qc, tr):
        """Each element's own gradient on its four faces, {f: (gx, gy)}: BR1 the corrected
        gradient extrapolated, BR2 the raw gradient extrapolated plus the face's lifting r."""
        if self.viscous == "br1":
            qx, qy = self.corrected_gradient(q, qc)
            gx, gy = self.face_values(qx), self.face_values(qy)
            return {f: (gx[f], gy[f]) for f in FACES}
        qx, qy = self.raw_gradient(q)
        gx, gy = self.face_values(qx), self.face_values(qy)
        out = {}
        for f in FACES:
            lift = self.cP * (qc[f] - tr[f]) / self.Jf[f][None]
            out[f] = (gx[f] + lift * self.Sout[f][0][None], gy[f] + lift * self.Sout[f][1][None])
        return out

    def shared_face_gradients(self, own):
        """The neighbour's own gradient on each shared face; a boundary side mirrors its own."""
        m = self.mesh
        opp = {"W": ("E", m.west), "E": ("W", m.east), "S": ("N", m.south), "N": ("S", m.north)}
        nb = {f: (own[o][0][:, idx].copy(), own[o][1][:, idx].copy()) for f, (o, idx) in opp.items()}
        for f in ("S", "N"):
            sel = self.on_bnd[f]
            nb[f][0][:, sel] = own[f][0][:, sel]
            nb[f][1][:, sel] = own[f][1][:, sel]
        return nb

    # ------------------------------------------------------------ residual
    def face_fluxes(self, tr, nbr, qc, own, nb):
        """F^num on the four faces of every element (inviscid minus viscous, along S)."""
        gam = self.gamma
        geo = self.geo
        S = {"W": geo.SW, "E": geo.SE, "S": geo.SS, "N": geo.SN}
        Fn = {}
        for f in FACES:
            left_nbr = f in ("W", "S")
            qL, qR = (nbr[f], tr[f]) if left_nbr else (tr[f], nbr[f])
            inv = face_flux(qL, qR, S[f], gam, self.flux)
            gx = 0.5 * (own[f][0] + nb[f][0])
            gy = 0.5 * (own[f][1] + nb[f][1])
            fvc, gvc = viscous_flux(qc[f], gx, gy, gam, self.rgas, self.mu, self.prandtl)
            vis = fvc * S[f][0] + gvc * S[f][1]
            if self.bc.get(f) == "wall":
                sel = self.on_bnd[f]
                p = pressure(tr[f][:, sel], gam)
                inv[:, sel] = np.stack([np.zeros_like(p), p * S[f][0][sel], p * S[f][1][sel], np.zeros_like(p)])
                vis[3, sel] = 0.0
            Fn[f] = inv - vis
        return Fn

    def residual_from(self, q, tr, nbr, qc, own, nb):
        b, geo, gam = self.b, self.geo, self.gamma
        from .euler import physical_flux
        qx, qy = self.corrected_gradient(q, qc)
        fI, gI = physical_flux(q, gam)
        fv, gv = viscous_flux(q, qx, qy, gam, self.rgas, self.mu, self.prandtl)
        ft, gt = fI - fv, gI - gv
        F = geo.y_eta * ft - geo.x_eta * gt
        G = -geo.y_xi * ft + geo.x_xi * gt
        Fl = {"W": np.einsum("a,veba->veb", b.lm, F), "E": np.einsum("a,veba->veb", b.lp, F),
              "S": np.einsum("b,veba->vea", b.lm, G), "N": np.einsum("b,veba->vea", b.lp, G)}
        Fn = self.face_fluxes(tr, nbr, qc, own, nb)
        div = (np.einsum("ac,vebc->veba", b.D, F)
               + (Fn["W"] - Fl["W"])[:, :, :, None] * b.gLp[None, None, None, :]
               + (Fn["E"] - Fl["E"])[:, :, :, None] * b.gRp[None, None, None, :]
               + np.einsum("bc,veca->veba", b.D, G)
               + (Fn["S"] - Fl["S"])[:, :, None, :] * b.gLp[None, None, :, None]
               + (Fn["N"] - Fl["N"])[:, :, None, :] * b.gRp[None, None, :, None])
        return -div / geo.J[None]

    def state(self, q):
        tr = self.traces(q)
        nbr = self.neighbour_traces(tr)
        qc = self.common_solution(tr, nbr)
        own = self.own_face_gradients(q, qc, tr)
        nb = self.shared_face_gradients(own)
        return tr, nbr, qc, own, nb

    def residual(self, U):
        q = self.shape(U)
        tr, nbr, qc, own, nb = self.state(q)
        return self.residual_from(q, tr, nbr, qc, own, nb).reshape(np.shape(U))

    def face_common_gradients(self, U):
        """The common gradient on every element's four faces, {f: (gx, gy)}, [v, e, j]."""
        q = self.shape(U)
        tr, nbr, qc, own, nb = self.state(q)
        return {f: (0.5 * (own[f][0] + nb[f][0]), 0.5 * (own[f][1] + nb[f][1])) for f in FACES}

    def boundary_fluxes(self, U):
        """{"S", "N"}: F^num on the boundary faces of the boundary rows, [v, ex, a] along the
        face's +eta normal (empty entries for periodic sides)."""
        q = self.shape(U)
        tr, nbr, qc, own, nb = self.state(q)
        Fn = self.face_fluxes(tr, nbr, qc, own, nb)
        return {f: Fn[f][:, self.on_bnd[f]] for f in ("S", "N")}

    def wall_force(self, U):
        """Force of the fluid on the wall at the eta = -1 boundary: minus the momentum
        flux through the wall faces, F^num integrated with the Gauss weights along each
        face (S is per unit reference length)."""
        if self.bc["S"] != "wall":
            raise ValueError("no wall on the south boundary")
        Fs = self.boundary_fluxes(U)["S"]
        w = self.b.w
        return -np.einsum("a,vea->v", w, Fs)[1:3]

    # ------------------------------------------------------------ element-local form (element-Jacobi)
    def local_residual_factory(self, U):
        """R_e as a function of the element's own state, every other element fixed at U.
        The neighbour's gradient on a shared face depends on the element through the
        shared common state only: BR1 through the neighbour's corrected gradient (its face
        correction), BR2 through the neighbour's lifting r, linear in q^com.  A boundary
        side depends on the element alone (its outside trace and mirrored gradient)."""
        q0 = self.shape(U)
        m = self.mesh
        tr0 = self.traces(q0)
        nbr_per = NavierStokesFR.neighbour_traces(self, tr0)     # the periodic neighbours' traces
        qc0 = self.common_solution(tr0, self.neighbour_traces(tr0))
        own0 = self.own_face_gradients(q0, qc0, tr0)
        opp = {"W": ("E", m.west), "E": ("W", m.east), "S": ("N", m.south), "N": ("S", m.north)}
        geo = self.geo
        br2 = self.viscous == "br2"
        if br2:
            qxr, qyr = self.raw_gradient(q0)
            rgx, rgy = self.face_values(qxr), self.face_values(qyr)
        nq = {f: q0[:, idx] for f, (o, idx) in opp.items()}
        nqc = {f: {g: qc0[g][:, idx] for g in FACES} for f, (o, idx) in opp.items()}
        nmet = {f: (geo.x_xi[idx], geo.x_eta[idx], geo.y_xi[idx], geo.y_eta[idx], geo.J[idx])
                for f, (o, idx) in opp.items()}

        def nbr_face_gradient(f, qc_shared):
            o, idx = opp[f]
            if br2:
                lift = self.cP * (qc_shared - tr0[o][:, idx]) / self.Jf[o][idx][None]
                return (rgx[o][:, idx] + lift * self.Sout[o][0][idx][None],
                        rgy[o][:, idx] + lift * self.Sout[o][1][idx][None])
            qcn = dict(nqc[f])
            qcn[o] = qc_shared
            qn = nq[f]
            trn = self.traces(qn)
            b = self.b
            dxi = (np.einsum("ac,vebc->veba", b.D, qn)
                   + (qcn["W"] - trn["W"])[:, :, :, None] * b.gLp[None, None, None, :]
                   + (qcn["E"] - trn["E"])[:, :, :, None] * b.gRp[None, None, None, :])
            deta = (np.einsum("bc,veca->veba", b.D, qn)
                    + (qcn["S"] - trn["S"])[:, :, None, :] * b.gLp[None, None, :, None]
                    + (qcn["N"] - trn["N"])[:, :, None, :] * b.gRp[None, None, :, None])
            xx, xe, yx, ye, J = nmet[f]
            qx = (ye * dxi - yx * deta) / J
            qy = (-xe * dxi + xx * deta) / J
            return self.face_values(qx)[o], self.face_values(qy)[o]

        def local(q):
            tr = self.traces(q)
            nbr = {f: nbr_per[f].copy() for f in FACES}
            for f in ("S", "N"):
                if self.bc[f] is not None:
                    sel = self.on_bnd[f]
                    nbr[f][:, sel] = self.ghost(f, tr[f][:, sel])
            qc = self.common_solution(tr, nbr)
            own = self.own_face_gradients(q, qc, tr)
            nb = {f: nbr_face_gradient(f, qc[f]) for f in FACES}
            for f in ("S", "N"):
                sel = self.on_bnd[f]
                nb[f] = (nb[f][0].copy(), nb[f][1].copy())
                nb[f][0][:, sel] = own[f][0][:, sel]
                nb[f][1][:, sel] = own[f][1][:, sel]
            return self.residual_from(q, tr, nbr, qc, own, nb)

        return local
