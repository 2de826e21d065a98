"""Oracle (test infrastructure only): bilinear quad geometry (Section 3, eqs. for
Q, F, G and the Jacobian of the map), restricted to 2D.

Each element is the bilinear image of [-1,1]^2 through its four corners.  At a
point the metric terms are x_xi, x_eta, y_xi, y_eta and |J| = x_xi y_eta - x_eta y_xi.
Since |J| xi_x = y_eta, |J| xi_y = -x_eta, |J| eta_x = -y_xi and |J| eta_y = x_xi,
the transformed fluxes are F = y_eta f - x_eta g and G = -y_xi f + x_xi g, and
the area-weighted face normals are S_xi = (y_eta, -x_eta) on xi-faces and
S_eta = (-y_xi, x_xi) on eta-faces, with |S| = |J| |grad xi| (eq. norm_num_f).
"""
from __future__ import annotations

import numpy as np

from .basis import Basis


class Mesh:
    """Doubly periodic structured quad mesh given by its vertex array
    nodes[j, i, (x, y)], j = 0..ny, i = 0..nx."""

    def __init__(self, nodes: np.ndarray):
        self.nodes = np.asarray(nodes, dtype=np.float64)
        self.ny = self.nodes.shape[0] - 1
        self.nx = self.nodes.shape[1] - 1
        self.nel = self.nx * self.ny
        ex = np.arange(self.nel) % self.nx
        ey = np.arange(self.nel) // self.nx
        self.ex, self.ey = ex, ey
        self.east = ey * self.nx + (ex + 1) % self.nx
        self.west = ey * self.nx + (ex - 1) % self.nx
        self.north = ((ey + 1) % self.ny) * self.nx + ex
        self.south = ((ey - 1) % self.ny) * self.nx + ex
        nd = self.nodes
        self.c00 = nd[ey, ex]          # (nel, 2)
        self.c10 = nd[ey, ex + 1]
        self.c01 = nd[ey + 1, ex]
        self.c11 = nd[ey + 1, ex + 1]


def bilinear(mesh: Mesh, xi, eta):
    """Position and metric terms at reference points (xi, eta) of every element.

    xi, eta: arrays of equal shape S.  Returns dict of arrays of shape (nel,)+S.
    """
    xi = np.asarray(xi, dtype=np.float64)
    eta = np.asarray(eta, dtype=np.float64)
    sh = (mesh.nel,) + (1,) * xi.ndim
    out = {}
    for c, name in ((0, "x"), (1, "y")):
        p00 = mesh.c00[:, c].reshape(sh)
        p10 = mesh.c10[:, c].reshape(sh)
        p01 = mesh.c01[:, c].reshape(sh)
        p11 = mesh.c11[:, c].reshape(sh)
        out[name] = 0.25 * ((1 - xi) * (1 - eta) * p00 + (1 + xi) * (1 - eta) * p10
                            + (1 - xi) * (1 + eta) * p01 + (1 + xi) * (1 + eta) * p11)
        out[name + "_xi"] = 0.25 * (-(1 - eta) * p00 + (1 - eta) * p10 - (1 + eta) * p01 + (1 + eta) * p11)
        out[name + "_eta"] = 0.25 * (-(1 - xi) * p00 - (1 + xi) * p10 + (1 - xi) * p01 + (1 + xi) * p11)
    out["J"] = out["x_xi"] * out["y_eta"] - out["x_eta"] * out["y_xi"]
    return out


class Geometry:
    """Metric terms at solution points and face normals of a mesh for degree P."""

    def __init__(self, mesh: Mesh, basis: Basis):
        self.mesh = mesh
        self.basis = basis
        xs = basis.x
        # solution points, indexed [e, b, a] (a along xi, b along eta)
        XI, ETA = np.meshgrid(xs, xs, indexing="xy")   # XI[b, a] = xs[a], ETA[b, a] = xs[b]
        g = bilinear(mesh, XI, ETA)
        self.x, self.y = g["x"], g["y"]
        self.x_xi, self.x_eta, self.y_xi, self.y_eta, self.J = g["x_xi"], g["x_eta"], g["y_xi"], g["y_eta"], g["J"]
        # xi-faces: normal S_xi = (y_eta, -x_eta) at (xi = +-1, eta_b), shape (nel, n)
        ge = bilinear(mesh, np.ones_like(xs), xs)
        gw = bilinear(mesh, -np.ones_like(xs), xs)
        self.SE = np.stack([ge["y_eta"], -ge["x_eta"]])   # (2, nel, n)
        self.SW = np.stack([gw["y_eta"], -gw["x_eta"]])
        # eta-faces: S_eta = (-y_xi, x_xi) at (xi_a, eta = +-1)
        gn = bilinear(mesh, xs, np.ones_like(xs))
        gs = bilinear(mesh, xs, -np.ones_like(xs))
        self.SN = np.stack([-gn["y_xi"], gn["x_xi"]])
        self.SS = np.stack([-gs["y_xi"], gs["x_xi"]])

    def points(self):
        """Physical coordinates of the solution points, each (nel, n*n) in k = b*n + a order."""
        nel = self.mesh.nel
        return self.x.reshape(nel, -1), self.y.reshape(nel, -1)
