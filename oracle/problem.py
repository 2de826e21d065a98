"""Oracle (test infrastructure only): set-up helpers tying a mesh, a basis and a
residual operator together, plus the L2 error of Section 5.1."""
from __future__ import annotations

import numpy as np

from .basis import Basis
from .geometry import Geometry, Mesh
from .euler import EulerFR
from .ns import NavierStokesFR


def make_euler(nodes, P, gamma=1.4, flux="rusanov"):
    geo = Geometry(Mesh(nodes), Basis(P))
    return EulerFR(geo, gamma=gamma, flux=flux)


def make_ns(nodes, P, gamma=1.4, flux="rusanov", rgas=1.0, mu=1e-4, prandtl=0.71):
    geo = Geometry(Mesh(nodes), Basis(P))
    return NavierStokesFR(geo, gamma=gamma, flux=flux, rgas=rgas, mu=mu, prandtl=prandtl)


def sample_state(op, fn):
    """Evaluate a closed-form state fn(x, y) -> (4, ...) at all solution points, [v, e, k] layout."""
    x, y = op.geo.points()
    return np.asarray(fn(x, y), dtype=np.float64).reshape(4, op.nel, -1)


def l2_error(op, s_num, s_exact):
    """sqrt( int (s_exact - s_num)^2 dV / V ) (Section 5.1) with the tensor Gauss rule
    of the solution points; s_* indexed [e, k]."""
    w = op.b.w
    wk = (w[:, None] * w[None, :]).reshape(-1)          # weight of point k = b*n + a
    Jk = op.geo.J.reshape(op.nel, -1)
    vol = np.sum(wk[None, :] * Jk)
    d = np.asarray(s_num) - np.asarray(s_exact)
    return float(np.sqrt(np.sum(wk[None, :] * Jk * d * d) / vol))


def make_ns_bc(nodes, P, gamma=1.4, flux="rusanov", rgas=1.0, mu=1e-4, prandtl=0.71, viscous="br1",
               bc_south=None, bc_north=None, q_far=None):
    from .ns_bc import NavierStokesBC
    geo = Geometry(Mesh(nodes), Basis(P))
    return NavierStokesBC(geo, gamma=gamma, flux=flux, rgas=rgas, mu=mu, prandtl=prandtl, viscous=viscous,
                          bc_south=bc_south, bc_north=bc_north, q_far=q_far)
