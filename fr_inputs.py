"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This module holds no arithmetic of the FR method, the linear solvers or the
time integrators.  It only produces input data:

* quad-mesh vertex arrays (uniform, or with interior nodes randomly moved),
* closed-form flow states of the two test problems as functions of the
  physical position (x, y) and time t,
* seeded random vectors used as GMRES right-hand sides and Krylov vectors.

Vertex array layout: ``nodes[j, i, c]`` with ``j = 0..ny``, ``i = 0..nx`` and
``c`` in {x, y}.  Element (ex, ey) has corners (ex, ey), (ex+1, ey),
(ex, ey+1), (ex+1, ey+1).  The domain is doubly periodic, so node (nx, j)
is the copy of node (0, j) shifted by Lx (likewise in y); boundary nodes are
never moved, which keeps that identification exact.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 1.4


def uniform_nodes(nx: int, ny: int, x0: float, y0: float, lx: float, ly: float) -> np.ndarray:
    xs = x0 + lx * np.arange(nx + 1) / nx
    ys = y0 + ly * np.arange(ny + 1) / ny
    nodes = np.empty((ny + 1, nx + 1, 2))
    nodes[:, :, 0] = xs[None, :]
    nodes[:, :, 1] = ys[:, None]
    # make the periodic copies exact: last column/row = first + L
    nodes[:, nx, 0] = nodes[:, 0, 0] + lx
    nodes[ny, :, 1] = nodes[0, :, 1] + ly
    return nodes


def perturbed_nodes(nx: int, ny: int, x0: float, y0: float, lx: float, ly: float,
                    frac: float, seed: int) -> np.ndarray:
    """Uniform grid whose interior nodes are moved by iid U(-frac*h, frac*h)
    in x and in y (h = L/N per direction), drawn in (j, i, {x,y}) order."""
    nodes = uniform_nodes(nx, ny, x0, y0, lx, ly)
    rng = np.random.default_rng(seed)
    d = rng.uniform(-1.0, 1.0, size=(ny - 1, nx - 1, 2))
    nodes[1:ny, 1:nx, 0] += frac * (lx / nx) * d[:, :, 0]
    nodes[1:ny, 1:nx, 1] += frac * (ly / ny) * d[:, :, 1]
    return nodes


@dataclass(frozen=True)
class Vortex:
    """Isentropic vortex convected by a uniform stream (Section 5.1, eq. VP_Solution).

    Defaults follow the 2D Euler workloads: free stream (rho,u,v,p)=(1,1,1,1),
    R=1, strength alpha=5, phi=1/2, centre (0,0), periodic box [-5,5]^2.
    """
    rho_inf: float = 1.0
    u_inf: float = 1.0
    v_inf: float = 1.0
    p_inf: float = 1.0
    rgas: float = 1.0
    gamma: float = GAMMA
    alpha: float = 5.0
    phi: float = 0.5
    xc: float = 0.0
    yc: float = 0.0
    xlo: float = -5.0
    ylo: float = -5.0
    lx: float = 10.0
    ly: float = 10.0

    def primitive(self, x, y, t=0.0):
        """(rho, u, v, p) of the exact solution at time t."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        # position relative to the convected centre, wrapped into the periodic box
        xb = x - self.xc - self.u_inf * t
        yb = y - self.yc - self.v_inf * t
        xb = _wrap(xb, self.lx)
        yb = _wrap(yb, self.ly)
        r2 = xb * xb + yb * yb
        ex = np.exp(self.phi * (1.0 - r2))
        du = -self.alpha / (2.0 * math.pi) * yb * ex
        dv = self.alpha / (2.0 * math.pi) * xb * ex
        t_inf = self.p_inf / (self.rho_inf * self.rgas)
        dT = -(self.alpha ** 2) * (self.gamma - 1.0) / (16.0 * self.phi * self.gamma * math.pi ** 2) * ex * ex
        T = t_inf + dT
        # isentropic: p/rho^gamma constant, p = rho R T
        rho = self.rho_inf * (T / t_inf) ** (1.0 / (self.gamma - 1.0))
        p = rho * self.rgas * T
        return rho, self.u_inf + du, self.v_inf + dv, p

    def conservative(self, x, y, t=0.0):
        rho, u, v, p = self.primitive(x, y, t)
        return np.stack([rho, rho * u, rho * v, p / (self.gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def paper_vortex(mach: float = 0.5, speed: str = "magnitude") -> Vortex:
    """The vortex of the paper's own study (Section 5.1): free stream (rho, u, v) = (1, 1, 1)
    at Mach 0.5, R = 1, alpha = 5, phi = 1/2, periodic box [-10, 10]^2 (period 20).  The
    velocity the Mach number refers to is not stated: speed = "magnitude" reads
    Ma = |V|/c with |V| = sqrt(2) (c = 2 sqrt 2, p = 8/1.4), speed = "u" reads Ma = u/c
    (c = 2, p = 4/1.4)."""
    vel = math.sqrt(2.0) if speed == "magnitude" else 1.0
    c = vel / mach
    return Vortex(p_inf=c * c / GAMMA, xlo=-10.0, ylo=-10.0, lx=20.0, ly=20.0)


def _wrap(d, L):
    """Map a displacement into [-L/2, L/2)."""
    return d - L * np.floor(d / L + 0.5)


@dataclass(frozen=True)
class ShearLayer:
    """Doubly periodic shear layer on [0,1]^2 (Navier-Stokes workload).

    u = tanh(80(y-1/4)) for y <= 1/2 and tanh(80(3/4-y)) above; v = 0.05 sin(2 pi x);
    rho = 1; p = 1/(gamma M^2) with M = 0.1.  mu = 1e-4 (Re = 1e4), Pr = 0.71.
    """
    gamma: float = GAMMA
    rgas: float = 1.0
    mach: float = 0.1
    width: float = 80.0
    amp: float = 0.05
    mu: float = 1e-4
    prandtl: float = 0.71

    def primitive(self, x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        ym = y - np.floor(y)
        u = np.where(ym <= 0.5, np.tanh(self.width * (ym - 0.25)), np.tanh(self.width * (0.75 - ym)))
        v = self.amp * np.sin(2.0 * math.pi * x)
        rho = np.ones_like(u)
        p = np.full_like(u, 1.0 / (self.gamma * self.mach ** 2))
        return rho, u, v, p

    def conservative(self, x, y):
        rho, u, v, p = self.primitive(x, y)
        return np.stack([rho, rho * u, rho * v, p / (self.gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def ogrid_nodes(nx: int, ny: int, r0: float = 0.5, r1: float = 100.0, first: float | None = None) -> np.ndarray:
    """O-grid of straight-sided quads around the circle of radius r0 (a cylinder of diameter
    2 r0) out to radius r1: i runs along the angle theta_i = -2 pi i / nx (clockwise, so the
    map from (xi, eta) = (angle index, radius index) has a positive Jacobian), j along the
    radius.  Radii r_j = r0 + first (s^j - 1)/(s - 1) with the ratio s > 1 chosen so that
    r_ny = r1 (bisection); first = None spaces the radii evenly.  Column nx repeats column 0
    exactly (the periodic seam); row 0 lies on the circle (the wall), row ny on the outer
    circle (the far field)."""
    if first is None:
        r = r0 + (r1 - r0) * np.arange(ny + 1) / ny
    else:
        span = r1 - r0
        if first * ny >= span:
            raise ValueError("first layer too thick for a growing spacing")
        lo, hi = 1.0 + 1e-12, 2.0
        while first * (hi ** ny - 1.0) / (hi - 1.0) < span:
            hi *= 2.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if first * (mid ** ny - 1.0) / (mid - 1.0) < span:
                lo = mid
            else:
                hi = mid
        s = 0.5 * (lo + hi)
        r = r0 + first * (s ** np.arange(ny + 1) - 1.0) / (s - 1.0)
        r[ny] = r1
    th = -2.0 * math.pi * np.arange(nx + 1) / nx
    c, sn = np.cos(th), np.sin(th)
    c[nx], sn[nx] = c[0], sn[0]
    nodes = np.empty((ny + 1, nx + 1, 2))
    nodes[:, :, 0] = r[:, None] * c[None, :]
    nodes[:, :, 1] = r[:, None] * sn[None, :]
    return nodes


@dataclass(frozen=True)
class Cylinder:
    """Laminar flow past a circular cylinder of diameter 1 (Section 5.2): Ma = 0.1 and
    Re = 1200 on the diameter and the free stream.  Velocity scale (not stated by the paper):
    the free stream u = 1, so the convective time D/u is the time unit; rho = 1, c = u/Ma = 10,
    p = rho c^2 / gamma, v = 0, mu = rho u D / Re.  The far-field state is the free stream."""
    gamma: float = GAMMA
    rgas: float = 1.0
    mach: float = 0.1
    reynolds: float = 1200.0
    prandtl: float = 0.71
    speed: float = 1.0

    @property
    def mu(self) -> float:
        return self.speed / self.reynolds

    @property
    def p_inf(self) -> float:
        c = self.speed / self.mach
        return c * c / self.gamma

    def far_state(self) -> np.ndarray:
        rho, u, p = 1.0, self.speed, self.p_inf
        return np.array([rho, rho * u, 0.0, p / (self.gamma - 1.0) + 0.5 * rho * u * u])

    def conservative(self, x, y, perturb: float = 0.0):
        """The free stream everywhere (an impulsive start); perturb > 0 adds a small
        cross-stream velocity bump behind the cylinder, v = perturb u exp(-((x - 1.5)^2 + y^2) / 0.5),
        which breaks the mesh's symmetry so that vortex shedding sets in."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        q = self.far_state()
        rho, u = q[0], q[1] / q[0]
        v = perturb * u * np.exp(-((x - 1.5) ** 2 + y ** 2) / 0.5)
        p = self.p_inf
        return np.stack([np.full_like(x, rho), np.full_like(x, rho * u), rho * v,
                         p / (self.gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


class TaylorGreen:
    """Taylor-Green vortex (Section 5.3): u = V0 sin(x/L) cos(y/L) cos(z/L),
    v = -V0 cos(x/L) sin(y/L) cos(z/L), w = 0,
    p = p0 + rho0 V0^2 / 16 (cos(2x/L) + cos(2y/L)) (cos(2z/L) + 2), on [-pi L, pi L]^3,
    Re = rho0 V0 L / mu = 1600, Pr = 0.71, Ma = V0 / c0 = 0.1 (c0 from p0 and rho0),
    density rho = p / (R T0) at the uniform temperature T0 = p0 / (rho0 R)."""

    def __init__(self, L=1.0, V0=1.0, rho0=1.0, mach=0.1, reynolds=1600.0, gamma=GAMMA, rgas=1.0, prandtl=0.71):
        self.L, self.V0, self.rho0, self.gamma, self.rgas, self.prandtl = L, V0, rho0, gamma, rgas, prandtl
        c0 = V0 / mach
        self.p0 = rho0 * c0 * c0 / gamma
        self.mu = rho0 * V0 * L / reynolds

    def conservative(self, x, y, z):
        L, V0 = self.L, self.V0
        u = V0 * np.sin(x / L) * np.cos(y / L) * np.cos(z / L)
        v = -V0 * np.cos(x / L) * np.sin(y / L) * np.cos(z / L)
        w = np.zeros_like(u)
        p = self.p0 + self.rho0 * V0 * V0 / 16.0 * (np.cos(2 * x / L) + np.cos(2 * y / L)) * (np.cos(2 * z / L) + 2.0)
        rho = p / self.p0 * self.rho0
        return np.stack([rho, rho * u, rho * v, rho * w, p / (self.gamma - 1.0) + 0.5 * rho * (u * u + v * v)])



def random_vector(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded standard-normal array (GMRES right-hand sides, Krylov test vectors)."""
    return scale * np.random.default_rng(seed).standard_normal(size=shape)


# Named workloads: mesh size, polynomial degree, domain and mesh seed.
WORKLOADS = {
    "vortex8_p2": dict(nx=8, ny=8, p=2, x0=-5.0, y0=-5.0, lx=10.0, ly=10.0, perturb=0.0, seed=None),
    "vortex64_p3_perturbed": dict(nx=64, ny=64, p=3, x0=-5.0, y0=-5.0, lx=10.0, ly=10.0, perturb=0.1, seed=2),
    "shear256_p3": dict(nx=256, ny=256, p=3, x0=0.0, y0=0.0, lx=1.0, ly=1.0, perturb=0.0, seed=None),
    "vortex512_p4_perturbed": dict(nx=512, ny=512, p=4, x0=-5.0, y0=-5.0, lx=10.0, ly=10.0, perturb=0.1, seed=5),
    # the paper's own vortex study (Section 5.1)
    "vortex50_p6_paper": dict(nx=50, ny=50, p=6, x0=-10.0, y0=-10.0, lx=20.0, ly=20.0, perturb=0.0, seed=None),
    # cylinder O-grids (Section 5.2 sizes: about 5,700 P3 elements, first layer 0.0033, far field at 100)
    "cylinder120x48_p3": dict(ogrid=True, nx=120, ny=48, p=3, r0=0.5, r1=100.0, first=0.0033),
    "cylinder480x192_p3": dict(ogrid=True, nx=480, ny=192, p=3, r0=0.5, r1=100.0, first=0.0033 / 4),
}


def workload_nodes(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    if w.get("ogrid"):
        return ogrid_nodes(w["nx"], w["ny"], w["r0"], w["r1"], w["first"])
    if w["perturb"] > 0.0:
        return perturbed_nodes(w["nx"], w["ny"], w["x0"], w["y0"], w["lx"], w["ly"], w["perturb"], w["seed"])
    return uniform_nodes(w["nx"], w["ny"], w["x0"], w["y0"], w["lx"], w["ly"])
