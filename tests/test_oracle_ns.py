"""Pins of the oracle's BR1 Navier-Stokes residual (Sections 2-3) against
invariants, the inviscid limit, the PDE itself and a brute-force Jacobian."""
import math

import numpy as np
import pytest

import fr_inputs as fi
from oracle import euler, linear
from oracle.ns import viscous_flux
from oracle.problem import make_euler, make_ns, sample_state

GAM = 1.4


def _manufactured(x, y):
    k = 2 * math.pi / 10.0
    rho = 1.0 + 0.2 * np.sin(k * x) * np.cos(k * y)
    u = 1.0 + 0.1 * np.sin(k * y)
    v = 0.5 + 0.1 * np.cos(k * x)
    p = 1.0 + 0.1 * np.sin(k * (x + y))
    return np.stack([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])


def _total_flux(x, y, mu):
    h = 1e-30
    q = _manufactured(x, y)
    qx = _manufactured(x + 1j * h, y + 0j).imag / h       # exact gradient (complex step)
    qy = _manufactured(x + 0j, y + 1j * h).imag / h
    f, g = euler.physical_flux(q, GAM)
    fv, gv = viscous_flux(q, qx, qy, GAM, 1.0, mu, 0.71)
    return f - fv, g - gv


def _exact_rhs(x, y, mu, h=1e-3):
    """-div(F - F_v) of the manufactured field: 4th-order differences of the exact flux."""
    fx = (-_total_flux(x + 2 * h, y, mu)[0] + 8 * _total_flux(x + h, y, mu)[0]
          - 8 * _total_flux(x - h, y, mu)[0] + _total_flux(x - 2 * h, y, mu)[0]) / (12 * h)
    gy = (-_total_flux(x, y + 2 * h, mu)[1] + 8 * _total_flux(x, y + h, mu)[1]
          - 8 * _total_flux(x, y - h, mu)[1] + _total_flux(x, y - 2 * h, mu)[1]) / (12 * h)
    return -(fx + gy)


def test_viscous_flux_of_a_shear_and_a_temperature_gradient():
    # u = a y (simple shear): tau_xy = mu a, energy flux u tau_xy; rho = 1, p const
    mu, a = 0.3, 2.0
    y = np.array([0.7])
    rho, u, v, p = 1.0, a * y, 0.0 * y, 1.0
    q = np.stack([rho + 0 * y, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * u * u])
    qx = np.zeros_like(q)
    qy = np.stack([0 * y, rho * a + 0 * y, 0 * y, rho * u * a])
    fv, gv = viscous_flux(q, qx, qy, GAM, 1.0, mu, 0.71)
    assert np.allclose(fv[:, 0], [0, 0, mu * a, 0]) and np.allclose(gv[:, 0], [0, mu * a, 0, u[0] * mu * a])
    # at rest with T = p/(rho R) varying in x through rho only: heat flux kappa dT/dx
    x = np.array([0.3])
    rho = 1.0 + 0.1 * x
    q = np.stack([rho, 0 * x, 0 * x, 1.0 / (GAM - 1) + 0 * x])
    qx = np.stack([0.1 + 0 * x, 0 * x, 0 * x, 0 * x])
    fv, _ = viscous_flux(q, qx, np.zeros_like(q), GAM, 1.0, mu, 0.71)
    kappa = mu * (GAM / (GAM - 1)) / 0.71
    dTdx = -1.0 * 0.1 / rho ** 2            # T = p / rho with p = 1
    assert np.allclose(fv[3], kappa * dTdx)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_ns_freestream_and_conservation(P):
    op = make_ns(fi.perturbed_nodes(5, 4, -5, -5, 10, 10, 0.1, 7), P, mu=0.1)
    one = np.ones((op.nel, (P + 1) ** 2))
    Uf = np.stack([1.2 * one, 0.84 * one, -0.48 * one, (0.9 / 0.4 + 0.5 * 1.2 * (0.49 + 0.16)) * one])
    assert np.abs(op.residual(Uf)).max() < 1e-12
    U = sample_state(op, _manufactured)
    R = op.residual(U).reshape(4, op.nel, -1)
    w = op.b.w
    wk = (w[:, None] * w[None, :]).reshape(-1)
    J = op.geo.J.reshape(op.nel, -1)
    for var in range(4):
        assert abs(np.sum(wk * J * R[var])) < 1e-12


def test_ns_inviscid_limit_is_the_euler_residual():
    nodes = fi.perturbed_nodes(5, 4, -5, -5, 10, 10, 0.1, 7)
    v = fi.Vortex()
    for flux in ("rusanov", "roe"):
        op0, ope = make_ns(nodes, 3, mu=0.0, flux=flux), make_euler(nodes, 3, flux=flux)
        U = sample_state(ope, lambda x, y: v.conservative(x, y, 0.3))
        assert np.array_equal(op0.residual(U), ope.residual(U))


@pytest.mark.parametrize("P", [2, 3, 4])
def test_ns_residual_converges_to_pde_rhs(P):
    mu = 0.05
    errs = []
    for n in (4, 8, 16):
        op = make_ns(fi.uniform_nodes(n, n, -5, -5, 10, 10), P, mu=mu)
        U = sample_state(op, _manufactured)
        R = op.residual(U).reshape(4, op.nel, -1)
        x, y = op.geo.points()
        errs.append(np.sqrt(np.mean((R - _exact_rhs(x, y, mu)) ** 2)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > P - 0.5, (errs, rates)


def test_ns_element_local_residual_and_blocks_match_bruteforce():
    op = make_ns(fi.perturbed_nodes(4, 4, -5, -5, 10, 10, 0.1, 9), 2, mu=0.05)
    v = fi.Vortex()
    U = sample_state(op, lambda x, y: v.conservative(x, y, 0.2))
    local = op.local_residual_factory(U)
    assert np.array_equal(local(op.shape(U)).reshape(U.shape), op.residual(U))
    N = U.size
    Uf = U.reshape(-1)
    J = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = 1e-6
        J[:, j] = (op.residual((Uf + e).reshape(U.shape)) - op.residual((Uf - e).reshape(U.shape))).reshape(-1) / 2e-6
    shift = 3.0
    blocks = linear.ejacobi_blocks(op, U, shift)
    Np = 9
    for el in range(op.nel):
        idx = np.array([(var * op.nel + el) * Np + k for var in range(4) for k in range(Np)])
        ref = shift * np.eye(4 * Np) - J[np.ix_(idx, idx)]
        assert np.linalg.norm(blocks[el] - ref) <= 1e-6 * np.linalg.norm(ref)
    # the neighbour-gradient path matters: dropping it (Euler-style frozen traces only) is wrong
    R0 = op.residual(U)
    vv = fi.random_vector(U.shape, seed=4)
    Av = linear.jf_matvec(op.residual, U, R0, vv, shift)
    assert np.linalg.norm(Av.reshape(-1) - (shift * vv.reshape(-1) - J @ vv.reshape(-1))) <= 1e-6 * np.linalg.norm(Av)


def test_ns_symmetries():
    P, nx, ny = 3, 5, 4
    nodes = fi.perturbed_nodes(nx, ny, -5, -5, 10, 10, 0.1, seed=5)
    rng = np.random.default_rng(4)
    n = P + 1
    op = make_ns(nodes, P, mu=0.05, flux="roe")
    shape = (op.nel, n, n)
    rho = rng.uniform(0.9, 1.1, shape)
    u = 0.3 + rng.uniform(-0.1, 0.1, shape)
    w = -0.2 + rng.uniform(-0.1, 0.1, shape)
    p = rng.uniform(0.9, 1.1, shape)
    q = np.stack([rho, rho * u, rho * w, p / (GAM - 1) + 0.5 * rho * (u * u + w * w)])
    R = op.residual(q.reshape(4, op.nel, -1)).reshape(4, ny, nx, n, n)
    qg = q.reshape(4, ny, nx, n, n)
    nodes_t = nodes.transpose(1, 0, 2)[:, :, ::-1].copy()
    op_t = make_ns(nodes_t, P, mu=0.05, flux="roe")
    q_t = qg.transpose(0, 2, 1, 4, 3)[[0, 2, 1, 3]]
    R_t = op_t.residual(q_t.reshape(4, -1, n * n)).reshape(4, nx, ny, n, n)
    assert np.allclose(R_t, R.transpose(0, 2, 1, 4, 3)[[0, 2, 1, 3]], rtol=1e-11, atol=1e-11)
    op_r = make_ns(-nodes[::-1, ::-1], P, mu=0.05, flux="roe")
    sgn = np.array([1, -1, -1, 1])[:, None, None, None, None]
    R_r = op_r.residual((qg[:, ::-1, ::-1, ::-1, ::-1] * sgn).reshape(4, -1, n * n)).reshape(4, ny, nx, n, n)
    assert np.allclose(R_r, R[:, ::-1, ::-1, ::-1, ::-1] * sgn, rtol=1e-11, atol=1e-11)
