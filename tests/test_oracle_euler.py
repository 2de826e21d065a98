"""Pins of the oracle's FR Euler residual (Section 3) against invariants,
closed forms and the PDE itself."""
import math

import numpy as np
import pytest

import fr_inputs as fi
from oracle import euler
from oracle.problem import make_euler, sample_state

GAM = 1.4


def _freestream(x, y, rho=1.0, u=1.0, v=1.0, p=1.0):
    one = np.ones_like(x)
    return np.stack([rho * one, rho * u * one, rho * v * one, (p / (GAM - 1) + 0.5 * rho * (u * u + v * v)) * one])


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_freestream_preserved_on_perturbed_mesh(P, flux):
    nodes = fi.perturbed_nodes(5, 4, -5, -5, 10, 10, 0.1, seed=7)
    op = make_euler(nodes, P, flux=flux)
    U = sample_state(op, lambda x, y: _freestream(x, y, 1.2, 0.7, -0.4, 0.9))
    R = op.residual(U)
    # |F| ~ 3, 1/h ~ 0.5: the residual is exactly zero in exact arithmetic
    assert np.abs(R).max() < 1e-12


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_discrete_conservation(P, flux):
    nodes = fi.perturbed_nodes(6, 5, -5, -5, 10, 10, 0.1, seed=3)
    op = make_euler(nodes, P, flux=flux)
    v = fi.Vortex()
    U = sample_state(op, lambda x, y: v.conservative(x, y, 0.3))
    R = op.residual(U).reshape(4, op.nel, -1)
    w = op.b.w
    wk = (w[:, None] * w[None, :]).reshape(-1)
    J = op.geo.J.reshape(op.nel, -1)
    scale = np.sum(wk * J * np.abs(R[0]))
    for var in range(4):
        assert abs(np.sum(wk * J * R[var])) < 1e-13 * max(1.0, scale) * 100


def _rand_state(rng, shape, mach_hi=0.8):
    rho = rng.uniform(0.5, 1.5, shape)
    u = rng.uniform(-mach_hi, mach_hi, shape)
    v = rng.uniform(-mach_hi, mach_hi, shape)
    p = rng.uniform(0.7, 1.3, shape)
    return np.stack([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])


@pytest.mark.parametrize("name", ["rusanov", "roe"])
def test_common_flux_consistent(name):
    rng = np.random.default_rng(0)
    q = _rand_state(rng, 50)
    th = rng.uniform(0, 2 * math.pi, 50)
    nx, ny = np.cos(th), np.sin(th)
    fc = euler.FLUXES[name](q, q, nx, ny, GAM)
    assert np.allclose(fc, euler.normal_flux(q, nx, ny, GAM), rtol=1e-14, atol=1e-14)


def test_roe_upwinds_supersonic_states():
    # With every eigenvalue positive, the Roe flux is the left flux exactly; this holds only
    # if the averaged matrix satisfies A(qR - qL) = f(qR) - f(qL) (Roe's property).
    rng = np.random.default_rng(1)
    n = 40
    rho = rng.uniform(0.5, 1.5, (2, n))
    p = rng.uniform(0.5, 1.0, (2, n))
    u = rng.uniform(3.0, 4.0, (2, n))
    v = rng.uniform(-0.3, 0.3, (2, n))
    q = np.stack([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])
    qL, qR = q[:, 0], q[:, 1]
    fc = euler.roe(qL, qR, 1.0, 0.0, GAM)
    assert np.allclose(fc, euler.normal_flux(qL, 1.0, 0.0, GAM), rtol=1e-13, atol=1e-13)


def _flux_jacobian(q, nx, ny):
    """dF_n/dq by complex step (exact to rounding): columns j."""
    A = np.zeros((4, 4))
    h = 1e-30
    for j in range(4):
        qc = q.astype(complex)
        qc[j] += 1j * h
        A[:, j] = (euler.normal_flux(qc, nx, ny, GAM)).imag / h
    return A


def test_roe_dissipation_matches_eigendecomposition():
    # Independent route: |A| = V |Lambda| V^{-1} of the flux Jacobian at the Roe-averaged state.
    rng = np.random.default_rng(2)
    for _ in range(20):
        qL = _rand_state(rng, 1)[:, 0]
        qR = _rand_state(rng, 1)[:, 0]
        th = rng.uniform(0, 2 * math.pi)
        nx, ny = math.cos(th), math.sin(th)
        sl, sr = math.sqrt(qL[0]), math.sqrt(qR[0])
        u = (qL[1] / sl + qR[1] / sr) / (sl + sr)
        v = (qL[2] / sl + qR[2] / sr) / (sl + sr)
        HL = (qL[3] + euler.pressure(qL, GAM)) / qL[0]
        HR = (qR[3] + euler.pressure(qR, GAM)) / qR[0]
        H = (sl * HL + sr * HR) / (sl + sr)
        rho = sl * sr
        p = (GAM - 1) * rho * (H - 0.5 * (u * u + v * v)) / GAM
        qhat = np.array([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])
        A = _flux_jacobian(qhat, nx, ny)
        lam, V = np.linalg.eig(A)
        absA = (V @ np.diag(np.abs(lam)) @ np.linalg.inv(V)).real
        expect = 0.5 * (euler.normal_flux(qL, nx, ny, GAM) + euler.normal_flux(qR, nx, ny, GAM)) - 0.5 * absA @ (qR - qL)
        got = euler.roe(qL[:, None], qR[:, None], nx, ny, GAM)[:, 0]
        assert np.allclose(got, expect, rtol=1e-10, atol=1e-10)


def _smooth_rand_state(rng, shape):
    """Random state close to a uniform stream: positive pressure at every face trace."""
    rho = rng.uniform(0.9, 1.1, shape)
    u = 0.3 + rng.uniform(-0.1, 0.1, shape)
    v = -0.2 + rng.uniform(-0.1, 0.1, shape)
    p = rng.uniform(0.9, 1.1, shape)
    return np.stack([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])


def _manufactured(x, y):
    k = 2 * math.pi / 10.0
    rho = 1.0 + 0.2 * np.sin(k * x) * np.cos(k * y)
    u = 1.0 + 0.1 * np.sin(k * y)
    v = 0.5 + 0.1 * np.cos(k * x)
    p = 1.0 + 0.1 * np.sin(k * (x + y))
    return np.stack([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])


def _exact_rhs(x, y):
    """-(df/dx + dg/dy) of the manufactured field, by complex-step differentiation."""
    h = 1e-30
    f, _ = euler.physical_flux(_manufactured(x + 1j * h, y + 0j), GAM)
    _, g = euler.physical_flux(_manufactured(x + 0j, y + 1j * h), GAM)
    return -(f.imag + g.imag) / h


@pytest.mark.parametrize("P", [2, 3])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_residual_converges_to_pde_rhs(P, flux):
    # R(q_exact) -> -div F(q_exact) under h-refinement, at least at order P
    errs = []
    for n in (4, 8, 16):
        nodes = fi.uniform_nodes(n, n, -5, -5, 10, 10)
        op = make_euler(nodes, P, flux=flux)
        U = sample_state(op, _manufactured)
        R = op.residual(U).reshape(4, op.nel, -1)
        x, y = op.geo.points()
        ex = _exact_rhs(x, y)
        errs.append(np.sqrt(np.mean((R - ex) ** 2)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > P - 0.3, (errs, rates)


def test_residual_symmetries():
    # transposition (x,y)->(y,x) and rotation by 180 degrees map the discrete residual
    # onto itself with the state's components permuted / sign-flipped
    P, nx, ny = 3, 5, 4
    nodes = fi.perturbed_nodes(nx, ny, -5, -5, 10, 10, 0.1, seed=5)
    rng = np.random.default_rng(4)
    for flux in ("rusanov", "roe"):
        op = make_euler(nodes, P, flux=flux)
        n = P + 1
        q = _smooth_rand_state(rng, (op.nel, n, n))
        R = op.residual(q.reshape(4, op.nel, -1)).reshape(4, ny, nx, n, n)
        qg = q.reshape(4, ny, nx, n, n)
        # transpose
        nodes_t = nodes.transpose(1, 0, 2)[:, :, ::-1].copy()
        op_t = make_euler(nodes_t, P, flux=flux)
        q_t = qg.transpose(0, 2, 1, 4, 3)[[0, 2, 1, 3]]
        R_t = op_t.residual(q_t.reshape(4, -1, n * n)).reshape(4, nx, ny, n, n)
        assert np.allclose(R_t, R.transpose(0, 2, 1, 4, 3)[[0, 2, 1, 3]], rtol=1e-11, atol=1e-11)
        # rotate by 180 degrees
        nodes_r = -nodes[::-1, ::-1]
        op_r = make_euler(nodes_r, P, flux=flux)
        q_r = qg[:, ::-1, ::-1, ::-1, ::-1] * np.array([1, -1, -1, 1])[:, None, None, None, None]
        R_r = op_r.residual(q_r.reshape(4, -1, n * n)).reshape(4, ny, nx, n, n)
        expect = R[:, ::-1, ::-1, ::-1, ::-1] * np.array([1, -1, -1, 1])[:, None, None, None, None]
        assert np.allclose(R_r, expect, rtol=1e-11, atol=1e-11)
