"""Pins of the 3D hexahedral FR oracle (Section 3 hexahedral forms, BR2; the Taylor-Green
vortex of Section 5.3): kept free stream, conservation, the z-independent reduction to the
2D BR2 residual, axis-permutation symmetry, convergence to the PDE, the Taylor-Green
vortex's initial kinetic energy and dissipation rate, and the SSPRK3 amplification."""
import math

import numpy as np
import pytest

import fr_inputs as fi
from oracle.fr3d import Box3D, NavierStokes3D, dissipation, inviscid_flux, ssprk3_step, viscous_flux
from oracle.problem import make_ns_bc

GAM = 1.4


def _state3d(x, y, z):
    rho = 1.0 + 0.1 * np.sin(x + 0.3) * np.cos(y) * np.cos(z + 0.2)
    u = 0.3 + 0.1 * np.cos(y + z)
    v = -0.2 + 0.1 * np.sin(x - z)
    w = 0.1 + 0.05 * np.cos(x + y)
    p = 1.0 + 0.05 * np.sin(x + y + z)
    return np.stack([rho, rho * u, rho * v, rho * w, p / (GAM - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def _op(n, P, mu=0.05, flux="roe", L=2 * math.pi):
    box = Box3D(n, n, n, [0.0, 0.0, 0.0], [L, L, L], P)
    return NavierStokes3D(box, mu=mu, flux=flux)


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("mu", [0.0, 0.05])
def test_free_stream_and_conservation(flux, mu):
    op = _op(3, 2, mu=mu, flux=flux)
    x, y, z = op.box.points()
    one = np.ones_like(x)
    qf = np.stack([1.2 * one, 0.4 * one, -0.3 * one, 0.2 * one, (1.1 / 0.4 + 0.5 * (0.16 + 0.09 + 0.04) / 1.2) * one])
    assert np.abs(op.residual(qf)).max() < 1e-12
    U = _state3d(x, y, z)
    R = op.residual(U)
    w = op.box.weights()
    for v in range(5):
        assert abs(np.sum(w * R[v])) < 1e-12 * np.sum(w * np.abs(R[v])) + 1e-13


@pytest.mark.parametrize("flux", ["rusanov", "roe"])
@pytest.mark.parametrize("P", [2, 3])
def test_z_independent_flow_is_the_2d_br2_residual(flux, P):
    """w = 0 and no z-dependence: the 3D residual of rho, rho u, rho v, E on every z-slice is
    the 2D BR2 residual on the same uniform quads, and rho w stays at rest."""
    nx, ny, nz, L = 4, 3, 2, 2 * math.pi
    mu = 0.05
    box = Box3D(nx, ny, nz, [0.0, 0.0, 0.0], [L, L, L], P)
    op3 = NavierStokes3D(box, mu=mu, flux=flux)
    op2 = make_ns_bc(fi.uniform_nodes(nx, ny, 0.0, 0.0, L, L), P, mu=mu, flux=flux, viscous="br2")

    def st2(x, y):
        rho = 1.0 + 0.1 * np.sin(x + 0.3) * np.cos(y)
        u = 0.3 + 0.1 * np.cos(y)
        v = -0.2 + 0.1 * np.sin(x)
        p = 1.0 + 0.05 * np.sin(x + y)
        return np.stack([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])
    x, y, z = box.points()
    q2 = st2(x, y)
    U3 = np.stack([q2[0], q2[1], q2[2], np.zeros_like(x), q2[3]])
    R3 = op3.residual(U3)
    x2, y2 = op2.geo.points()
    R2 = op2.residual(st2(x2, y2).reshape(4, op2.nel, -1)).reshape(4, ny, nx, P + 1, P + 1)
    n = P + 1
    R3g = R3.reshape(5, nz, ny, nx, n, n, n)        # [v, ez, ey, ex, c, b, a]
    scale = np.abs(R2).max()
    for ez in range(nz):
        for c in range(n):
            for v3, v2 in ((0, 0), (1, 1), (2, 2), (4, 3)):
                assert np.allclose(R3g[v3, ez, :, :, c], R2[v2], rtol=0, atol=1e-12 * scale)
            assert np.abs(R3g[3, ez, :, :, c]).max() < 1e-13 * scale


def test_axis_permutation_symmetry():
    """Relabelling the axes (x, y, z) -> (y, z, x), with the velocity components permuted
    alike, permutes the residual the same way."""
    P, n = 2, 3
    nx = ny = nz = 3
    L = 2 * math.pi
    box = Box3D(nx, ny, nz, [0.0] * 3, [L] * 3, P)
    op = NavierStokes3D(box, mu=0.05, flux="roe")
    x, y, z = box.points()
    U = _state3d(x, y, z)
    R = op.residual(U).reshape(5, nz, ny, nx, n, n, n)

    def st_perm(x, y, z):          # the same flow seen in axes (X, Y, Z) = (y, z, x)
        q = _state3d(z, x, y)
        return np.stack([q[0], q[2], q[3], q[1], q[4]])
    Up = st_perm(x, y, z)
    Rp = op.residual(Up).reshape(5, nz, ny, nx, n, n, n)
    # element/point index maps: X = y, Y = z, Z = x  ->  new (ex', ey', ez') = (ey, ez, ex), (a', b', c') = (b, c, a)
    Rt = R.transpose(0, 3, 1, 2, 6, 4, 5)            # [v, ex, ez, ey, a, c, b] -> indexed as [v, ez', ey', ex', c', b', a']
    Rt = Rt[[0, 2, 3, 1, 4]]
    assert np.allclose(Rp, Rt, rtol=1e-11, atol=1e-11)


def _flux_div(x, y, z, mu, h=1e-3):
    """-div(F - F_v) of _state3d by 4th-order differences of the exact total flux (exact
    gradients by complex steps)."""
    def total(x, y, z, d):
        q = _state3d(x, y, z)
        grad = [(_state3d(x + 1e-30j * (k == 0), y + 1e-30j * (k == 1), z + 1e-30j * (k == 2)).imag / 1e-30)
                for k in range(3)]
        return inviscid_flux(q, d, GAM) - viscous_flux(q, grad, d, GAM, 1.0, mu, 0.71)
    out = 0.0
    for d in range(3):
        e = [h if k == d else 0.0 for k in range(3)]
        f = lambda s: total(x + s * e[0], y + s * e[1], z + s * e[2], d)
        out = out + (-f(2) + 8 * f(1) - 8 * f(-1) + f(-2)) / (12 * h)
    return -out


@pytest.mark.parametrize("P", [2, 3])
def test_residual_converges_to_pde_rhs(P):
    mu = 0.05
    errs = []
    for n in (2, 4, 8):
        op = _op(n, P, mu=mu)
        x, y, z = op.box.points()
        R = op.residual(_state3d(x, y, z))
        errs.append(np.sqrt(np.mean((R - _flux_div(x, y, z, mu)) ** 2)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[-1] > P - 0.5, (errs, rates)


def test_taylor_green_initial_energy_and_dissipation():
    """E_k(0) = V0^2 / 8 up to the O(M^2) density variation, eps3(0) = 0 (div u = 0) and
    eps1(0) = 2 mu <S:S> / rho0 = 3 mu V0^2 / (4 rho0 L^2), approached as the mesh refines."""
    tg = fi.TaylorGreen()
    errs = []
    for n in (4, 8):
        box = Box3D(n, n, n, [-math.pi] * 3, [2 * math.pi] * 3, 3)
        op = NavierStokes3D(box, mu=tg.mu)
        x, y, z = box.points()
        ek, e1, e3 = dissipation(op, tg.conservative(x, y, z), tg.rho0)
        assert abs(ek - 0.125) < 1e-4 and abs(e3) < 1e-12
        errs.append(abs(e1 - 0.75 * tg.mu))
    assert errs[1] < errs[0] / 8 and errs[1] < 1e-3 * 0.75 * tg.mu


def test_eps3_closed_form_and_constant_pressure():
    """u = a sin x, v = w = 0, rho = 1, p = p0 + b cos x: int p div u dV = a b V / 2, so
    eps3 = -a b / 2, approached as the mesh refines whatever p0 (here the Mach-0.1 size).
    Adding a constant to p does not move eps3 even when the velocity jumps between
    elements (a per-element slope), where int div u dV over the elements is not zero."""
    a, b, gam = 0.01, 0.5, 1.4

    def state(x, p0):
        rho = np.ones_like(x)
        u = a * np.sin(x)
        p = p0 + b * np.cos(x)
        zero = np.zeros_like(x)
        return np.stack([rho, rho * u, zero, zero, p / (gam - 1) + 0.5 * rho * u * u])
    errs = []
    for n in (3, 6):
        box = Box3D(n, 2, 2, [0.0] * 3, [2 * math.pi] * 3, 3)
        op = NavierStokes3D(box, mu=0.0)
        x, _, _ = box.points()
        _, _, e3 = dissipation(op, state(x, 1.0 / (gam * 0.01)), 1.0)
        errs.append(abs(e3 + a * b / 2))
    assert errs[1] < errs[0] / 8 and errs[1] < 1e-3 * a * b / 2
    rng = np.random.default_rng(4)
    box = Box3D(3, 3, 2, [0.0] * 3, [2 * math.pi] * 3, 2)
    op = NavierStokes3D(box, mu=0.0)
    x, _, _ = box.points()
    U = state(x, 1.0)
    U[1] += 0.02 * rng.standard_normal((box.nel, 1, 1, 1)) * x     # u jumps between elements (not
                                                                    # by per-element constants, which telescope)
    _, _, e3 = dissipation(op, U, 1.0)
    U2 = U.copy()
    U2[4] += 70.0 / (gam - 1)                                      # p -> p + 70
    _, _, e3b = dissipation(op, U2, 1.0)
    assert abs(e3b - e3) <= 1e-12 * 70
    # the jumps make int div u dV non-zero: the literal form would move by 70 times it
    w = box.weights()
    raw = op.raw_gradient(U)
    div = (raw[0][1] - U[1] / U[0] * raw[0][0]) / U[0]
    assert abs(70.0 * np.sum(w * div) / np.sum(w)) > 1e3 * abs(e3b - e3) + 1e-6


def test_ssprk3_amplification():
    """On dU/dt = lambda U one step multiplies by 1 + z + z^2/2 + z^3/6, z = lambda dt."""
    class Lin:
        def residual(self, U):
            return -0.7 * U
    U = np.array([1.0, -2.0])
    z = -0.7 * 0.3
    assert np.allclose(ssprk3_step(Lin(), U, 0.3), U * (1 + z + z * z / 2 + z ** 3 / 6), rtol=1e-15)


def _ns_small(nx, ny, nz, P, mu=0.05):
    box = Box3D(nx, ny, nz, [0.0] * 3, [2 * math.pi] * 3, P)
    op = NavierStokes3D(box, mu=mu)
    x, y, z = box.points()
    return box, op, _state3d(x, y, z)


def test_local_residual_and_element_blocks_by_definition():
    """The frozen-neighbour residual at U is R(U), and columns of the element-Jacobi blocks
    (Section 4.5) match the definition: perturb one entry of one element only, evaluate
    the full residual, take that element's rows (one-sided, step 1e-8 max(1, |q|))."""
    from oracle import linear
    box, op, U = _ns_small(3, 2, 2, 2)
    assert np.array_equal(op.local_residual_factory(U)(U), op.residual(U))
    shift = 3.0
    B = linear.ejacobi_blocks(op, U, shift)
    nb = 5 * 27
    assert B.shape == (box.nel, nb, nb)
    q = op.shape(U).reshape(5, box.nel, 27)
    R0 = op.residual(U).reshape(5, box.nel, 27)
    rng = np.random.default_rng(2)
    for j in rng.choice(nb, size=8, replace=False):
        v, k = divmod(int(j), 27)
        for e in range(box.nel):
            qp = q.copy()
            delta = 1e-8 * max(1.0, abs(qp[v, e, k]))
            qp[v, e, k] += delta
            Rp = op.residual(qp.reshape(U.shape)).reshape(5, box.nel, 27)
            col = -(Rp[:, e, :] - R0[:, e, :]).reshape(-1) / delta
            col[j] += shift
            assert np.linalg.norm(B[e, :, j] - col) <= 1e-6 * np.linalg.norm(col), (j, e)


def test_row3_step_local_order_3d():
    """One ROW3 step on the 3D Navier-Stokes residual (generic integrators with the 3D
    element-Jacobi): against SSPRK3 with 50 substeps the local error, relative to the
    step's own change (itself O(dt)), falls like dt^3 (local error dt^4)."""
    from oracle import integrators as I
    from oracle.tableaux import ROW
    box, op, U = _ns_small(2, 2, 2, 2)
    errs = []
    for dt in (0.02, 0.01):
        Ur, _ = I.row_step(op, ROW["ROW3"], dt, U, I.LinOpts(m=30, rtol=1e-12))
        Us = U.copy()
        for _ in range(50):
            Us = ssprk3_step(op, Us, dt / 50)
        errs.append(np.linalg.norm(Ur - Us) / np.linalg.norm(Us - U))
    rate = math.log2(errs[0] / errs[1])
    assert 2.7 < rate < 3.3, (errs, rate)
