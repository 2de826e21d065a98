"""Pins of the oracle's BR2 common gradient and wall / far-field boundaries (Section 3,
eq. com_grad_q and its lifting; the cylinder case of Section 5.2 names the boundaries):
uniform states the boundaries must keep, conservation with the boundary fluxes, no mass
or energy through a wall, supersonic upwinding at a far-field side, consistency of BR2
with the PDE, BR2 against BR1, element blocks against a brute-force Jacobian, and the
O-grid mesh."""
import math

import numpy as np
import pytest

import fr_inputs as fi
from oracle import linear
from oracle.problem import make_ns, make_ns_bc, sample_state
from tests.test_oracle_ns import _exact_rhs, _manufactured

GAM = 1.4


def _channel(nx=5, ny=4, seed=7):
    """Perturbed channel [-5, 5] x [-3, 3]: periodic in x, boundaries at y = -3 and y = 3."""
    return fi.perturbed_nodes(nx, ny, -5, -3, 10, 6, 0.1, seed)


def _prim_state(op, rho, u, v, p):
    one = np.ones((op.nel, op.n * op.n))
    return np.stack([rho * one, rho * u * one, rho * v * one, (p / (GAM - 1) + 0.5 * rho * (u * u + v * v)) * one])


def _wavy_state(op, seed=3):
    """A smooth non-uniform state with nonzero velocity at the walls."""
    def fn(x, y):
        rho = 1.0 + 0.1 * np.sin(0.7 * x + 0.3) * np.cos(0.5 * y)
        u = 0.4 + 0.1 * np.cos(0.6 * y + 0.2 * x)
        v = 0.1 * np.sin(0.9 * x) * np.cos(0.4 * y)
        p = 1.0 + 0.05 * np.cos(0.5 * x - 0.4 * y)
        return np.stack([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])
    return sample_state(op, fn)


def _weighted_total(op, R):
    w = op.b.w
    wk = (w[:, None] * w[None, :]).reshape(-1)
    J = op.geo.J.reshape(op.nel, -1)
    return np.einsum("k,ek,vek->v", wk, J, R.reshape(4, op.nel, -1))


@pytest.mark.parametrize("viscous", ["br1", "br2"])
@pytest.mark.parametrize("P", [2, 3])
def test_uniform_states_kept(viscous, P):
    """Free stream with far-field sides equal to it, and fluid at rest between walls."""
    qf = np.array([1.2, 1.2 * 0.7, 1.2 * -0.4, 0.9 / (GAM - 1) + 0.5 * 1.2 * (0.49 + 0.16)])
    op = make_ns_bc(_channel(), P, mu=0.05, viscous=viscous, bc_south="farfield", bc_north="farfield", q_far=qf)
    U = _prim_state(op, 1.2, 0.7, -0.4, 0.9)
    assert np.abs(op.residual(U)).max() < 1e-12
    opw = make_ns_bc(_channel(), P, mu=0.05, viscous=viscous, bc_south="wall", bc_north="wall")
    assert np.abs(opw.residual(_prim_state(opw, 0.8, 0.0, 0.0, 1.3))).max() < 1e-12
    # BR2 on a periodic mesh keeps a free stream too
    opp = make_ns_bc(fi.perturbed_nodes(5, 4, -5, -5, 10, 10, 0.1, 7), P, mu=0.05, viscous=viscous)
    assert np.abs(opp.residual(_prim_state(opp, 1.2, 0.7, -0.4, 0.9))).max() < 1e-12


@pytest.mark.parametrize("viscous", ["br1", "br2"])
@pytest.mark.parametrize("bcs", [("wall", "wall"), ("wall", "farfield"), ("farfield", "farfield")])
def test_conservation_with_boundary_fluxes(viscous, bcs):
    """sum_e sum_k w J R = (flux in through the eta = -1 side) - (flux out through eta = +1):
    interior faces cancel exactly; the boundary fluxes are what the residual used.  At a
    wall neither mass nor energy passes."""
    qf = np.array([1.0, 0.3, 0.05, 1.0 / (GAM - 1) + 0.5 * (0.09 + 0.0025)])
    op = make_ns_bc(_channel(), 3, mu=0.05, viscous=viscous, bc_south=bcs[0], bc_north=bcs[1], q_far=qf)
    U = _wavy_state(op)
    tot = _weighted_total(op, op.residual(U))
    bf = op.boundary_fluxes(U)
    w = op.b.w
    expect = np.einsum("a,vea->v", w, bf["S"]) - np.einsum("a,vea->v", w, bf["N"])
    scale = np.abs(np.einsum("a,vea->v", w, np.abs(bf["S"])) + np.einsum("a,vea->v", w, np.abs(bf["N"])))
    assert np.all(np.abs(tot - expect) <= 1e-12 * (1.0 + scale)), (tot, expect)
    for side in ("S", "N"):
        if op.bc[side] == "wall":
            assert np.abs(bf[side][0]).max() == 0.0 and np.abs(bf[side][3]).max() == 0.0
    if bcs == ("wall", "wall"):
        assert abs(tot[0]) < 1e-12 and abs(tot[3]) < 1e-12


def test_farfield_upwinds_supersonic_flow():
    """Inviscid, Roe flux, flow at Mach 2 in +y: the inflow side (eta = -1) takes the far-field
    flux whatever the interior is, the outflow side (eta = +1) the interior trace's flux."""
    rho, u, v, p = 1.0, 0.1, 2.0 * math.sqrt(GAM), 1.0
    qf = np.array([rho, rho * u, rho * v, p / (GAM - 1) + 0.5 * rho * (u * u + v * v)])
    op = make_ns_bc(fi.uniform_nodes(4, 3, -2, -1.5, 4, 3), 2, mu=0.0, flux="roe", bc_south="farfield",
                    bc_north="farfield", q_far=qf)
    # interior: also supersonic in +y, but a different state
    r2, u2, v2, p2 = 0.9, -0.05, 1.9 * math.sqrt(GAM * 1.1 / 0.9), 1.1
    U = _prim_state(op, r2, u2, v2, p2)
    bf = op.boundary_fluxes(U)
    from oracle.euler import normal_flux
    S_s = op.geo.SS[:, op.on_bnd["S"]]
    S_n = op.geo.SN[:, op.on_bnd["N"]]
    q2 = U[:, 0, 0]
    f_far = normal_flux(qf.reshape(4, 1, 1), S_s[0], S_s[1], GAM)
    f_in = normal_flux(q2.reshape(4, 1, 1), S_n[0], S_n[1], GAM)
    assert np.allclose(bf["S"], f_far, rtol=1e-13, atol=1e-13)
    assert np.allclose(bf["N"], f_in, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_br2_residual_converges_to_pde_rhs(P):
    mu = 0.05
    errs = []
    for n in (4, 8, 16):
        op = make_ns_bc(fi.uniform_nodes(n, n, -5, -5, 10, 10), P, mu=mu, viscous="br2")
        U = sample_state(op, _manufactured)
        R = op.residual(U).reshape(4, op.nel, -1)
        x, y = op.geo.points()
        errs.append(np.sqrt(np.mean((R - _exact_rhs(x, y, mu)) ** 2)))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > P - 0.5, (errs, rates)


def test_br2_differs_from_br1_and_periodic_br1_is_the_ns_module():
    nodes = fi.perturbed_nodes(5, 4, -5, -5, 10, 10, 0.1, 7)
    op1 = make_ns_bc(nodes, 3, mu=0.05, viscous="br1")
    op2 = make_ns_bc(nodes, 3, mu=0.05, viscous="br2")
    ref = make_ns(nodes, 3, mu=0.05)
    U = sample_state(op1, _manufactured)
    R1, R2 = op1.residual(U), op2.residual(U)
    assert np.array_equal(R1, ref.residual(U))
    d = np.linalg.norm(R2 - R1) / np.linalg.norm(R1)
    assert 1e-6 < d < 1e-1, d
    # the difference is viscous: it vanishes with mu
    op1i = make_ns_bc(nodes, 3, mu=0.0, viscous="br1")
    op2i = make_ns_bc(nodes, 3, mu=0.0, viscous="br2")
    assert np.array_equal(op1i.residual(U), op2i.residual(U))


@pytest.mark.parametrize("viscous", ["br1", "br2"])
@pytest.mark.parametrize("bcs", [("wall", "farfield"), ("farfield", "wall")])
def test_blocks_match_bruteforce_with_boundaries(viscous, bcs):
    qf = np.array([1.0, 0.3, 0.05, 1.0 / (GAM - 1) + 0.5 * (0.09 + 0.0025)])
    op = make_ns_bc(_channel(4, 3, seed=9), 2, mu=0.05, viscous=viscous, bc_south=bcs[0], bc_north=bcs[1],
                    q_far=qf)
    U = _wavy_state(op)
    local = op.local_residual_factory(U)
    assert np.allclose(local(op.shape(U)).reshape(U.shape), op.residual(U), rtol=1e-13, atol=1e-13)
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
        assert np.linalg.norm(blocks[el] - ref) <= 1e-6 * np.linalg.norm(ref), el


def test_wall_force():
    """At rest with uniform pressure the closed wall feels no force; between two walls of a
    channel the residual's momentum total is the momentum the walls take (conservation),
    the wall force being minus the momentum flux through the wall faces."""
    op = make_ns_bc(fi.ogrid_nodes(12, 4, 0.5, 5.0, 0.05), 3, mu=0.01, bc_south="wall", bc_north="farfield",
                    q_far=np.array([1.0, 0.0, 0.0, 1.0 / (GAM - 1)]))
    assert np.abs(op.wall_force(_prim_state(op, 1.0, 0.0, 0.0, 1.0))).max() < 1e-12
    opc = make_ns_bc(_channel(), 3, mu=0.05, viscous="br2", bc_south="wall", bc_north="wall")
    U = _wavy_state(opc)
    tot = _weighted_total(opc, opc.residual(U))
    bf = opc.boundary_fluxes(U)
    w = opc.b.w
    north = np.einsum("a,vea->v", w, bf["N"])[1:3]
    assert np.allclose(tot[1:3], -opc.wall_force(U) - north, rtol=1e-12, atol=1e-12)
    # a pressure difference along a straight wall pushes on it: on the channel's lower wall
    # (normal +y into the fluid) the force is -y times the integrated pressure
    Ur = _prim_state(opc, 1.0, 0.0, 0.0, 2.0)
    f = opc.wall_force(Ur)
    assert abs(f[0]) < 1e-12 and abs(f[1] + 2.0 * 10.0) < 1e-11


def test_ogrid_mesh():
    nx, ny, r0, r1, h = 24, 10, 0.5, 20.0, 0.01
    nodes = fi.ogrid_nodes(nx, ny, r0, r1, h)
    r = np.hypot(nodes[..., 0], nodes[..., 1])
    assert np.allclose(r[0], r0, rtol=0, atol=1e-15) and np.allclose(r[ny], r1, rtol=0, atol=1e-12)
    assert np.array_equal(nodes[:, nx], nodes[:, 0])
    assert abs((r[1, 0] - r[0, 0]) - h) < 1e-12
    op = make_ns_bc(nodes, 2, bc_south="wall", bc_north="farfield", q_far=np.array([1.0, 0.1, 0.0, 2.5]))
    assert op.geo.J.min() > 0
    w = op.b.w
    area = np.einsum("a,b,eba->", w, w, op.geo.J)
    polygon = 0.5 * nx * math.sin(2 * math.pi / nx) * (r1 ** 2 - r0 ** 2)
    assert abs(area - polygon) < 1e-10 * polygon


@pytest.mark.parametrize("P", [2, 3, 4])
def test_br2_common_gradient_closed_form(P):
    """Piecewise-constant state, uniform unit squares: inside an element every raw gradient
    vanishes, so the BR2 common gradient on an x-face is the two liftings' mean,
    c_P |grad xi| (q+ - q-) / 2 + c_P |grad xi| (q+ - q-) / 2 = (P+1)(P+2)/2 * jump / h
    along +x (|grad xi| = 2/h, q^com - q_local = +-jump/2 with the outward normals +-x)."""
    nx, ny, h = 4, 3, 1.0
    op = make_ns_bc(fi.uniform_nodes(nx, ny, 0.0, 0.0, nx * h, ny * h), P, mu=0.05, viscous="br2")
    ucol = np.array([0.1, 0.3, -0.2, 0.25])
    n = P + 1
    u = np.repeat(ucol[op.mesh.ex][:, None], n * n, axis=1)
    one = np.ones_like(u)
    U = np.stack([one, u, 0 * one, (1.0 / (GAM - 1)) * one + 0.5 * u * u])
    g = op.face_common_gradients(U)
    cP = (P + 1) * (P + 2) / 2.0
    east = op.mesh.east
    jump = U[:, east, 0] - U[:, :, 0]                        # [v, e]: q(east neighbour) - q
    expect = cP * jump / h
    gx, gy = g["E"]
    assert np.allclose(gx, expect[:, :, None], rtol=1e-13, atol=1e-13)
    assert np.abs(gy).max() < 1e-13
    assert np.abs(g["N"][0]).max() < 1e-13 and np.abs(g["N"][1]).max() < 1e-13
