"""Pins of the oracle's p-multigrid preconditioner (Section 4.5 names it beside
element-Jacobi): the transfers are exact interpolation and L2 projection (closed forms
on polynomials), the V-cycle equals its dense-matrix composition, and FGMRES needs
fewer iterations with it than with element-Jacobi."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import fr_inputs as fi
from oracle import linear
from oracle.basis import gauss_points
from oracle.pmg import PMultigrid, apply_2d, transfer_1d
from oracle.problem import make_euler, sample_state


@pytest.mark.parametrize("P,Pc", [(3, 2), (4, 2), (6, 4), (5, 3)])
def test_transfers_on_polynomials(P, Pc):
    Pi, I = transfer_1d(P, Pc)
    xf, _ = gauss_points(P)
    xc, _ = gauss_points(Pc)
    rng = np.random.default_rng(P * 10 + Pc)
    # interpolation of a coarse polynomial is exact at the fine points
    c = rng.standard_normal(Pc + 1)
    assert np.allclose(I @ npleg.legval(xc, c), npleg.legval(xf, c), atol=1e-13)
    # projection reproduces polynomials of degree <= Pc and undoes interpolation
    assert np.allclose(Pi @ npleg.legval(xf, c), npleg.legval(xc, c), atol=1e-13)
    assert np.allclose(Pi @ I, np.eye(Pc + 1), atol=1e-13)
    # it annihilates the Legendre polynomials of degree Pc+1 .. P (orthogonal to degree <= Pc)
    for k in range(Pc + 1, P + 1):
        e = np.zeros(k + 1)
        e[k] = 1.0
        assert np.allclose(Pi @ npleg.legval(xf, e), 0.0, atol=1e-13)


def test_2d_transfer_is_the_tensor_product():
    P, Pc = 4, 2
    Pi, I = transfer_1d(P, Pc)
    v = np.random.default_rng(0).standard_normal((4, 3, (P + 1) ** 2))
    out = apply_2d(Pi, v, 3, P + 1)
    K = np.kron(Pi, Pi)            # k = b n + a: the eta index is the slow one
    for var in range(4):
        for e in range(3):
            assert np.allclose(out[var, e], K @ v[var, e], atol=1e-14)


def _case(nx, ny, P, Pc, flux="roe", seed=3):
    nodes = fi.perturbed_nodes(nx, ny, -5, -5, 10, 10, 0.1, seed)
    op = make_euler(nodes, P, flux=flux)
    opc = make_euler(nodes, Pc, flux=flux)
    vx = fi.Vortex()
    return op, opc, sample_state(op, lambda x, y: vx.conservative(x, y, 0.3))


def _dense(residual, U, shift, h=1e-6):
    u = U.reshape(-1)
    A = np.empty((u.size, u.size))
    for j in range(u.size):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        A[:, j] = -(residual(up.reshape(U.shape)) - residual(um.reshape(U.shape))).reshape(-1) / (2 * h)
        A[j, j] += shift
    return A


def test_vcycle_equals_dense_composition():
    op, opc, U = _case(3, 2, 3, 2)
    shift = 4.0
    mg = PMultigrid(op, opc, U, shift, nu1=1, nu2=1, nc=2)
    A = _dense(op.residual, U, shift)
    Ac = _dense(opc.residual, mg.Uc, shift)

    def blockinv(pc, n_per):
        nel = op.nel
        Minv = np.zeros((4 * nel * n_per, 4 * nel * n_per))
        for e in range(nel):
            idx = np.array([v * nel * n_per + e * n_per + k for v in range(4) for k in range(n_per)])
            Minv[np.ix_(idx, idx)] = np.linalg.inv(pc.blocks[e])
        return Minv

    Dinv, Dcinv = blockinv(mg.D, 16), blockinv(mg.Dc, 9)
    nel = op.nel
    Pi, I = transfer_1d(3, 2)
    R2 = np.zeros((4 * nel * 9, 4 * nel * 16))
    I2 = np.zeros((4 * nel * 16, 4 * nel * 9))
    for v in range(4):
        for e in range(nel):
            rc = slice(v * nel * 9 + e * 9, v * nel * 9 + e * 9 + 9)
            rf = slice(v * nel * 16 + e * 16, v * nel * 16 + e * 16 + 16)
            R2[rc, rf] = np.kron(Pi, Pi)
            I2[rf, rc] = np.kron(I, I)
    r = fi.random_vector(U.shape, seed=4).reshape(-1)
    z = Dinv @ r
    rc = R2 @ (r - A @ z)
    zc = Dcinv @ rc
    zc = zc + Dcinv @ (rc - Ac @ zc)
    z = z + I2 @ zc
    z = z + Dinv @ (r - A @ z)
    zm = mg.apply(r.reshape(U.shape)).reshape(-1)
    assert np.linalg.norm(zm - z) <= 1e-6 * np.linalg.norm(z)


def test_fgmres_needs_fewer_iterations_with_pmg():
    op, opc, U = _case(8, 8, 4, 2, flux="rusanov")
    R0 = op.residual(U)
    shift = 1.0 / (0.25 * 0.4)

    def A(v):
        return linear.jf_matvec(op.residual, U, R0, v, shift)

    _, sj = linear.fgmres(A, linear.ElementJacobi(op, U, shift).apply, R0, m=30, rtol=1e-8)
    x, sm = linear.fgmres(A, PMultigrid(op, opc, U, shift).apply, R0, m=30, rtol=1e-8)
    assert sj.converged and sm.converged
    assert sm.iters < 0.7 * sj.iters, (sm.iters, sj.iters)
    assert np.linalg.norm(R0 - A(x)) <= 1e-6 * np.linalg.norm(R0)
