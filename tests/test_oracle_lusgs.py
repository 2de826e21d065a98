"""Pins of the oracle's matrix-free LU-SGS preconditioner (Section 4.5 names it beside
element-Jacobi): the checkerboard colouring decouples the elements of one colour, the
matrix-free application equals (D + L) D^{-1} (D + U) formed from the dense Jacobian,
and FGMRES needs fewer iterations with it than with element-Jacobi."""
import numpy as np
import pytest

import fr_inputs as fi
from oracle import linear
from oracle.lusgs import LUSGS, colours, lusgs_dense
from oracle.problem import make_euler, sample_state


def _case(nx, ny, P, flux="roe", seed=3):
    nodes = fi.perturbed_nodes(nx, ny, -5, -5, 10, 10, 0.1, seed)
    op = make_euler(nodes, P, flux=flux)
    v = fi.Vortex()
    return op, sample_state(op, lambda x, y: v.conservative(x, y, 0.3))


def _dense(op, U, shift, h=1e-6):
    u = U.reshape(-1)
    n = u.size
    A = np.empty((n, n))
    for j in range(n):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        A[:, j] = -(op.residual(up.reshape(U.shape)) - op.residual(um.reshape(U.shape))).reshape(-1) / (2 * h)
        A[j, j] += shift
    return A


def test_colours_decouple_elements():
    op, U = _case(4, 4, 2)
    A = _dense(op, U, 3.0)
    Np = 9
    el = (np.arange(A.shape[0]) // Np) % op.nel
    c = colours(op.mesh)
    same = (c[el][:, None] == c[el][None, :]) & (el[:, None] != el[None, :])
    assert np.count_nonzero(A[same]) == 0
    assert np.count_nonzero(A[~same & (el[:, None] != el[None, :])]) > 0   # neighbours do couple


@pytest.mark.parametrize("P", [2, 3])
def test_matrix_free_apply_equals_dense_preconditioner(P):
    op, U = _case(4, 4, P)
    shift = 5.0
    pc = LUSGS(op, U, shift)
    A = _dense(op, U, shift)
    Minv = lusgs_dense(A, pc.blocks, colours(op.mesh) == 0, 4 * (P + 1) ** 2)
    r = fi.random_vector(U.shape, seed=4)
    z = pc.apply(r)
    zd = Minv(r)
    assert np.linalg.norm(z - zd) <= 1e-6 * np.linalg.norm(zd)
    # and it is not element-Jacobi
    zj = linear.ejacobi_apply(op, pc.blocks, r)
    assert np.linalg.norm(zj - zd) > 1e-3 * np.linalg.norm(zd)


def test_lusgs_rejects_odd_meshes():
    op, U = _case(5, 4, 2)
    with pytest.raises(ValueError):
        LUSGS(op, U, 1.0)


def test_fgmres_needs_fewer_iterations_with_lusgs():
    op, U = _case(8, 8, 3, flux="rusanov")
    R0 = op.residual(U)
    shift = 1.0 / (0.25 * 0.4)
    b = R0.copy()

    def A(v):
        return linear.jf_matvec(op.residual, U, R0, v, shift)

    _, sj = linear.fgmres(A, linear.ElementJacobi(op, U, shift).apply, b, m=30, rtol=1e-8)
    x, sl = linear.fgmres(A, LUSGS(op, U, shift).apply, b, m=30, rtol=1e-8)
    assert sj.converged and sl.converged
    assert sl.iters < 0.8 * sj.iters, (sl.iters, sj.iters)
    assert np.linalg.norm(b - A(x)) <= 1e-6 * np.linalg.norm(b)
