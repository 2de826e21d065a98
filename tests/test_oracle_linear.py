"""Pins of the oracle's Jacobian-free product, element-Jacobi blocks and FGMRES
(Section 4.5) against brute force and dense linear algebra."""
import numpy as np
import pytest

import fr_inputs as fi
from oracle import linear
from oracle.problem import make_euler, sample_state


def _vortex_op(n, P, flux="rusanov", seed=None):
    nodes = fi.uniform_nodes(n, n, -5, -5, 10, 10) if seed is None else fi.perturbed_nodes(n, n, -5, -5, 10, 10, 0.1, seed)
    op = make_euler(nodes, P, flux=flux)
    v = fi.Vortex()
    return op, sample_state(op, lambda x, y: v.conservative(x, y, 0.2))


def _central_jacobian(op, U, h=1e-6):
    N = U.size
    Uf = U.reshape(-1)
    J = np.zeros((N, N))
    for j in range(N):
        e = np.zeros(N)
        e[j] = h
        J[:, j] = (op.residual((Uf + e).reshape(U.shape)) - op.residual((Uf - e).reshape(U.shape))).reshape(-1) / (2 * h)
    return J


@pytest.fixture(scope="module", params=[(2, "rusanov"), (3, "roe")])
def brute(request):
    n, flux = request.param
    op, U = _vortex_op(n, 2, flux, seed=9)
    return op, U, _central_jacobian(op, U)


def test_jf_matvec_matches_bruteforce_jacobian(brute):
    op, U, J = brute
    R0 = op.residual(U)
    rng = np.random.default_rng(3)
    shift = 7.0
    for mode, scale in (("rms", 1.0), ("rms", 1e-4), ("abs", 1.0)):
        v = scale * rng.standard_normal(U.shape)
        Av = linear.jf_matvec(op.residual, U, R0, v, shift, mode=mode)
        ref = shift * v.reshape(-1) - J @ v.reshape(-1)
        assert np.linalg.norm(Av.reshape(-1) - ref) <= 1e-6 * np.linalg.norm(ref)


def test_ejacobi_blocks_are_jacobian_diagonal_blocks(brute):
    op, U, J = brute
    shift = 3.0
    blocks = linear.ejacobi_blocks(op, U, shift)
    Np = op.n ** 2
    Nb = 4 * Np
    # DOF (v, e, k) sits at flat index (v*nel + e)*Np + k
    for e in range(op.nel):
        idx = np.array([(v * op.nel + e) * Np + k for v in range(4) for k in range(Np)])
        ref = shift * np.eye(Nb) - J[np.ix_(idx, idx)]
        assert np.linalg.norm(blocks[e] - ref) <= 1e-6 * np.linalg.norm(ref)
    # and the off-diagonal blocks of the true Jacobian are not zero (the test is not vacuous)
    idx0 = np.array([(v * op.nel + 0) * Np + k for v in range(4) for k in range(Np)])
    idx1 = np.array([(v * op.nel + 1) * Np + k for v in range(4) for k in range(Np)])
    assert np.linalg.norm(J[np.ix_(idx0, idx1)]) > 1e-3


def test_ejacobi_apply_inverts_blocks():
    op, U = _vortex_op(3, 3, seed=4)
    blocks = linear.ejacobi_blocks(op, U, 5.0)
    r = np.random.default_rng(1).standard_normal(U.shape)
    z = linear.ejacobi_apply(op, blocks, r)
    back = np.einsum("eij,ej->ei", blocks, linear.to_blocks(op, z))
    assert np.allclose(back, linear.to_blocks(op, r), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("n", [6, 25])
def test_fgmres_full_space_equals_dense_solve(n):
    rng = np.random.default_rng(n)
    A = 2 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    M = np.linalg.inv(np.diag(np.diag(A)))
    x, st = linear.fgmres(lambda v: A @ v, lambda r: M @ r, b, m=n, rtol=1e-14)
    xd = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A)
    assert st.iters <= n
    assert np.linalg.norm(x - xd) <= kappa * 1e-13 * np.linalg.norm(xd)


def test_fgmres_exact_preconditioner_breaks_down_after_one_step():
    # M^{-1} = A^{-1}: A z_0 = v_0, so the first Arnoldi step leaves w' at rounding level,
    # the Krylov space is invariant and x = A^{-1} b after one step even with rtol = 0
    rng = np.random.default_rng(8)
    n = 30
    A = 2 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    Ainv = np.linalg.inv(A)
    b = rng.standard_normal(n)
    x, st = linear.fgmres(lambda v: A @ v, lambda r: Ainv @ r, b, m=20, rtol=0.0)
    assert st.iters == 1 and st.converged and st.restarts == 0
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-13 * np.linalg.cond(A) * np.linalg.norm(b)


def test_fgmres_residual_estimate_monotone_and_true():
    rng = np.random.default_rng(5)
    n = 40
    A = 3 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    hist = []
    x, st = linear.fgmres(lambda v: A @ v, lambda r: r, b, m=n, rtol=1e-9, history=hist)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))
    assert abs(np.linalg.norm(b - A @ x) - hist[-1]) <= 1e-10 * np.linalg.norm(b)


def test_fgmres_one_step_is_minimal_residual_step():
    rng = np.random.default_rng(6)
    n = 12
    A = 3 * np.eye(n) + rng.standard_normal((n, n))
    Minv = np.diag(1.0 / np.diag(A))
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    x, st = linear.fgmres(lambda v: A @ v, lambda r: Minv @ r, b, x0=x0, m=1, rtol=1e-30, max_iters=1)
    r = b - A @ x0
    z = Minv @ r
    Az = A @ z
    alpha = np.dot(r, Az) / np.dot(Az, Az)
    assert np.allclose(x, x0 + alpha * z, rtol=1e-12, atol=1e-12)


def test_fgmres_restarts_converge_and_report():
    rng = np.random.default_rng(7)
    n = 60
    A = 4 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    x, st = linear.fgmres(lambda v: A @ v, lambda r: r, b, m=5, rtol=1e-10)
    assert st.converged and st.restarts >= 1
    assert np.linalg.norm(b - A @ x) <= 1.5e-10 * np.linalg.norm(b)
