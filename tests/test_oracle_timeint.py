"""Pins of the oracle's time integrators (Section 4): order conditions of the
coefficient tables, stability functions, and empirical order on ODEs with known
exact solutions; PTC against Newton's method."""
import math

import numpy as np
import pytest

import fr_inputs as fi
from oracle import integrators as I
from oracle import linear
from oracle.problem import make_euler, sample_state
from oracle.tableaux import ESDIRK, ROW


def _row_conditions(alpha, gam, b):
    """The Rosenbrock order conditions up to order 4 (Hairer & Wanner II, Table IV.7.1),
    beta = alpha + Gamma, beta'_i = sum_{j<i} beta_ij, alpha_i = sum_j alpha_ij."""
    g = gam[0, 0]
    beta = alpha + gam
    bs = np.tril(beta, -1)
    ai = alpha.sum(1)
    bp = bs.sum(1)
    return [
        (1, b.sum() - 1.0),
        (2, b @ bp - (0.5 - g)),
        (3, b @ ai ** 2 - 1.0 / 3.0),
        (3, b @ (bs @ bp) - (1.0 / 6.0 - g + g * g)),
        (4, b @ ai ** 3 - 0.25),
        (4, b @ (ai * (alpha @ bp)) - (1.0 / 8.0 - g / 3.0)),
        (4, b @ (bs @ ai ** 2) - (1.0 / 12.0 - g / 3.0)),
        (4, b @ (bs @ (bs @ bp)) - (1.0 / 24.0 - g / 2.0 + 1.5 * g * g - g ** 3)),
    ]


@pytest.mark.parametrize("name,order", [("ROW2", 2), ("ROW3", 3), ("ROW4", 4)])
def test_row_order_conditions(name, order):
    t = ROW[name]
    alpha, gam, b = t.standard()
    assert np.allclose(np.diag(gam), t.gamma, atol=1e-14)
    for p, res in _row_conditions(alpha, gam, b):
        if p <= order:
            assert abs(res) < 1e-13, (name, p, res)
    # stiffly accurate: b_i = beta_si
    assert np.allclose(b, (alpha + gam)[-1], atol=1e-13)


def _stability(B, b, z):
    s = len(b)
    return 1.0 + z * (b @ np.linalg.solve(np.eye(s) - z * B, np.ones(s)))


@pytest.mark.parametrize("name", ["ROW2", "ROW3", "ROW4", "ESDIRK2", "ESDIRK3", "ESDIRK4"])
def test_a_and_l_stability(name):
    if name in ROW:
        alpha, gam, b = ROW[name].standard()
        B = alpha + gam
    else:
        B, b = ESDIRK[name].A, ESDIRK[name].b
    for y in np.logspace(-3, 4, 300):
        assert abs(_stability(B, b, 1j * y)) <= 1.0 + 1e-12
    assert abs(_stability(B, b, -1e9)) < 1e-6


def _rk_conditions(A, b):
    c = A.sum(1)
    return [(1, b.sum() - 1), (2, b @ c - 0.5), (3, b @ c ** 2 - 1 / 3), (3, b @ A @ c - 1 / 6),
            (4, b @ c ** 3 - 0.25), (4, b @ (c * (A @ c)) - 1 / 8), (4, b @ A @ c ** 2 - 1 / 12),
            (4, b @ A @ A @ c - 1 / 24)]


@pytest.mark.parametrize("name,order", [("ESDIRK2", 2), ("ESDIRK3", 3), ("ESDIRK4", 4)])
def test_esdirk_tables(name, order):
    t = ESDIRK[name]
    for p, res in _rk_conditions(t.A, t.b):
        if p <= order:
            assert abs(res) < 1e-13, (name, p, res)
    assert np.all(t.A[0] == 0.0)                               # explicit first stage
    assert np.allclose(np.diag(t.A)[1:], t.gamma, atol=0)      # a_ii = omega, i >= 2
    assert np.allclose(t.b, t.A[-1])                           # stiffly accurate


def test_esdirk3_gamma_is_the_l_stable_root():
    g = ESDIRK["ESDIRK3"].gamma
    assert abs(6 * g ** 3 - 18 * g ** 2 + 9 * g - 1) < 1e-11


def test_row_transformed_roundtrip():
    for t in ROW.values():
        alpha, gam, b = t.standard()
        t2 = type(t).from_standard("x", alpha, gam, b)
        assert np.allclose(t2.A, t.A, atol=1e-12) and np.allclose(t2.C, t.C, atol=1e-11)
        assert np.allclose(t2.m, t.m, atol=1e-12)


class DenseODE:
    """y' = f(y) for a small system; the 'preconditioner' is the exact inverse of
    shift I - df/dy (by central differences), so GMRES converges at once."""

    def __init__(self, f):
        self.f = f

    def residual(self, U):
        return self.f(U)

    def preconditioner(self, U, shift):
        n = U.size
        J = np.zeros((n, n))
        for j in range(n):
            e = np.zeros(n)
            e[j] = 1e-6
            J[:, j] = (self.f(U + e.reshape(U.shape)) - self.f(U - e.reshape(U.shape))).reshape(-1) / 2e-6
        Minv = np.linalg.inv(shift * np.eye(n) - J)

        class _P:
            def apply(self_, r):
                return (Minv @ r.reshape(-1)).reshape(r.shape)
        return _P()


LAM = np.array([[-2.0, 1.0], [0.5, -30.0]])


def _riccati(U):
    return -U * U


def _linear(U):
    return LAM @ U


def _solve_ode(kind, scheme, dt, T):
    if kind == "riccati":
        op, U, exact = DenseODE(_riccati), np.array([1.0, 0.5]), lambda t: np.array([1 / (1 + t), 0.5 / (1 + 0.5 * t)])
    else:
        w, V = np.linalg.eig(LAM)
        y0 = np.array([1.0, 1.0])
        cst = np.linalg.solve(V, y0)
        op, U, exact = DenseODE(_linear), y0, lambda t: (V @ (cst * np.exp(w * t))).real
    nsteps = int(round(T / dt))
    lin = I.LinOpts(m=4, rtol=1e-14)
    nl = I.NlOpts(tol_nl=1e-13)
    prev = None
    for n in range(nsteps):
        if scheme in ROW:
            U, _ = I.row_step(op, ROW[scheme], dt, U, lin)
        elif scheme in ESDIRK:
            U, _ = I.esdirk_step(op, ESDIRK[scheme], dt, U, lin, nl)
        else:
            Un = U
            U, _ = I.bdf2_step(op, dt, prev, U, lin, nl)
            prev = Un
    return np.abs(U - exact(T)).max()


@pytest.mark.parametrize("scheme,order", [("ROW2", 2), ("ROW3", 3), ("ROW4", 4), ("ESDIRK2", 2),
                                          ("ESDIRK3", 3), ("ESDIRK4", 4), ("BDF2", 2)])
@pytest.mark.parametrize("kind", ["riccati", "linear"])
def test_empirical_order(scheme, order, kind):
    dts = [0.2, 0.1, 0.05]
    errs = [_solve_ode(kind, scheme, dt, 2.0) for dt in dts]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(dts) - 1)]
    assert rates[-1] > order - 0.35, (errs, rates)


def test_bdf2_matches_linear_recurrence():
    # y' = lam y: (1 - (2/3) z) y_{n+1} = (4/3) y_n - (1/3) y_{n-1}, z = lam dt, after a BDF1 start
    lam, dt = -3.0, 0.1
    op = DenseODE(lambda U: lam * U)
    lin, nl = I.LinOpts(m=2, rtol=1e-15), I.NlOpts(tol_nl=1e-14)
    y = [np.array([1.0])]
    y1, _ = I.bdf2_step(op, dt, None, y[0], lin, nl)
    y.append(y1)
    ref = [1.0, 1.0 / (1 - lam * dt)]
    for n in range(10):
        yn, _ = I.bdf2_step(op, dt, y[-2], y[-1], lin, nl)
        y.append(yn)
        ref.append((4 / 3 * ref[-1] - 1 / 3 * ref[-2]) / (1 - 2 / 3 * lam * dt))
    assert np.allclose(np.array(y)[:, 0], ref, rtol=1e-12)


def test_ptc_stage_equals_newton_solution():
    nodes = fi.perturbed_nodes(2, 2, -5, -5, 10, 10, 0.1, seed=2)
    op = make_euler(nodes, 2)
    v = fi.Vortex()
    U = sample_state(op, lambda x, y: v.conservative(x, y))
    dt, omega = 0.2, 2.0 / 3.0
    const = U.copy()
    R = I.Counted(op)
    st = I.StepStats()
    q, _, ok = I.ptc_solve(op, R, const, omega * dt, U, None, I.LinOpts(m=30, rtol=1e-12),
                           I.NlOpts(tol_nl=1e-12), dt, st)
    assert ok
    # Newton with the dense central-difference Jacobian
    N = U.size

    def F(x):
        return (x - const) / (omega * dt) - op.residual(x)
    x = U.copy()
    for _ in range(12):
        J = np.zeros((N, N))
        for j in range(N):
            e = np.zeros(N)
            e[j] = 1e-6
            J[:, j] = (F(x + e.reshape(x.shape)) - F(x - e.reshape(x.shape))).reshape(-1) / 2e-6
        x = x - np.linalg.solve(J, F(x).reshape(-1)).reshape(x.shape)
    assert np.linalg.norm(q - x) <= 1e-9 * np.linalg.norm(x)


def test_ptc_rejection_halves_dtau_max():
    # a single GMRES iteration cannot reduce the residual tenfold here: every attempt is
    # rejected and dtau_max halves until the rejection cap returns "not converged"
    nodes = fi.uniform_nodes(3, 3, -5, -5, 10, 10)
    op = make_euler(nodes, 2)
    v = fi.Vortex()
    U = sample_state(op, lambda x, y: v.conservative(x, y))
    st = I.StepStats()
    q, _, ok = I.ptc_solve(op, I.Counted(op), U + 0.01, 0.5, U, None, I.LinOpts(m=1, rtol=1e-3, max_iters=1),
                           I.NlOpts(tol_nl=1e-8, max_reject=5, dtau_init=1e3), 1.0, st)
    assert not ok and st.rejections == 6 and np.array_equal(q, U)


def test_ptc_nan_state_is_not_converged():
    # a NaN anywhere in the state makes ||F|| NaN, which compares false with the tolerance:
    # the solve must end unconverged instead of taking the comparison as convergence
    nodes = fi.uniform_nodes(2, 2, -5, -5, 10, 10)
    op = make_euler(nodes, 2)
    v = fi.Vortex()
    U = sample_state(op, lambda x, y: v.conservative(x, y))
    U[0, 1, 2] = np.nan
    st = I.StepStats()
    _, _, ok = I.ptc_solve(op, I.Counted(op), U, 0.5, U, None, I.LinOpts(m=5, rtol=1e-1), I.NlOpts(tol_nl=1e-6),
                           1.0, st)
    assert not ok and st.ptc_iters == 0
    _, so = I.esdirk_step(op, ESDIRK["ESDIRK3"], 0.5, U)
    assert not so.converged
