"""Oracle (test infrastructure only): time integrators of Section 4 on the
semi-discrete system dq/dt = R(q) (eq. simplified_ode).

* row_step: eq. Rosenbrock_General with the Jacobian frozen at q^n; each stage
  is one Jacobian-free GMRES solve.
* esdirk_step: eq. ESDIRK2; each implicit stage solves F(q_i) = 0
  (eq. SDIRK_newton) by pseudo-transient continuation.
* bdf2_step: eq. BDF with s = 2, F from eq. BDF_newton, same nonlinear solver.
* ptc_solve: pseudo-transient continuation (eq. linearized_pseudo_transient_final)
  with SER time-step adaptation and the rejection rule of Section 4.4.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import linear


@dataclass
class LinOpts:
    m: int = 20
    rtol: float = 1e-8
    max_iters: int | None = None
    eps: float = linear.JF_EPS
    eps_mode: str = "rms"


@dataclass
class NlOpts:
    tol_nl: float = 1e-8
    dtau_init: float | None = None   # None -> dt (Section 4.4)
    dtau_max: float = 1e20
    max_ptc: int = 200
    max_reject: int = 30


@dataclass
class StepStats:
    gmres_iters: int = 0
    ptc_iters: int = 0
    rejections: int = 0
    residual_evals: int = 0
    converged: bool = True
    per_solve: list = field(default_factory=list)
    stage_increments: list = field(default_factory=list)   # ROW: the stage solutions Y_i


class Counted:
    """Residual operator wrapper that counts evaluations."""

    def __init__(self, op):
        self.op = op
        self.count = 0

    def __call__(self, U):
        self.count += 1
        return self.op.residual(U)


def preconditioner(op, U, shift):
    """The operator's own preconditioner if it has one, element-Jacobi otherwise."""
    if hasattr(op, "preconditioner"):
        return op.preconditioner(U, shift)
    return linear.ElementJacobi(op, U, shift)


def linear_solve(op, R, U, R0, shift, b, lin: LinOpts, st: StepStats, x0=None, ref_norm=None):
    """Solve (shift I - dR/dq(U)) x = b by JF FGMRES, preconditioned at U."""
    pc = preconditioner(op, U, shift)
    return linear_solve_with(op, R, U, R0, shift, pc, b, lin, st, x0, ref_norm)


def linear_solve_with(op, R, U, R0, shift, pc, b, lin, st, x0=None, ref_norm=None):
    x, gs = linear.fgmres(
        lambda v: linear.jf_matvec(R, U, R0, v, shift, lin.eps, lin.eps_mode),
        pc.apply,
        b, x0=x0, m=lin.m, rtol=lin.rtol, ref_norm=ref_norm, max_iters=lin.max_iters)
    st.gmres_iters += gs.iters
    st.per_solve.append(gs)
    return x, gs


def row_step(op, table, dt, U, lin: LinOpts = LinOpts()):
    """One step of a ROW scheme in transformed form (eq. Rosenbrock_General)."""
    R = Counted(op)
    st = StepStats()
    R0 = R(U)
    shift = 1.0 / (table.gamma * dt)
    pc = preconditioner(op, U, shift)     # Jacobian (and preconditioner) frozen at q^n
    Y = []
    for i in range(table.s):
        if i == 0 or not np.any(table.A[i, :i]):
            Ri = R0
        else:
            Ri = R(U + sum(table.A[i, j] * Y[j] for j in range(i)))
        rhs = Ri + sum(table.C[i, j] * Y[j] for j in range(i)) / dt if i > 0 else Ri.copy()
        y, gs = linear_solve_with(op, R, U, R0, shift, pc, rhs, lin, st)
        st.converged &= gs.converged
        Y.append(y)
    st.residual_evals = R.count
    st.stage_increments = Y
    return U + sum(table.m[j] * Y[j] for j in range(table.s)), st


def ptc_solve(op, R, const, omega_dt, q0, Rq0, lin: LinOpts, nl: NlOpts, dt, st: StepStats):
    """Solve F(q) = (q - const)/(omega dt) - R(q) = 0 by pseudo-transient continuation.

    Each iteration solves (I/dtau + I/(omega dt) - dR/dq)^k dq = -F(q^k)
    (eq. linearized_pseudo_transient_final) with JF FGMRES and element-Jacobi at q^k.
    dtau follows SER: dtau^{k+1} = min(dtau^k ||F^k|| / ||F^{k+1}||, dtau_max).
    If GMRES does not reduce the linear residual by a factor of ten, the
    iteration is rejected and dtau_max is halved (Section 4.4).
    Stops when ||F|| <= tol_nl * ||F(q0)||; a non-finite ||F|| ends it unconverged.
    Returns (q, R(q), converged).
    """
    q = q0.copy()
    Rq = Rq0 if Rq0 is not None else R(q)
    F = (q - const) / omega_dt - Rq
    nF = float(np.linalg.norm(F))
    nF0 = nF
    dtau = dt if nl.dtau_init is None else nl.dtau_init
    dtau_max = nl.dtau_max
    rejects = 0
    k = 0
    while not nF <= nl.tol_nl * nF0:       # a NaN norm enters the loop and fails the solve
        if not np.isfinite(nF) or k >= nl.max_ptc or rejects > nl.max_reject:
            return q, Rq, False
        shift = 1.0 / dtau + 1.0 / omega_dt
        dq, gs = linear_solve(op, R, q, Rq, shift, -F, lin, st)
        if not gs.r_final <= 0.1 * gs.r_ref:
            st.rejections += 1
            rejects += 1
            dtau_max *= 0.5
            dtau = min(dtau, dtau_max)
            continue
        q = q + dq
        Rq = R(q)
        F = (q - const) / omega_dt - Rq
        nF_new = float(np.linalg.norm(F))
        dtau = min(dtau * nF / nF_new, dtau_max) if nF_new > 0 else dtau_max
        nF = nF_new
        k += 1
        st.ptc_iters += 1
    return q, Rq, True


def esdirk_step(op, table, dt, U, lin: LinOpts = LinOpts(rtol=1e-1), nl: NlOpts = NlOpts()):
    """One ESDIRK step (eq. ESDIRK2); stage i >= 2 starts PTC from q_{i-1}."""
    R = Counted(op)
    st = StepStats()
    w = table.gamma
    Rs = [R(U)]
    q_prev, R_prev = U, Rs[0]
    for i in range(1, table.s):
        const = U + dt * sum(table.A[i, j] * Rs[j] for j in range(i))
        q, Rq, ok = ptc_solve(op, R, const, w * dt, q_prev, R_prev, lin, nl, dt, st)
        st.converged &= ok
        Rs.append(Rq)
        q_prev, R_prev = q, Rq
    st.residual_evals = R.count
    return U + dt * sum(table.b[i] * Rs[i] for i in range(table.s)), st


def bdf2_step(op, dt, U_nm1, U_n, lin: LinOpts = LinOpts(rtol=1e-1), nl: NlOpts = NlOpts()):
    """One BDF2 step (eq. BDF: omega = 2/3, a_1 = 4/3, a_2 = -1/3).  With no
    previous level (U_nm1 None) it takes a BDF1 step (omega = 1, a_1 = 1)."""
    R = Counted(op)
    st = StepStats()
    if U_nm1 is None:
        omega, const = 1.0, U_n
    else:
        omega, const = 2.0 / 3.0, (4.0 / 3.0) * U_n - (1.0 / 3.0) * U_nm1
    q, _, ok = ptc_solve(op, R, const, omega * dt, U_n, None, lin, nl, dt, st)
    st.converged = ok
    st.residual_evals = R.count
    return q, st
