"""Oracle (test infrastructure only): the linear-algebra layer of Section 4.5.

* jf_matvec: A v = s v - [R(q + eps v) - R(q)] / eps, the Jacobian-free product
  of the Jacobian-free GMRES subsection with A = D - dR/dq and D = s I.
* ejacobi_blocks: the element-Jacobi preconditioner, i.e. the diagonal
  (element) blocks s I - dR_e/dq_e of A, by one-sided finite differences.
* fgmres: restarted GMRES(m), right-preconditioned in its flexible form.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

JF_EPS = 1e-8           # epsilon of the Jacobian-free product (Section 4.5)
BLOCK_FD_REL = 1e-8     # relative step of the finite-difference block columns


def jf_eps(v, eps=JF_EPS, mode="rms"):
    """Perturbation size.  'abs' is the paper's literal eps; 'rms' scales it by the
    root-mean-square entry of v so that eps*v has entries of size eps, the size
    the literal rule assumes for O(1) entries."""
    if mode == "abs":
        return eps
    nv = float(np.sqrt(np.sum(np.asarray(v, dtype=np.float64) ** 2)))
    if nv == 0.0:
        return 0.0
    return eps / (nv / math.sqrt(np.size(v)))


def jf_matvec(residual, U, R0, v, shift, eps=JF_EPS, mode="rms"):
    """A v ~= shift v - [R(U + e v) - R(U)] / e   (Section 4.5)."""
    e = jf_eps(v, eps, mode)
    if e == 0.0:
        return np.zeros_like(v)
    return shift * v - (residual(U + e * v) - R0) / e


def ejacobi_blocks(op, U, shift):
    """Element blocks P_e = shift I - dR_e/dq_e (Section 4.5, element-Jacobi).

    Column j = (v, k) of block e is a one-sided difference of the element's
    residual when only entry (v, e, k) of the state moves by
    delta = BLOCK_FD_REL * max(1, |q|), with every other entry, in particular
    the neighbours' states, held fixed.  The operator supplies the element-local
    residual (own state in, neighbours frozen at U), so all elements' column j is
    formed in one vectorised evaluation.

    Returns blocks[e, row, col] with row/col index j = v * Np + k.
    """
    q = op.shape(U)
    nel = op.nel
    nv, Np = _layout(op)
    Nb = nv * Np
    local = op.local_residual_factory(U)
    R0 = local(q).reshape(nv, nel, Np)
    qf = q.reshape(nv, nel, Np)
    blocks = np.zeros((nel, Nb, Nb))
    for v in range(nv):
        for k in range(Np):
            delta = BLOCK_FD_REL * np.maximum(1.0, np.abs(qf[v, :, k]))
            qp = qf.copy()
            qp[v, :, k] += delta
            Rp = local(qp.reshape(q.shape)).reshape(nv, nel, Np)
            col = -(Rp - R0) / delta[None, :, None]          # -dR/dq_j, [v', e, k']
            blocks[:, :, v * Np + k] = col.transpose(1, 0, 2).reshape(nel, Nb)
    blocks += shift * np.eye(Nb)[None]
    return blocks


def _layout(op):
    """(variables, points per element): 2D operators (4, n^2); others state theirs."""
    return getattr(op, "nvar", 4), getattr(op, "npts", op.n * op.n)


def to_blocks(op, r):
    """[v, e, k] vector -> per-element vectors [e, v*Np + k]."""
    nv, Np = _layout(op)
    return np.asarray(r).reshape(nv, op.nel, Np).transpose(1, 0, 2).reshape(op.nel, nv * Np)


def from_blocks(op, z, shape):
    nv, Np = _layout(op)
    return z.reshape(op.nel, nv, Np).transpose(1, 0, 2).reshape(shape)


def ejacobi_apply(op, blocks, r):
    """z = P_e^{-1} r_e per element: LU with partial pivoting (LAPACK gesv)."""
    z = np.linalg.solve(blocks, to_blocks(op, r)[:, :, None])[:, :, 0]
    return from_blocks(op, z, np.shape(r))


class ElementJacobi:
    """Element-Jacobi preconditioner of an FR operator at state U with shift s."""

    def __init__(self, op, U, shift):
        self.op = op
        self.blocks = ejacobi_blocks(op, U, shift)

    def apply(self, r):
        return ejacobi_apply(self.op, self.blocks, r)


@dataclass
class GmresStats:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    r_ref: float = 0.0
    r_final: float = 0.0
    matvecs: int = 0


def fgmres(matvec, precond, b, x0=None, m=20, rtol=1e-8, ref_norm=None, max_iters=None,
           breakdown_tol=1e-14, history=None):
    """Restarted flexible GMRES(m) (Section 4.5; Saad's FGMRES form).

    Minimises ||b - A x|| over x0 + span{z_1..z_j}, z_j = M^{-1} v_j, with the
    Arnoldi basis v_j from modified Gram-Schmidt and the least-squares problem
    reduced by Givens rotations.  Stops when the least-squares residual
    |g_{j+1}| <= rtol * r_ref, where r_ref is ref_norm if given (> 0) and the
    initial residual ||b - A x0|| otherwise (Section 5.1: tolerances are relative
    to the residual at the first step).  After a full cycle without convergence
    the true residual is recomputed (one product) and GMRES restarts.
    """
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    bf = b.reshape(-1)
    x = np.zeros_like(bf) if x0 is None else np.asarray(x0, dtype=np.float64).reshape(-1).copy()
    max_iters = 50 * m if max_iters is None else max_iters
    st = GmresStats()

    def A(v):
        st.matvecs += 1
        return matvec(v.reshape(shape)).reshape(-1)

    def M(v):
        return precond(v.reshape(shape)).reshape(-1)

    r = bf - A(x) if np.any(x) else bf.copy()
    beta = float(np.linalg.norm(r))
    st.r_ref = ref_norm if (ref_norm is not None and ref_norm > 0) else beta
    target = rtol * st.r_ref
    st.r_final = beta
    if beta <= target:
        st.converged = True
        return x.reshape(shape), st
    while True:
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        j_done = 0
        conv = False
        for j in range(m):
            z = M(V[j])
            Z.append(z)
            w = A(z)
            w0 = float(np.linalg.norm(w))
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            hn = float(np.linalg.norm(w))
            H[j + 1, j] = hn
            st.iters += 1
            j_done = j + 1
            # apply the previous rotations to the new column, then a new rotation
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            st.r_final = float(abs(g[j + 1]))
            if history is not None:
                history.append(st.r_final)
            if st.r_final <= target:
                conv = True
                break
            if hn <= breakdown_tol * w0:
                # invariant Krylov space: the least-squares solution is exact
                conv = True
                break
            if st.iters >= max_iters:
                break
            V.append(w / hn)
        # x <- x + Z y with H[:j, :j] y = g[:j]
        k = j_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
        for i in range(k):
            x = x + y[i] * Z[i]
        if conv:
            st.converged = True
            return x.reshape(shape), st
        if st.iters >= max_iters:
            r = bf - A(x)
            st.r_final = float(np.linalg.norm(r))
            st.converged = st.r_final <= target
            return x.reshape(shape), st
        r = bf - A(x)
        beta = float(np.linalg.norm(r))
        st.r_final = beta
        st.restarts += 1
        if beta <= target:
            st.converged = True
            return x.reshape(shape), st
