"""GPU parity of the implicit steps on the 3D hexahedral path (fr3d_ejacobi_*,
fr3d_gmres_solve, fr3d_row_step, fr3d_esdirk_step, fr3d_bdf2_step) against the FP64
oracle: element-Jacobi blocks of 5 (P+1)^3 rows (Section 4.5) assembled by coloured
differences on the GPU and element by element with frozen neighbours in the oracle, their
Gauss-Jordan inverses, FGMRES, and ROW / ESDIRK / BDF2 steps (Sections 4.1-4.4) on the
BR2 Navier-Stokes residual."""
import math

import numpy as np
import pytest

from oracle import integrators as I
from oracle import linear
from oracle.fr3d import Box3D, NavierStokes3D
from oracle.tableaux import ESDIRK, ROW
from tests.gpu_common import rel, to_gpu, to_np
from tests.test_oracle_fr3d import _state3d

pytestmark = pytest.mark.gpu


def _pair(nx, ny, nz, P, mu=0.05):
    from paper_1904_04825_amd import Disc3D
    box = Box3D(nx, ny, nz, [0.0] * 3, [2 * math.pi] * 3, P)
    op = NavierStokes3D(box, mu=mu)
    disc = Disc3D(nx, ny, nz, P, (0.0,) * 3, (2 * math.pi,) * 3, flux="roe", mu=mu)
    x, y, z = box.points()
    U = _state3d(x, y, z).reshape(5, box.nel, -1)
    return box, op, disc, U


@pytest.mark.parametrize("dims,P", [((3, 2, 2), 2), ((2, 2, 2), 3), ((2, 3, 4), 2)])
def test_blocks_parity(dims, P):
    """Odd sizes need three colours (3 mod 2 = 1), even ones two."""
    box, op, disc, U = _pair(*dims, P)
    Bo = linear.ejacobi_blocks(op, U, 4.0)
    Bg = disc.ejacobi_assemble(to_gpu(U), 4.0).cpu().numpy()
    worst = max(np.linalg.norm(Bg[e] - Bo[e]) / np.linalg.norm(Bo[e]) for e in range(box.nel))
    print(f"{dims} P{P}: worst block rel diff {worst:.2e}", flush=True)
    assert worst <= 1e-6


@pytest.mark.parametrize("shift", [0.5, 50.0])
def test_inverse_and_apply(shift):
    """The Gauss-Jordan inverses against the GPU's own blocks (pivoting happens at the small
    shift, where the blocks are far from diagonally dominant): inv B = I and z = B^{-1} r
    to rounding times the condition number."""
    box, op, disc, U = _pair(2, 2, 2, 3)
    Ug = to_gpu(U)
    B = disc.ejacobi_assemble(Ug, shift).cpu().numpy()
    inv = disc.ejacobi_factor(Ug, shift)
    Inv = inv.cpu().numpy().transpose(0, 2, 1)          # stored column-major
    r = np.random.default_rng(1).standard_normal(U.shape)
    z = to_np(disc.ejacobi_apply(inv, to_gpu(r)))
    zb = linear.to_blocks(op, z)
    rb = linear.to_blocks(op, r)
    for e in range(box.nel):
        kappa = np.linalg.cond(B[e])
        assert np.abs(Inv[e] @ B[e] - np.eye(B.shape[1])).max() <= 1e-13 * kappa, e
        ze = np.linalg.solve(B[e], rb[e])
        assert np.linalg.norm(zb[e] - ze) <= 1e-13 * kappa * np.linalg.norm(ze), e
    print(f"shift {shift}: condition numbers up to {max(np.linalg.cond(B[e]) for e in range(box.nel)):.1e}")


@pytest.mark.parametrize("m", [8, 30])
def test_gmres_parity(m):
    """FGMRES(m) to 1e-10 on both sides (m = 8 restarts): the same solution up to the
    Jacobian-free products' finite-difference noise."""
    from paper_1904_04825_amd import GmresOpts
    box, op, disc, U = _pair(3, 2, 2, 2)
    R0 = op.residual(U)
    b = np.random.default_rng(3).standard_normal(U.shape)
    shift = 5.0
    pc = linear.ElementJacobi(op, U, shift)
    xo, so = linear.fgmres(lambda v: linear.jf_matvec(op.residual, U, R0, v, shift), pc.apply, b, m=m, rtol=1e-10)
    Ug = to_gpu(U)
    inv = disc.ejacobi_factor(Ug, shift)
    xg, sg = disc.gmres_solve(inv, Ug, to_gpu(R0), shift, to_gpu(b), opts=GmresOpts(m=m, rtol=1e-10))
    print(f"m={m}: gpu {sg['iters']} iterations ({sg['restarts']} restarts), oracle {so.iters}", flush=True)
    assert sg["status"] == 0 and so.converged
    assert abs(sg["iters"] - so.iters) <= 2
    assert rel(to_np(xg), xo) <= 1e-7


@pytest.mark.parametrize("scheme", ["ROW2", "ROW3", "ROW4"])
def test_row_step_parity(scheme):
    from paper_1904_04825_amd import GmresOpts, SolverOpts
    box, op, disc, U = _pair(2, 2, 2, 2)
    dt = 0.05
    Uo, so = I.row_step(op, ROW[scheme], dt, U, I.LinOpts(m=20, rtol=1e-10))
    Ug = to_gpu(U)
    st = disc.row_step(Ug, int(scheme[3]), dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-10)))
    print(scheme, "gpu", st, "oracle gmres", so.gmres_iters, flush=True)
    assert st["status"] == 0 and so.converged
    assert rel(to_np(Ug), Uo) <= 1e-8


def test_esdirk3_and_bdf2_parity():
    """Stage solves to 1e-10 on both sides (the paper's linear 1e-1 inside PTC), so the
    states agree whatever the pseudo-time paths."""
    from paper_1904_04825_amd import GmresOpts, SolverOpts
    box, op, disc, U = _pair(2, 2, 2, 2)
    dt = 0.1
    lin, nl = I.LinOpts(m=20, rtol=1e-1), I.NlOpts(tol_nl=1e-10)
    opts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-10)
    Uo, so = I.esdirk_step(op, ESDIRK["ESDIRK3"], dt, U, lin, nl)
    Ug = to_gpu(U)
    st = disc.esdirk_step(Ug, 3, dt, opts)
    print("ESDIRK3 gpu", st, "oracle ptc", so.ptc_iters, flush=True)
    assert st["status"] == 0 and so.converged
    assert rel(to_np(Ug), Uo) <= 1e-8
    U1o, _ = I.bdf2_step(op, dt, None, U, lin, nl)
    U2o, _ = I.bdf2_step(op, dt, U, U1o, lin, nl)
    U0g = to_gpu(U)
    U1g, s1 = disc.bdf2_step(None, U0g, dt, opts)
    U2g, s2 = disc.bdf2_step(U0g, U1g, dt, opts)
    assert s1["status"] == 0 and s2["status"] == 0
    assert rel(to_np(U2g), U2o) <= 1e-8


def test_nan_state_and_invalid_calls():
    from paper_1904_04825_amd import Disc3D, FrError, GmresOpts, SolverOpts
    box, op, disc, U = _pair(2, 2, 2, 2)
    Un = U.copy()
    Un[1, 3, 5] = np.nan
    st = disc.esdirk_step(to_gpu(Un), 3, 0.1, SolverOpts(lin=GmresOpts(m=10, rtol=1e-1), tol_nl=1e-6))
    assert st["status"] == 3                        # FR_ENAN
    with pytest.raises(FrError):
        disc.row_step(to_gpu(U), 3, 0.1, SolverOpts(lin=GmresOpts(m=10), precond_precision=7))
    with pytest.raises(ValueError):
        disc.step_workspace(65)
    d4 = Disc3D(2, 2, 2, 4, (0.0,) * 3, (1.0,) * 3, mu=0.01)
    with pytest.raises(FrError):
        d4.row_step(d4.empty().fill_(1.0), 3, 0.1, SolverOpts(lin=GmresOpts(m=4)))


def test_tgv16_p3_blocks_and_inverses_sampled():
    """At the size the Taylor-Green implicit study runs (16^3 P3, 4,096 blocks of 320 rows,
    shift 1/(gamma dt) of ROW4 at dt = t_c/25): three block columns of every element against
    the oracle's frozen-neighbour differences, and inverse x block = I on sampled elements.
    At Ma = 0.1 the pressure (about 71) dwarfs the residual, so a difference quotient with
    step 1e-8 |q| carries rounding near 1e-6 of the column; the columns are held to 1e-6 or
    to 3x the oracle's own spread under a one-ulp change of the state, whichever is larger."""
    import fr_inputs as fi
    import torch
    from paper_1904_04825_amd import Disc3D
    tg = fi.TaylorGreen()
    L = tg.L
    box = Box3D(16, 16, 16, [-math.pi * L] * 3, [2 * math.pi * L] * 3, 3)
    op = NavierStokes3D(box, mu=tg.mu, prandtl=tg.prandtl, gamma=tg.gamma, rgas=tg.rgas)
    disc = Disc3D(16, 16, 16, 3, (-math.pi * L,) * 3, (2 * math.pi * L,) * 3, flux="roe", mu=tg.mu,
                  prandtl=tg.prandtl, gamma=tg.gamma, rgas=tg.rgas)
    x, y, z = box.points()
    U = tg.conservative(x, y, z).reshape(5, box.nel, -1)
    shift = 1.0 / (0.25 * 0.04 * L / tg.V0)
    Ug = to_gpu(U)
    B = disc.ejacobi_assemble(Ug, shift)                 # [e, row, col] view
    rng = np.random.default_rng(6)
    U2 = np.nextafter(U, rng.choice([-np.inf, np.inf], size=U.shape))

    def column(Us, j):
        local = op.local_residual_factory(Us)
        v, k = divmod(j, 64)
        qp = Us.copy()
        delta = 1e-8 * np.maximum(1.0, np.abs(qp[v, :, k]))
        qp[v, :, k] += delta
        col = -(local(qp).reshape(5, box.nel, 64) - local(Us).reshape(5, box.nel, 64)) / delta[None, :, None]
        col = col.transpose(1, 0, 2).reshape(box.nel, 320)
        col[:, j] += shift
        return col

    def rel_rows(a, b):
        return float(np.max(np.linalg.norm(a - b, axis=1) / np.linalg.norm(b, axis=1)))
    for j in (0, 137, 319):
        col = column(U, j)
        err = rel_rows(B[:, :, j].cpu().numpy(), col)
        spread = rel_rows(column(U2, j), col)
        print(f"16^3 P3 block column {j}: gpu vs oracle {err:.2e}, oracle spread under one ulp {spread:.2e}",
              flush=True)
        assert err <= max(1e-6, 3 * spread)
    Bs = {e: B[e].cpu().numpy() for e in (0, 1234, 4095)}
    del B
    torch.cuda.empty_cache()
    inv = disc.ejacobi_factor(Ug, shift)
    for e, Be in Bs.items():
        Ie = inv[e].cpu().numpy().T
        assert np.abs(Ie @ Be - np.eye(320)).max() <= 1e-13 * np.linalg.cond(Be), e


def test_runs_of_several_steps():
    """Run-level parity: four ROW3 steps and three BDF2 steps (BDF1 start) on 3 x 2 x 2 P2
    against the oracle, the stage solves to 1e-10 (ROW) and 1e-10 nonlinear (BDF2)."""
    from paper_1904_04825_amd import GmresOpts, SolverOpts
    box, op, disc, U = _pair(3, 2, 2, 2)
    dt = 0.05
    Uo = U.copy()
    Ug = to_gpu(U)
    for _ in range(4):
        Uo, so = I.row_step(op, ROW["ROW3"], dt, Uo, I.LinOpts(m=20, rtol=1e-10))
        st = disc.row_step(Ug, 3, dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-10)))
        assert st["status"] == 0 and so.converged
    err = rel(to_np(Ug), Uo)
    print(f"4 ROW3 steps: {err:.2e}", flush=True)
    assert err <= 1e-8
    lin, nl = I.LinOpts(m=20, rtol=1e-1), I.NlOpts(tol_nl=1e-10)
    opts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-10)
    prev_o, cur_o = None, U.copy()
    prev_g, cur_g = None, to_gpu(U)
    for _ in range(3):
        nxt_o, so = I.bdf2_step(op, dt, prev_o, cur_o, lin, nl)
        nxt_g, sg = disc.bdf2_step(prev_g, cur_g, dt, opts)
        assert sg["status"] == 0 and so.converged
        prev_o, cur_o = cur_o, nxt_o
        prev_g, cur_g = cur_g, nxt_g
    err = rel(to_np(cur_g), cur_o)
    print(f"3 BDF2 steps: {err:.2e}", flush=True)
    assert err <= 1e-8


def test_fp32_preconditioner_steps():
    """The FP32 element-Jacobi (blocks rounded to FP32, inverted and applied in FP32) only
    preconditions: ROW3 and ESDIRK3 steps with stage solves to 1e-10 end where the FP64
    oracle's do, P2 and P3."""
    from paper_1904_04825_amd import F32, GmresOpts, SolverOpts
    for P in (2, 3):
        box, op, disc, U = _pair(2, 2, 2, P)
        dt = 0.05
        Uo, so = I.row_step(op, ROW["ROW3"], dt, U, I.LinOpts(m=20, rtol=1e-10))
        Ug = to_gpu(U)
        st = disc.row_step(Ug, 3, dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-10), precond_precision=F32))
        print(f"P{P} ROW3 FP32 pc: gpu {st['gmres_iters']} GMRES iterations, oracle (FP64 pc) {so.gmres_iters}",
              flush=True)
        assert st["status"] == 0 and so.converged
        assert rel(to_np(Ug), Uo) <= 1e-8
    box, op, disc, U = _pair(2, 2, 2, 2)
    Uo, so = I.esdirk_step(op, ESDIRK["ESDIRK3"], 0.1, U, I.LinOpts(m=20, rtol=1e-1), I.NlOpts(tol_nl=1e-10))
    Ug = to_gpu(U)
    st = disc.esdirk_step(Ug, 3, 0.1, SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-10, precond_precision=F32))
    assert st["status"] == 0 and so.converged
    assert rel(to_np(Ug), Uo) <= 1e-8
