"""GPU parity at the paper's high degrees, P5 (N_b = 144) and P6 (N_b = 196, the
degree of the paper's vortex study), through the C ABI against the FP64 oracle:
residual (small tiles with ragged tails, and the large-tile launch at P6), JF product,
element-Jacobi blocks, their inversion (FP64 and FP32, with forced pivoting) and
application, GMRES(60) and a ROW4 step."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
from oracle import integrators as I
from oracle import linear
from oracle.tableaux import ROW
from tests.gpu_common import (check_residual, dense_operator, gmres_solution_bound, rel, setup, to_gpu, to_np,
                              vortex_state)

pytestmark = pytest.mark.gpu

# small tiles 3x2 (P5) and 2x2 (P6): ragged in both directions
MESHES = {5: (8, 5), 6: (7, 5)}


@pytest.mark.parametrize("P", [5, 6])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_residual_and_matvec_parity(P, flux):
    _, op, disc = setup(*MESHES[P], P, flux, seed=3)
    U = vortex_state(op)
    Ro = op.residual(U)
    Ug = to_gpu(U)
    Rg = to_np(disc.residual(Ug))
    check_residual(Rg, Ro, op, U, f"P{P} {flux}")
    from paper_1904_04825_amd import EPS_ABS, EPS_RMS
    for mode, scale in (("rms", 1e-3), ("abs", 1.0)):
        v = fi.random_vector(U.shape, seed=5 + P, scale=scale)
        Ao = linear.jf_matvec(op.residual, U, Ro, v, 4.0, mode=mode)
        Ag = to_np(disc.jf_matvec(Ug, to_gpu(Ro), to_gpu(v), 4.0, 1e-8, EPS_RMS if mode == "rms" else EPS_ABS))
        print(f"  JF product ({mode}) rel err {rel(Ag, Ao):.2e}", flush=True)
        assert rel(Ag, Ao) <= 1e-6


def test_residual_large_tiles_p6():
    # 226x183 at P6: 46 x 46 = 2116 large (5x4) tiles, ragged in both directions
    _, op, disc = setup(226, 183, 6, "roe", seed=4)
    U = vortex_state(op)
    print("226x183 P6: oracle residual", flush=True)
    Ro = op.residual(U)
    Rg = to_np(disc.residual(to_gpu(U)))
    check_residual(Rg, Ro, op, U, "226x183 P6")


@pytest.mark.parametrize("P", [5, 6])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_ejacobi_assemble_parity(P, flux):
    _, op, disc = setup(4, 3, P, flux, seed=6)
    U = vortex_state(op)
    Bo = linear.ejacobi_blocks(op, U, 3.0)
    Bg = to_np(disc.ejacobi_assemble(to_gpu(U), 3.0))
    for e in range(op.nel):
        assert np.linalg.norm(Bg[e] - Bo[e]) <= 1e-6 * np.linalg.norm(Bo[e])


@pytest.mark.parametrize("P", [5, 6])
def test_ejacobi_inverse_and_solve_parity(P):
    from paper_1904_04825_amd import F32, F64
    _, op, disc = setup(4, 3, P, "roe", seed=7)
    U = vortex_state(op)
    Bo = linear.ejacobi_blocks(op, U, 2.0)
    r = fi.random_vector(U.shape, seed=11)
    zo = linear.ejacobi_apply(op, Bo, r)
    kappa = max(np.linalg.cond(b) for b in Bo)
    zg = to_np(disc.ejacobi_solve(disc.ejacobi_factor_blocks(torch.as_tensor(Bo), F64), to_gpu(r)))
    z32 = to_np(disc.ejacobi_solve(disc.ejacobi_factor_blocks(torch.as_tensor(Bo), F32), to_gpu(r)))
    print(f"P{P}: kappa {kappa:.1f}, FP64 rel {rel(zg, zo):.2e}, FP32 rel {rel(z32, zo):.2e}", flush=True)
    assert rel(zg, zo) <= 1e-14 * kappa * 10
    assert rel(z32, zo) <= kappa * 6e-8 * 10
    # assembled and inverted on the GPU in one call
    for prec, tol in ((F64, 1e-6), (F32, 1e-5)):
        zf = to_np(disc.ejacobi_solve(disc.ejacobi_factor(to_gpu(U), 2.0, prec), to_gpu(r)))
        assert rel(zf, zo) <= tol


@pytest.mark.parametrize("P", [5, 6])
def test_block_inverse_needs_pivoting(P):
    """Blocks with a zero diagonal and one dominant entry per row on a random permutation:
    the inversion has to pivot in nearly every step (FP64 and FP32)."""
    from paper_1904_04825_amd import F32, F64
    _, op, disc = setup(3, 2, P, "rusanov", seed=5)
    nb = 4 * (P + 1) ** 2
    rng = np.random.default_rng(31 + P)
    B = rng.standard_normal((op.nel, nb, nb))
    for e in range(op.nel):
        B[e, np.arange(nb), np.arange(nb)] = 0.0
        B[e, np.arange(nb), rng.permutation(nb)] += 4.0 * np.sqrt(nb)
    r = fi.random_vector((4, op.nel, (P + 1) ** 2), seed=12)
    zo = linear.ejacobi_apply(op, B, r)
    kappa = max(np.linalg.cond(b) for b in B)
    zg = to_np(disc.ejacobi_solve(disc.ejacobi_factor_blocks(torch.as_tensor(B), F64), to_gpu(r)))
    z32 = to_np(disc.ejacobi_solve(disc.ejacobi_factor_blocks(torch.as_tensor(B), F32), to_gpu(r)))
    print(f"P{P}: kappa {kappa:.1f}, FP64 rel {rel(zg, zo):.2e}, FP32 rel {rel(z32, zo):.2e}", flush=True)
    assert rel(zg, zo) <= 1e-14 * kappa * 10
    assert rel(z32, zo) <= kappa * 6e-8 * 10


def test_gmres60_parity_p6():
    """The paper's restart length at the paper's degree: GMRES(60), Roe flux."""
    from paper_1904_04825_amd import F64, GmresOpts
    _, op, disc = setup(3, 3, 6, "roe", seed=12, lo=-10.0, L=20.0)
    U = vortex_state(op)
    R0 = op.residual(U)
    shift = 1.0 / (0.25 * 0.2)
    b = fi.random_vector(U.shape, seed=21)
    rtol = 1e-10
    pc_o = linear.ElementJacobi(op, U, shift)
    xo, so = linear.fgmres(lambda v: linear.jf_matvec(op.residual, U, R0, v, shift), pc_o.apply, b, m=60, rtol=rtol)
    Ug = to_gpu(U)
    pc = disc.ejacobi_factor(Ug, shift, F64)
    xg, sg = disc.gmres_solve(pc, Ug, to_gpu(R0), shift, to_gpu(b), opts=GmresOpts(m=60, rtol=rtol))
    xg = to_np(xg)
    A = dense_operator(op.residual, U, shift)
    rho, bound = gmres_solution_bound(A, b, xo, so.r_ref, rtol)
    res_g = float(np.linalg.norm(b.reshape(-1) - A @ xg.reshape(-1)))
    print("oracle", so, "gpu", sg, f"rel {rel(xg, xo):.2e} bound {bound:.2e}", flush=True)
    assert sg["status"] == 0 and abs(sg["iters"] - so.iters) <= 1
    assert res_g <= 2 * rho and rel(xg, xo) <= bound


@pytest.mark.parametrize("P", [5, 6])
def test_row4_step_parity(P):
    from paper_1904_04825_amd import GmresOpts, SolverOpts
    _, op, disc = setup(*MESHES[P], P, "roe", seed=2)
    U = vortex_state(op, 0.0)
    Ug = to_gpu(U)
    st = disc.row_step(Ug, 4, 0.1, SolverOpts(lin=GmresOpts(m=60, rtol=1e-10)))
    Uo, so = I.row_step(op, ROW["ROW4"], 0.1, U, I.LinOpts(m=60, rtol=1e-10))
    print(f"P{P} ROW4: gpu {st['gmres_iters']} oracle {so.gmres_iters} GMRES iterations, "
          f"rel {rel(to_np(Ug), Uo):.2e}", flush=True)
    assert st["status"] == 0
    assert rel(to_np(Ug), Uo) <= 1e-8
