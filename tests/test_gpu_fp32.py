"""FP32 element-Jacobi factored on MFMA: parity with the FP64 path and with the
oracle's blocks, and flexible GMRES keeping the FP64 tolerance."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
from oracle import integrators as I
from oracle import linear
from oracle.problem import make_ns, sample_state
from oracle.tableaux import ROW
from tests.gpu_common import rel, setup, to_gpu, to_np, vortex_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P", [2, 3, 4])
def test_fp32_mfma_inverse_matches_fp64(P):
    from paper_1904_04825_amd import F32, F64
    nx, ny = (7, 5) if P < 4 else (5, 4)
    _, op, disc = setup(nx, ny, P, "roe", seed=17)
    U = vortex_state(op)
    shift = 1.0 / (0.25 * 0.1)
    Bo = linear.ejacobi_blocks(op, U, shift)
    kappa = max(np.linalg.cond(b) for b in Bo)
    r = fi.random_vector(U.shape, seed=2)
    zo = linear.ejacobi_apply(op, Bo, r)
    Ug, rg = to_gpu(U), to_gpu(r)
    z64 = to_np(disc.ejacobi_solve(disc.ejacobi_factor(Ug, shift, F64), rg))
    z32 = to_np(disc.ejacobi_solve(disc.ejacobi_factor(Ug, shift, F32), rg))
    print(f"P={P} kappa={kappa:.1f} rel(z32,z64)={rel(z32, z64):.2e} rel(z64,oracle)={rel(z64, zo):.2e}", flush=True)
    assert rel(z64, zo) <= 1e-6
    assert rel(z32, z64) <= kappa * 6e-8 * 10


def test_fp32_ns_blocks():
    from paper_1904_04825_amd import Disc, F32, F64
    nodes = fi.perturbed_nodes(5, 4, 0, 0, 1, 1, 0.1, 3)
    op = make_ns(nodes, 3, mu=0.01)
    disc = Disc(nodes, 3, physics="ns", mu=0.01)
    U = sample_state(op, fi.ShearLayer(width=8.0, mach=0.3).conservative)
    Bo = linear.ejacobi_blocks(op, U, 40.0)
    kappa = max(np.linalg.cond(b) for b in Bo)
    r = fi.random_vector(U.shape, seed=3)
    Ug, rg = to_gpu(U), to_gpu(r)
    z64 = to_np(disc.ejacobi_solve(disc.ejacobi_factor(Ug, 40.0, F64), rg))
    z32 = to_np(disc.ejacobi_solve(disc.ejacobi_factor(Ug, 40.0, F32), rg))
    assert rel(z64, linear.ejacobi_apply(op, Bo, r)) <= 1e-6
    assert rel(z32, z64) <= kappa * 6e-8 * 10


def test_row3_step_fp32_preconditioner_keeps_tolerance():
    from paper_1904_04825_amd import F32, GmresOpts, SolverOpts
    _, op, disc = setup(12, 12, 3, "rusanov", seed=2)
    U = vortex_state(op, 0.0)
    Uo, so = I.row_step(op, ROW["ROW3"], 0.1, U, I.LinOpts(m=20, rtol=1e-8))
    Ug = to_gpu(U)
    st = disc.row_step(Ug, 3, 0.1, SolverOpts(lin=GmresOpts(m=20, rtol=1e-8), precond_precision=F32))
    print("fp32 pc", st, "oracle iters", so.gmres_iters, flush=True)
    assert st["status"] == 0 and st["unconverged"] == 0
    # both solves meet rtol 1e-8 on every stage; the states agree to that level
    assert rel(to_np(Ug), Uo) <= 1e-8
