"""GPU parity of the p-multigrid preconditioner (Section 4.5 names it beside
element-Jacobi) against the oracle's: the V-cycle itself for several level pairs and
sweep counts, FGMRES with it (solution within the derived bound, fewer iterations than
element-Jacobi), and the host checks on the levels."""
import numpy as np
import pytest

import fr_inputs as fi
from oracle import linear
from oracle.pmg import PMultigrid
from oracle.problem import make_euler
from tests.gpu_common import dense_operator, gmres_solution_bound, rel, setup, to_gpu, to_np, vortex_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("P,Pc,sweeps", [(3, 2, (1, 1, 1)), (4, 2, (2, 1, 2)), (6, 4, (1, 1, 2)), (5, 3, (1, 0, 1))])
def test_pmg_apply_parity(P, Pc, sweeps):
    from paper_1904_04825_amd import F64, Pmg
    nodes, op, disc = setup(6, 5, P, "roe", seed=9)
    opc = make_euler(nodes, Pc, flux="roe")
    U = vortex_state(op)
    R0 = op.residual(U)
    shift = 4.0
    r = fi.random_vector(U.shape, seed=3)
    zo = PMultigrid(op, opc, U, shift, *sweeps).apply(r)
    Ug = to_gpu(U)
    mg = Pmg(disc, Pc, *sweeps)
    pc = disc.pmg_factor(Ug, shift, mg, F64)
    # the coarse level's state and residual as the oracle forms them
    assert rel(to_np(mg.Uc), PMultigrid(op, opc, U, shift, *sweeps).Uc) <= 1e-14
    zg = to_np(disc.pmg_apply(pc, Ug, to_gpu(R0), shift, to_gpu(r)))
    print(f"P{P}->P{Pc} sweeps {sweeps}: rel {rel(zg, zo):.2e}", flush=True)
    assert rel(zg, zo) <= 1e-6


def test_gmres_with_pmg():
    from paper_1904_04825_amd import F64, PC_PMG, GmresOpts, Pmg
    nodes, op, disc = setup(4, 4, 3, "roe", seed=12)
    opc = make_euler(nodes, 2, flux="roe")
    U = vortex_state(op)
    R0 = op.residual(U)
    shift = 1.0 / (0.25 * 0.4)
    b = fi.random_vector(U.shape, seed=21)
    rtol = 1e-10

    def A(v):
        return linear.jf_matvec(op.residual, U, R0, v, shift)

    xo, so = linear.fgmres(A, PMultigrid(op, opc, U, shift, 1, 1, 1).apply, b, m=30, rtol=rtol)
    _, sj = linear.fgmres(A, linear.ElementJacobi(op, U, shift).apply, b, m=30, rtol=rtol)
    Ug = to_gpu(U)
    pc = disc.pmg_factor(Ug, shift, Pmg(disc, 2, 1, 1, 1), F64)
    xg, sg = disc.gmres_solve(pc, Ug, to_gpu(R0), shift, to_gpu(b), opts=GmresOpts(m=30, rtol=rtol, precond=PC_PMG))
    xg = to_np(xg)
    Ad = dense_operator(op.residual, U, shift)
    rho, bound = gmres_solution_bound(Ad, b, xo, so.r_ref, rtol)
    res_g = float(np.linalg.norm(b.reshape(-1) - Ad @ xg.reshape(-1)))
    print(f"oracle p-MG {so.iters} it., element-Jacobi {sj.iters} it.; gpu {sg}; rel {rel(xg, xo):.2e} "
          f"bound {bound:.2e}", flush=True)
    assert sg["status"] == 0 and sg["converged"] == 1
    assert abs(sg["iters"] - so.iters) <= 1
    assert so.iters < sj.iters
    assert sg["residual_evals"] >= 3 * sg["iters"]
    assert res_g <= 2 * rho and rel(xg, xo) <= bound


def test_pmg_refuses_mismatched_levels():
    from paper_1904_04825_amd import F64, PC_PMG, FrError, GmresOpts, Pmg
    _, op, disc = setup(4, 4, 3, "rusanov", seed=2)
    U = to_gpu(vortex_state(op))
    with pytest.raises(FrError):
        disc.pmg_factor(U, 3.0, Pmg(disc, 3), F64)          # coarse degree not below the fine one
    pc = disc.ejacobi_factor(U, 3.0, F64)                    # no coarse level attached
    with pytest.raises(FrError):
        disc.gmres_solve(pc, U, disc.residual(U), 3.0, U, opts=GmresOpts(precond=PC_PMG))
