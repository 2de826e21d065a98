"""Temporal order of every GPU integrator on the vortex (Sections 4.2-4.4): the stage
solves converged far below the temporal error, the observed order of convergence in
dt against a ROW4 run at a much smaller dt on the same mesh (self-convergence, so the
spatial error cancels) reaches the scheme's nominal order within a margin.  The
order conditions and the oracle's ODE orders pin the coefficient tables; this checks
the whole GPU path (stage equations, JF products, PTC) on the PDE."""
import math

import numpy as np
import pytest
import torch

from tests.gpu_common import setup, to_gpu, vortex_state

pytestmark = pytest.mark.gpu

T = 2.0
DTS = (0.2, 0.1, 0.05)


def _run(disc, U0, kind, order, dt):
    from paper_1904_04825_amd import GmresOpts, SolverOpts
    n = int(round(T / dt))
    U = U0.clone()
    if kind == "ROW":
        opts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-12))
        for _ in range(n):
            assert disc.row_step(U, order, dt, opts)["status"] == 0
        return U
    opts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-3), tol_nl=1e-12)
    if kind == "ESDIRK":
        for _ in range(n):
            assert disc.esdirk_step(U, order, dt, opts)["status"] == 0
        return U
    Unm1 = None
    for _ in range(n):
        Unp1, st = disc.bdf2_step(Unm1, U, dt, opts)
        assert st["status"] == 0
        Unm1, U = U, Unp1
    return U


@pytest.fixture(scope="module")
def problem():
    _, op, disc = setup(12, 12, 3, "rusanov", seed=6)
    U0 = to_gpu(vortex_state(op, 0.0))
    ref = _run(disc, U0, "ROW", 4, 0.00625)
    return disc, U0, ref


@pytest.mark.parametrize("kind,order", [("ROW", 2), ("ROW", 3), ("ROW", 4), ("ESDIRK", 2), ("ESDIRK", 3),
                                        ("ESDIRK", 4), ("BDF2", 2)])
def test_temporal_order(problem, kind, order):
    disc, U0, ref = problem
    errs = []
    for dt in DTS:
        U = _run(disc, U0, kind, order, dt)
        errs.append(float(torch.linalg.norm(U[0] - ref[0]) / math.sqrt(ref[0].numel())))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"{kind}{order}: e_time(rho) {['%.3e' % e for e in errs]}, observed orders "
          f"{['%.2f' % q for q in orders]}", flush=True)
    assert np.all(np.diff(errs) < 0)
    assert orders[-1] >= order - 0.35
