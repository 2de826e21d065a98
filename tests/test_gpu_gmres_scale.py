"""GPU FGMRES at the mesh sizes and launch configurations the benchmark runs.

* 72x72 P3 (324 residual tiles, more than the 256 compute units, at most 1024 so the
  JF product also carries the first DCGS2 pass): the bench's GMRES(20) path, and the
  paper's restart length m = 60 (CGS2), element by element against the oracle's solve.
* 250x645 P2 (2064 large residual tiles, ragged in both directions): the solve path of
  the large meshes (separate DCGS2 passes, norms over 1024 workgroups), checked by a
  property that holds at any size: the GPU solution's true residual under the oracle's
  own Jacobian-free operator meets the tolerance.
"""
import numpy as np
import pytest

import fr_inputs as fi
from oracle import linear
from oracle.tableaux import ROW
from tests.gpu_common import rel, setup, to_gpu, to_np, vortex_state

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m", [20, 60])
def test_gmres_parity_multitile_72x72_p3(m):
    from paper_1904_04825_amd import F64, GmresOpts
    _, op, disc = setup(72, 72, 3, "rusanov", seed=2)
    U = vortex_state(op, 0.0)
    R0 = op.residual(U)
    shift = 1.0 / (ROW["ROW3"].gamma * 0.1)      # a ROW3 stage at dt = 0.1
    b = R0.copy()                                 # the first stage's right-hand side
    rtol = 1e-8
    print(f"72x72 P3 m={m}: oracle solve", flush=True)
    pc_o = linear.ElementJacobi(op, U, shift)

    def A_o(v):
        return linear.jf_matvec(op.residual, U, R0, v, shift)

    xo, so = linear.fgmres(A_o, pc_o.apply, b, m=m, rtol=rtol)
    Ug = to_gpu(U)
    pc = disc.ejacobi_factor(Ug, shift, F64)
    xg, sg = disc.gmres_solve(pc, Ug, to_gpu(R0), shift, to_gpu(b), opts=GmresOpts(m=m, rtol=rtol))
    xg = to_np(xg)
    nb = float(np.linalg.norm(b))
    res_o = float(np.linalg.norm(b - A_o(xo)))
    res_g = float(np.linalg.norm(b - A_o(xg)))
    rho = rtol * so.r_ref + res_o
    print(f"  oracle {so}\n  gpu {sg}\n  rel {rel(xg, xo):.2e}  true residual gpu {res_g / nb:.2e} "
          f"oracle {res_o / nb:.2e}", flush=True)
    assert sg["status"] == 0 and sg["converged"] == 1
    # restarted cycles: DCGS2/CGS2 against MGS rounding; counts agree within a few steps
    assert abs(sg["iters"] - so.iters) <= max(2, 0.05 * so.iters)
    assert res_g <= 2 * rho
    # kappa(A) of this operator is about 20-40 on the small meshes (dense SVD):
    # solutions within 3 rho kappa / ||b||
    assert rel(xg, xo) <= 3 * 50 * rho / nb


def test_gmres_large_tiles_250x645_p2():
    from paper_1904_04825_amd import F32, F64, GmresOpts
    _, op, disc = setup(250, 645, 2, "rusanov", seed=7)
    U = vortex_state(op, 0.2)
    shift = 1.0 / (ROW["ROW3"].gamma * 0.05)
    print("250x645 P2: oracle R(U)", flush=True)
    R0 = op.residual(U)
    b = R0.copy()
    rtol = 1e-6
    Ug, R0g, bg = to_gpu(U), to_gpu(R0), to_gpu(b)
    nb = float(np.linalg.norm(b))
    for prec in (F64, F32):
        pc = disc.ejacobi_factor(Ug, shift, prec)
        for m in (20, 40):
            xg, sg = disc.gmres_solve(pc, Ug, R0g, shift, bg, opts=GmresOpts(m=m, rtol=rtol))
            xg = to_np(xg)
            res = float(np.linalg.norm(b - linear.jf_matvec(op.residual, U, R0, xg, shift)))
            print(f"  precision {prec} m={m}: gpu {sg}, true residual under the oracle's operator {res / nb:.2e}",
                  flush=True)
            assert sg["status"] == 0 and sg["converged"] == 1 and sg["iters"] > 1
            assert sg["r_final"] <= rtol * sg["r_ref"]
            assert res <= 2 * rtol * nb
