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
    Ax_g = disc.jf_matvec(Ug, to_gpu(R0), xg, shift)      # the GPU's own operator on x_g
    Ax_2 = disc.jf_matvec(Ug, to_gpu(R0), xg, shift, eps=2e-8)
    xg = to_np(xg)
    Ax_g = to_np(Ax_g)
    fd = float(np.linalg.norm(Ax_g - to_np(Ax_2)))     # the finite-difference product's own error
    nb = float(np.linalg.norm(b))
    Ax_o = A_o(xg)
    res_o = float(np.linalg.norm(b - A_o(xo)))        # oracle solution, oracle operator
    own_g = float(np.linalg.norm(b - Ax_g))            # GPU solution, GPU operator
    delta = float(np.linalg.norm(Ax_g - Ax_o))         # the two operators on x_g
    rho = rtol * so.r_ref + res_o
    print(f"  oracle {so}\n  gpu {sg}\n  rel {rel(xg, xo):.2e}; true residuals: gpu (own operator) "
          f"{own_g / nb:.2e}, oracle {res_o / nb:.2e}; operators differ on x_g by {delta / nb:.2e}, "
          f"eps vs 2 eps by {fd / nb:.2e}", flush=True)
    assert sg["status"] == 0 and sg["converged"] == 1
    # restarted cycles: DCGS2/CGS2 against MGS rounding; counts agree within a few steps
    assert abs(sg["iters"] - so.iters) <= max(2, 0.05 * so.iters)
    # each solve is as accurate under its own finite-difference operator (the true
    # residual of a Jacobian-free solve stops at the products' own error, which the
    # oracle's true residual shows); the two operators differ on x_g by rounding of R
    # amplified by 1/eps, the same noise as between eps and 2 eps
    assert own_g <= 2 * rho
    assert delta <= 4 * fd
    # kappa(A) of this operator is about 20-40 on the small meshes (dense SVD): the
    # solutions lie within kappa (2 rho + delta) / ||b|| of each other
    assert rel(xg, xo) <= 50 * (2 * rho + delta) / nb


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
            xgt = xg
            Ax1 = to_np(disc.jf_matvec(Ug, R0g, xgt, shift))              # eps = 1e-8 / rms(x)
            Ax2 = to_np(disc.jf_matvec(Ug, R0g, xgt, shift, eps=2e-8))    # twice the step
            xg = to_np(xg)
            Ao = linear.jf_matvec(op.residual, U, R0, xg, shift)
            own = float(np.linalg.norm(b - Ax1))
            fd = float(np.linalg.norm(Ax1 - Ax2))       # the finite-difference product's own error
            delta = float(np.linalg.norm(Ax1 - Ao))
            print(f"  precision {prec} m={m}: gpu {sg}; true residual (own operator) {own / nb:.2e}, "
                  f"product error (eps vs 2 eps) {fd / nb:.2e}, GPU vs oracle operator on x {delta / nb:.2e}",
                  flush=True)
            assert sg["status"] == 0 and sg["converged"] == 1 and sg["iters"] > 1
            assert sg["r_final"] <= rtol * sg["r_ref"]
            # the true residual of a Jacobian-free solve: the tolerance plus the
            # products' own error; the GPU's and the oracle's products on x differ by
            # rounding of R amplified by 1/eps, the same noise as between eps and 2 eps
            assert own <= 2 * rtol * nb + 2 * fd
            assert delta <= 4 * fd
