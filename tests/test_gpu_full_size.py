"""GPU parity at the full workload sizes, in the launch configuration the benchmark
times (large tiles, thousands of workgroups): the whole residual and Jacobian-free
product of the 512x512 P4 perturbed vortex (26.2M DOFs) and the whole BR1 residual
of the 256x256 P3 shear layer (4.2M DOFs), element by element against the oracle."""
import numpy as np
import pytest

import fr_inputs as fi
from oracle import linear
from oracle.problem import make_euler, make_ns, sample_state
from tests.gpu_common import check_residual, rel, to_gpu, to_np

pytestmark = pytest.mark.gpu


def test_vortex_512x512_p4_residual_and_matvec():
    from paper_1904_04825_amd import Disc
    nodes = fi.workload_nodes("vortex512_p4_perturbed")
    op = make_euler(nodes, 4, flux="rusanov")
    disc = Disc(nodes, 4)
    v = fi.Vortex()
    U = sample_state(op, lambda x, y: v.conservative(x, y, 0.3))
    print("512x512 P4: oracle residual", flush=True)
    Ro = op.residual(U)
    Ug = to_gpu(U)
    Rg = to_np(disc.residual(Ug))
    worst = int(np.argmax(np.abs(Rg - Ro).reshape(4, op.nel, -1).max(axis=(0, 2))))
    print(f"  largest difference in element {worst}", flush=True)
    check_residual(Rg, Ro, op, U, "512x512 P4")
    vv = fi.random_vector(U.shape, seed=17, scale=1e-3)
    print("512x512 P4: oracle JF product", flush=True)
    Ao = linear.jf_matvec(op.residual, U, Ro, vv, 80.0, mode="rms")
    Ag = to_np(disc.jf_matvec(Ug, to_gpu(Ro), to_gpu(vv), 80.0))
    print(f"  matvec rel err {rel(Ag, Ao):.3e}", flush=True)
    assert rel(Ag, Ao) <= 1e-6


def test_shear_layer_256x256_p3_br1_residual():
    from paper_1904_04825_amd import Disc
    nodes = fi.workload_nodes("shear256_p3")
    sl = fi.ShearLayer()
    op = make_ns(nodes, 3, mu=sl.mu, prandtl=sl.prandtl)
    disc = Disc(nodes, 3, physics="ns", mu=sl.mu, prandtl=sl.prandtl)
    U = sample_state(op, sl.conservative)
    print("256x256 P3 BR1: oracle residual", flush=True)
    Ro = op.residual(U)
    Rg = to_np(disc.residual(to_gpu(U)))
    check_residual(Rg, Ro, op, U, "256x256 P3 BR1")
