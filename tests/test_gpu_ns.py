"""GPU parity of the BR1 Navier-Stokes path against the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import fr_inputs as fi
from oracle import integrators as I
from oracle import linear
from oracle.problem import make_ns, sample_state
from oracle.tableaux import ESDIRK, ROW
from tests.gpu_common import check_residual, rel, to_gpu, to_np

pytestmark = pytest.mark.gpu

MESHES = {2: (11, 9), 3: (9, 10), 4: (7, 6)}


def _setup(nx, ny, P, flux="rusanov", mu=0.01, seed=3, box=(0.0, 1.0)):
    from paper_1904_04825_amd import Disc
    lo, L = box
    nodes = fi.perturbed_nodes(nx, ny, lo, lo, L, L, 0.1, seed)
    op = make_ns(nodes, P, flux=flux, mu=mu)
    disc = Disc(nodes, P, physics="ns", flux=flux, mu=mu, prandtl=0.71)
    return op, disc


def _shear(op, width=8.0):
    sl = fi.ShearLayer(width=width, mach=0.3)
    return sample_state(op, sl.conservative)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("flux", ["rusanov", "roe"])
def test_ns_residual_parity(P, flux):
    nx, ny = MESHES[P]
    op, disc = _setup(nx, ny, P, flux)
    U = _shear(op)
    Rg = to_np(disc.residual(to_gpu(U)))
    Ro = op.residual(U)
    check_residual(Rg, Ro, op, U, f"NS P={P} {flux}")


def test_ns_residual_conservation_and_freestream():
    op, disc = _setup(9, 10, 3, "roe")
    R = to_np(disc.residual(to_gpu(_shear(op)))).reshape(4, op.nel, -1)
    w = op.b.w
    wk = (w[:, None] * w[None, :]).reshape(-1)
    J = op.geo.J.reshape(op.nel, -1)
    for v in range(4):
        assert abs(np.sum(wk * J * R[v])) < 1e-10
    one = np.ones((op.nel, 16))
    Uf = np.stack([1.2 * one, 0.84 * one, -0.48 * one, (0.9 / 0.4 + 0.5 * 1.2 * (0.49 + 0.16)) * one])
    assert np.abs(to_np(disc.residual(to_gpu(Uf)))).max() < 1e-11


@pytest.mark.parametrize("P", [2, 3])
def test_ns_jf_matvec_parity(P):
    nx, ny = MESHES[P]
    op, disc = _setup(nx, ny, P, "roe")
    U = _shear(op)
    R0 = op.residual(U)
    v = fi.random_vector(U.shape, seed=7, scale=1e-2)
    Ao = linear.jf_matvec(op.residual, U, R0, v, 9.0)
    Ag = to_np(disc.jf_matvec(to_gpu(U), to_gpu(R0), to_gpu(v), 9.0))
    assert rel(Ag, Ao) <= 1e-6


@pytest.mark.parametrize("P", [2, 3, 4])
def test_ns_ejacobi_blocks_parity(P):
    op, disc = _setup(4, 4, P, "rusanov", mu=0.02, seed=9)
    U = _shear(op)
    Bo = linear.ejacobi_blocks(op, U, 5.0)
    Bg = to_np(disc.ejacobi_assemble(to_gpu(U), 5.0))
    for e in range(op.nel):
        assert np.linalg.norm(Bg[e] - Bo[e]) <= 1e-6 * np.linalg.norm(Bo[e])


def test_ns_row4_and_esdirk4_steps():
    from paper_1904_04825_amd import GmresOpts, SolverOpts
    op, disc = _setup(6, 5, 2, "roe", mu=0.01, seed=2)
    U = _shear(op)
    dt = 0.02
    Ug = to_gpu(U)
    st = disc.row_step(Ug, 4, dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-10)))
    Uo, so = I.row_step(op, ROW["ROW4"], dt, U, I.LinOpts(m=20, rtol=1e-10))
    assert st["status"] == 0 and rel(to_np(Ug), Uo) <= 1e-8
    Ug = to_gpu(U)
    st = disc.esdirk_step(Ug, 4, dt, SolverOpts(lin=GmresOpts(m=20, rtol=1e-10), tol_nl=1e-10))
    Uo, so = I.esdirk_step(op, ESDIRK["ESDIRK4"], dt, U, I.LinOpts(m=20, rtol=1e-10), I.NlOpts(tol_nl=1e-10))
    assert st["status"] == 0 and rel(to_np(Ug), Uo) <= 1e-8
