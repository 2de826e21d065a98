"""GPU parity of the 3D hexahedral FR path (fr3d_*) against the FP64 oracle: residual
(Euler and BR2 Navier-Stokes, Rusanov and Roe, P2-P4, boxes that are not cubes),
Jacobian-free product, SSPRK3 steps and the Taylor-Green dissipation diagnostics."""
import math

import numpy as np
import pytest
import torch

import fr_inputs as fi
from oracle.fr3d import Box3D, NavierStokes3D, dissipation, ssprk3_step
from tests.gpu_common import rel, to_gpu, to_np
from tests.test_oracle_fr3d import _state3d

pytestmark = pytest.mark.gpu


def _pair(nx, ny, nz, P, mu, flux, lo=(0.0, 0.0, 0.0), L=(2 * math.pi,) * 3):
    from paper_1904_04825_amd import Disc3D
    box = Box3D(nx, ny, nz, list(lo), list(L), P)
    op = NavierStokes3D(box, mu=mu, flux=flux)
    disc = Disc3D(nx, ny, nz, P, lo, L, flux=flux, mu=mu)
    return box, op, disc


def _state(box):
    x, y, z = box.points()
    return _state3d(x, y, z).reshape(5, box.nel, -1)


def _floor(op, U, R, seed=0):
    """The oracle's own rounding floor: relative change of R under 1-ulp moves of U."""
    rng = np.random.default_rng(seed)
    Up = np.nextafter(U, rng.choice([-np.inf, np.inf], size=np.shape(U)))
    return rel(op.residual(Up), R)


@pytest.mark.parametrize("P", [2, 3, 4])
@pytest.mark.parametrize("mu,flux", [(0.0, "rusanov"), (0.0, "roe"), (0.05, "rusanov"), (0.05, "roe")])
def test_residual_parity(P, mu, flux):
    box, op, disc = _pair(3, 4, 5, P, mu, flux)
    U = _state(box)
    Ro = op.residual(U)
    Rg = to_np(disc.residual(to_gpu(U)))
    err = rel(Rg, Ro)
    fl = _floor(op, U, Ro) if err > 1e-12 else float("nan")
    print(f"P={P} mu={mu} {flux}: rel err {err:.2e}, floor {fl:.2e}", flush=True)
    assert err <= 1e-12 or err <= 10 * fl


def test_free_stream_and_xyz():
    box, op, disc = _pair(3, 3, 4, 3, 0.05, "roe", lo=(-1.0, 0.5, 2.0), L=(2.0, 3.0, 1.5))
    xyz = disc.solution_points()
    x, y, z = box.points()
    assert np.allclose(xyz, np.stack([x.reshape(-1), y.reshape(-1), z.reshape(-1)]), rtol=0, atol=1e-14)
    one = np.ones((box.nel, 64))
    qf = np.stack([1.2 * one, 0.4 * one, -0.3 * one, 0.2 * one, (1.1 / 0.4 + 0.5 * 0.29 / 1.2) * one])
    assert np.abs(to_np(disc.residual(to_gpu(qf)))).max() < 1e-11


@pytest.mark.parametrize("mu", [0.0, 0.05])
def test_jf_product_parity(mu):
    from oracle import linear
    box, op, disc = _pair(3, 3, 3, 2, mu, "roe")
    U = _state(box)
    R0 = op.residual(U)
    v = np.random.default_rng(3).standard_normal(U.shape) * 1e-2
    Ao = linear.jf_matvec(op.residual, U, R0, v, 7.0)
    Ag = to_np(disc.jf_matvec(to_gpu(U), to_gpu(R0), to_gpu(v), 7.0))
    assert rel(Ag, Ao) <= 1e-6


def test_taylor_green_ssprk3_and_dissipation():
    """The Taylor-Green vortex on 4^3 P3: three SSPRK3 steps of dt = 0.02 t_c agree with the
    oracle's, and so do E_k, eps1 and eps3 before and after."""
    tg = fi.TaylorGreen()
    box, op, disc = _pair(4, 4, 4, 3, tg.mu, "roe", lo=(-math.pi,) * 3, L=(2 * math.pi,) * 3)
    x, y, z = box.points()
    U = tg.conservative(x, y, z).reshape(5, box.nel, -1)
    Ug = to_gpu(U)
    do = dissipation(op, U, tg.rho0)
    dg = disc.dissipation(Ug, tg.rho0)
    print("dissipation gpu", dg, "oracle", do, flush=True)
    assert np.allclose(dg, do, rtol=1e-12, atol=1e-16)
    Uo = U.copy()
    for _ in range(3):
        disc.ssprk3_step(Ug, 0.02)
        Uo = ssprk3_step(op, Uo, 0.02)
    assert rel(to_np(Ug), Uo) <= 1e-12
    do2 = dissipation(op, Uo, tg.rho0)
    dg2 = disc.dissipation(Ug, tg.rho0)
    assert np.allclose(dg2, do2, rtol=1e-10, atol=1e-14)
    assert dg2[0] < dg[0]                       # kinetic energy decays


def test_dissipation_with_jumps_at_low_mach_pressure():
    """E_k, eps1 and eps3 of a state whose velocity jumps between elements (per-element
    slopes) at the Mach-0.1 pressure level (p about 71): eps3 takes p about its volume mean
    on both sides, so p's constant part cancels and the two agree to rounding."""
    box, op, disc = _pair(3, 4, 2, 3, 0.05, "roe")
    U = _state(box).reshape(5, box.nel, 4, 4, 4).copy()
    x, _, z = box.points()
    rng = np.random.default_rng(9)
    U[1] += 0.05 * rng.standard_normal((box.nel, 1, 1, 1)) * x
    U[3] += 0.05 * rng.standard_normal((box.nel, 1, 1, 1)) * z
    U[4] += 70.0 / 0.4
    U = U.reshape(5, box.nel, -1)
    do = dissipation(op, U, 1.0)
    dg = disc.dissipation(to_gpu(U), 1.0)
    print("dissipation gpu", dg, "oracle", do, flush=True)
    assert np.allclose(dg, do, rtol=1e-11, atol=1e-12)
