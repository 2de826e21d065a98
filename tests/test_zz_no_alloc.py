"""fr_jf_matvec_noalloc (no workspace: the library's static per-GPU scratch) against
fr_jf_matvec (caller workspace) on the same inputs, through the C ABI.  Both run the
same kernels, so the products must agree bit for bit.  Calls in a row reuse the
scratch: a large mesh first, then a smaller one; Euler (norm partial sums only) and
Navier-Stokes BR1 (gradient traces in the scratch too).  A mesh whose traces exceed
the scratch is refused on the host with FR_ESIZE."""
import numpy as np
import pytest
import torch

import fr_inputs as fi
from oracle import linear
from oracle.problem import make_ns, sample_state
from tests.gpu_common import rel, setup, to_gpu, to_np, vortex_state

pytestmark = pytest.mark.gpu


def _euler(nx, ny, P, seed):
    _, op, disc = setup(nx, ny, P, "roe", seed=seed)
    U = vortex_state(op)
    Ug = to_gpu(U)
    return disc, Ug, disc.residual(Ug), to_gpu(fi.random_vector(U.shape, seed=seed, scale=1e-3))


def _ns(nx, ny, P, seed):
    from paper_1904_04825_amd import Disc
    nodes = fi.perturbed_nodes(nx, ny, 0.0, 0.0, 1.0, 1.0, 0.1, seed)
    sl = fi.ShearLayer(width=8.0, mach=0.3)
    op = make_ns(nodes, P, mu=1e-3, prandtl=0.71)
    disc = Disc(nodes, P, physics="ns", mu=1e-3, prandtl=0.71)
    U = sample_state(op, sl.conservative)
    Ug = to_gpu(U)
    return disc, Ug, disc.residual(Ug), to_gpu(fi.random_vector(U.shape, seed=seed, scale=1e-3)), op, U


def test_noalloc_matches_workspace_product_twice():
    from paper_1904_04825_amd import EPS_ABS, EPS_RMS
    cases = [_euler(80, 70, 3, 1), _euler(9, 7, 2, 2)]       # the second call on a smaller mesh
    for disc, U, R0, v in cases:
        for mode in (EPS_RMS, EPS_ABS):
            ref = disc.jf_matvec(U, R0, v, 7.0, 1e-8, mode)
            out = disc.jf_matvec_noalloc(U, R0, v, 7.0, 1e-8, mode)
            torch.cuda.synchronize()
            print(f"{disc.nx}x{disc.ny} P{disc.p} mode {mode}: max |diff| "
                  f"{float((out - ref).abs().max()):.3e}", flush=True)
            assert torch.equal(out, ref)


def test_noalloc_navier_stokes_and_size_limit():
    from paper_1904_04825_amd import EPS_RMS, FrError
    disc, U, R0, v, op, Un = _ns(12, 10, 3, 3)
    ref = disc.jf_matvec(U, R0, v, 5.0, 1e-8, EPS_RMS)
    out = disc.jf_matvec_noalloc(U, R0, v, 5.0, 1e-8, EPS_RMS)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
    # and against the oracle, to the JF product's parity budget
    Ro = op.residual(Un)
    Ao = linear.jf_matvec(op.residual, Un, Ro, to_np(v), 5.0, mode="rms")
    assert rel(to_np(out), Ao) <= 1e-6
    # 128x128 P3: 16,777,216 bytes of traces > the 4 MiB scratch
    big, Ub, Rb, vb, _, _ = _ns(128, 128, 3, 4)
    with pytest.raises(FrError) as ei:
        big.jf_matvec_noalloc(Ub, Rb, vb, 5.0)
    assert ei.value.status == -3
    # a call after the refusal still works on the small mesh
    out2 = disc.jf_matvec_noalloc(U, R0, v, 5.0, 1e-8, EPS_RMS)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref)
