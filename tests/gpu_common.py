"""Shared set-up for the GPU parity tests: the same seeded mesh and state go to
the HIP path and to the oracle."""
import numpy as np
import torch

import fr_inputs as fi
from oracle.problem import make_euler, sample_state


def setup(nx, ny, P, flux="rusanov", seed=3, perturb=0.1, lo=-5.0, L=10.0):
    from paper_1904_04825_amd import Disc
    nodes = fi.perturbed_nodes(nx, ny, lo, lo, L, L, perturb, seed) if perturb > 0 else fi.uniform_nodes(nx, ny, lo, lo, L, L)
    op = make_euler(nodes, P, flux=flux)
    disc = Disc(nodes, P, flux=flux)
    return nodes, op, disc


def vortex_state(op, t=0.3):
    v = fi.Vortex()
    return sample_state(op, lambda x, y: v.conservative(x, y, t))


def to_gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def to_np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def residual_scale(op, U):
    """||F||/h: the size of the flux differences that cancel inside R (the parity
    budget of a single residual is 1e-12 times max(||R||, ||F||/h))."""
    from oracle.euler import physical_flux
    q = op.shape(U)
    f, g = physical_flux(q, op.gamma)
    nd = op.mesh.nodes
    h = min((nd[0, -1, 0] - nd[0, 0, 0]) / op.mesh.nx, (nd[-1, 0, 1] - nd[0, 0, 1]) / op.mesh.ny)
    return float(np.sqrt(np.sum(f * f) + np.sum(g * g)) / h)


def residual_parity(Rg, Ro, op, U):
    """Relative error of a GPU residual, measured against max(||R||, ||F||/h)."""
    d = np.linalg.norm(np.asarray(Rg).reshape(-1) - np.asarray(Ro).reshape(-1))
    return float(d / max(np.linalg.norm(Ro), residual_scale(op, U)))
