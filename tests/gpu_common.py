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


def _rebuilt(op, nodes):
    """The same oracle operator on another vertex array."""
    from oracle.ns import NavierStokesFR
    from oracle.ns_bc import NavierStokesBC
    from oracle.problem import make_ns, make_ns_bc
    P = op.n - 1
    if isinstance(op, NavierStokesBC):
        return make_ns_bc(nodes, P, gamma=op.gamma, flux=op.flux, rgas=op.rgas, mu=op.mu, prandtl=op.prandtl,
                          viscous=op.viscous, bc_south=op.bc["S"], bc_north=op.bc["N"], q_far=op.q_far)
    if isinstance(op, NavierStokesFR):
        return make_ns(nodes, P, gamma=op.gamma, flux=op.flux, rgas=op.rgas, mu=op.mu, prandtl=op.prandtl)
    return make_euler(nodes, P, gamma=op.gamma, flux=op.flux)


def ulp_nodes(nodes, rng, periodic_y=True):
    """Every vertex coordinate moved by one unit in its last place (seeded random
    direction), the periodic copies kept exact copies shifted by the box lengths (in y
    only on doubly periodic meshes)."""
    nd = np.nextafter(nodes, rng.choice([-np.inf, np.inf], size=np.shape(nodes)))
    ny, nx = nd.shape[0] - 1, nd.shape[1] - 1
    lx = nodes[0, nx, 0] - nodes[0, 0, 0]
    ly = nodes[ny, 0, 1] - nodes[0, 0, 1]
    nd[:, nx, 0] = nd[:, 0, 0] + lx
    nd[:, nx, 1] = nd[:, 0, 1]
    if periodic_y:
        nd[ny, :, 1] = nd[0, :, 1] + ly
        nd[ny, :, 0] = nd[0, :, 0]
    return nd


def rounding_floor(op, U, R, trials=2, seed=0):
    """The oracle's own rounding floor for R(U): the largest relative change of R when
    every entry of U and every vertex coordinate move by one unit in their last place,
    each in a seeded random direction.  Two correct FP64 evaluations that round in
    different orders (the metrics from the vertices included) differ by about this much:
    R is a small difference of fluxes of size |F|/h, so rounding in the metric terms is
    amplified by (|F|/h)/|R|."""
    rng = np.random.default_rng(seed)
    worst = 0.0
    for _ in range(trials):
        Up = np.nextafter(U, rng.choice([-np.inf, np.inf], size=np.shape(U)))
        bounded = getattr(op, "bc", {}).get("S") is not None or getattr(op, "bc", {}).get("N") is not None
        opp = _rebuilt(op, ulp_nodes(op.mesh.nodes, rng, periodic_y=not bounded))
        worst = max(worst, rel(opp.residual(Up), R))
    return worst


# A GPU residual may differ from the oracle's by at most this many times the oracle's
# own rounding floor where that floor lies above 1e-12 relative.
FLOOR_MULT = 10.0


def check_residual(Rg, Ro, op, U, label=""):
    """Assert the relative error of a GPU residual: 1e-12 where FP64 allows it, else
    FLOOR_MULT times the measured rounding floor of the oracle.  Returns (error, floor)."""
    err = rel(Rg, Ro)
    floor = rounding_floor(op, U, Ro) if err > 1e-12 else float("nan")
    print(f"  {label} residual rel err {err:.3e}, oracle rounding floor {floor:.3e}", flush=True)
    assert err <= 1e-12 or err <= FLOOR_MULT * floor, (err, floor)
    return err, floor


def dense_operator(residual, U, shift, h=1e-6):
    """A = shift I - dR/dq at U as a dense matrix, by central differences of the oracle's
    residual (one column per degree of freedom; small meshes only)."""
    u = np.asarray(U, dtype=np.float64).reshape(-1)
    n = u.size
    A = np.empty((n, n))
    for j in range(n):
        up, um = u.copy(), u.copy()
        up[j] += h
        um[j] -= h
        A[:, j] = -(residual(up.reshape(np.shape(U))) - residual(um.reshape(np.shape(U)))).reshape(-1) / (2 * h)
        A[j, j] += shift
    return A


def gmres_solution_bound(A, b, x_ref, r_ref, rtol):
    """Derived parity bound for two GMRES solutions of A x = b.  Each solve stops when its
    residual estimate is at most rtol r_ref; the finite-difference products add their own
    error, which the reference solution's true residual under A shows.  With
    rho = rtol r_ref + ||b - A x_ref||, a solution x with ||b - A x|| <= 2 rho lies within
    ||A^{-1}|| (2 rho + ||b - A x_ref||) <= 3 rho / sigma_min(A) of x_ref.
    Returns (rho, relative bound 3 rho / (sigma_min ||x_ref||))."""
    smin = np.linalg.svd(A, compute_uv=False)[-1]
    rho = rtol * r_ref + float(np.linalg.norm(b.reshape(-1) - A @ x_ref.reshape(-1)))
    return rho, 3.0 * rho / (smin * float(np.linalg.norm(x_ref)))
