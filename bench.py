"""Benchmark: Jacobian-free implicit time steps of the FR/CPR vortex on one MI355X.

A step is one ROW3 (ROS34PW2) time step of the isentropic vortex on the
64x64 perturbed quad mesh at P = 3 (262,144 DOFs), dt = 0.1, GMRES(20) with
rtol 1e-8 and the FP64 element-Jacobi preconditioner, Rusanov flux: residual
evaluations, Jacobian-free products, element-Jacobi assembly, inversion and
application, and the Arnoldi/Givens loop all run in the HIP library.  Inputs
(mesh, state) are synthetic and resident in HBM before timing.

value = DOF-residuals/s = ndof x (residual evaluations incl. JF products) / wall time.
The JSON line also carries the roofline of the dominant kernel (live HIP-event
timing on the launch stream) and the FP64 oracle's rate on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "vortex64_p3_perturbed"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dt", type=float, default=0.1)
    ap.add_argument("--scheme", type=int, default=3)
    ap.add_argument("--precond", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernels", action="store_true", help="skip the per-kernel timing block")
    ap.add_argument("--no-fp32-leg", action="store_true", help="skip the FP32-preconditioner comparison")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device-to-device copy (counter calibration for rocprofv3 --pmc runs)")
    return ap.parse_args()


def source_sha(rel):
    """Hash of the source file of a kernel: counter-derived traffic is reported only while
    the kernel is unchanged since the counters were taken."""
    with open(os.path.join(ROOT, rel), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def time_kernel(fn, reps=50, warm=5):
    """Average duration of fn() (one launch on torch's current stream) by HIP events."""
    import torch
    for _ in range(warm):
        fn()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    e.synchronize()
    return s.elapsed_time(e) / reps * 1e-3


def cpu_baseline(nodes, U0, dt):
    """The FP64 oracle on the host: R(U), the element-Jacobi blocks at q^n and the
    first 30 FGMRES iterations of ROW3 stage 1 of the same workload (single thread)."""
    from threadpoolctl import threadpool_limits

    from oracle import integrators as I
    from oracle import linear
    from oracle.problem import make_euler
    from oracle.tableaux import ROW
    op = make_euler(nodes, 3, flux="rusanov")
    with threadpool_limits(1):
        t0 = time.perf_counter()
        R = I.Counted(op)
        R0 = R(U0)
        shift = 1.0 / (ROW["ROW3"].gamma * dt)
        pc = linear.ElementJacobi(op, U0, shift)
        x, st = linear.fgmres(lambda v: linear.jf_matvec(R, U0, R0, v, shift), pc.apply, R0, m=20, rtol=1e-8,
                              max_iters=30)
        wall = time.perf_counter() - t0
    evals = R.count
    return {"value": op.ndof * evals / wall, "unit": "DOF-residuals/s", "cores": 1, "kind": "oracle",
            "sample": f"R(U) + element-Jacobi assembly + {st.iters} FGMRES(20) iterations of ROW3 stage 1 on the "
                      f"same 64x64 P3 mesh: {evals} residual evaluations in {wall:.1f} s, numpy, 1 thread"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import fr_inputs as fi
    from paper_1904_04825_amd import F32, F64, Disc, GmresOpts, SolverOpts

    dev = torch.device("cuda:0")
    nodes = fi.workload_nodes(WORKLOAD)
    disc = Disc(nodes, 3, flux="rusanov", device=dev)
    vortex = fi.Vortex()
    xy = disc.solution_points().cpu().numpy()
    U0_np = vortex.conservative(xy[0], xy[1], 0.0)
    U0 = torch.as_tensor(U0_np, device=dev).contiguous()
    prec = F64 if args.precond == "f64" else F32
    opts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-8), precond_precision=prec)
    U = U0.clone()
    for _ in range(args.warmup):
        disc.row_step(U, args.scheme, args.dt, opts)
    U.copy_(U0)
    torch.cuda.synchronize()
    evals = iters = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = disc.row_step(U, args.scheme, args.dt, opts)
        if st["status"] != 0:
            raise RuntimeError(f"row_step status {st['status']}")
        evals += st["residual_evals"]
        iters += st["gmres_iters"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ndof = disc.ndof
    value = ndof * evals / wall
    t_phys = args.steps * args.dt
    err_rho = disc.l2_error_vortex(U, 0, t_phys, vortex)

    out = {
        "metric": "DOF-residuals/s", "value": value, "unit": "DOF-residuals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"isentropic vortex, 64x64 perturbed quads (seed 2), P3, 262144 DOFs, "
                               f"ROW{args.scheme} dt={args.dt}, FGMRES(20) rtol 1e-8, element-Jacobi "
                               f"{args.precond.upper()}, Rusanov, eps_rms 1e-8",
                   "ndof": ndof, "dt": args.dt},
        "extra": {"wall_s_per_time_unit": wall / t_phys, "gmres_iters_per_step": iters / args.steps,
                  "residual_evals_per_step": evals / args.steps, "l2_err_rho": err_rho, "t_end": t_phys},
    }

    if not args.no_kernels:
        # live per-kernel timing on the launch stream (torch's current stream)
        R0 = disc.residual(U0)
        v = torch.randn_like(U0) * 1e-3
        shift = 1.0 / (0.4358665215084590 * args.dt)
        pc = disc.ejacobi_factor(U0, shift, prec)
        z = disc.empty()
        t_res = time_kernel(lambda: disc.residual(U0, R0))
        Av = disc.empty()
        t_mv = time_kernel(lambda: disc.jf_matvec(U0, R0, v, shift, out=Av))
        t_sol = time_kernel(lambda: disc.ejacobi_solve(pc, v, z))
        t_fac = time_kernel(lambda: disc.ejacobi_factor(U0, shift, prec, pc), reps=10, warm=2)
        nb = disc.nb
        es = 8 if prec == F64 else 4
        solve_bytes = disc.nel * nb * nb * es + 16 * ndof          # block inverse + r in + z out
        res_bytes = 16 * ndof                                        # U in, R out
        kernels = {
            "fr_residual": {"us": t_res * 1e6, "alg_bytes": res_bytes, "GBs": res_bytes / t_res / 1e9,
                            "dof_res_per_s": ndof / t_res},
            "jf_matvec(norm+fused residual)": {"us": t_mv * 1e6, "alg_bytes": 40 * ndof,
                                               "GBs": 40 * ndof / t_mv / 1e9},
            "ejacobi_solve": {"us": t_sol * 1e6, "alg_bytes": solve_bytes, "GBs": solve_bytes / t_sol / 1e9},
            "ejacobi_factor(assemble+invert)": {"us": t_fac * 1e6, "alg_bytes": disc.nel * nb * nb * es,
                                                "GBs": disc.nel * nb * nb * es / t_fac / 1e9},
        }
        out["extra"]["kernels"] = kernels
        dom = "ejacobi_solve"
        traffic = None
        tp = os.path.join(ROOT, "profiles", "traffic.json")
        if os.path.exists(tp):
            with open(tp) as fh:
                tj = json.load(fh)
            if tj.get("kernel") == dom and tj.get("source_sha") == source_sha(tj["source"]) \
                    and prec == F64 and WORKLOAD == "vortex64_p3_perturbed":
                traffic = tj.get("bytes_per_launch")
        ach = kernels[dom]["GBs"]
        out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                           "alg_bytes_per_launch": solve_bytes}

    if args.precond == "f64" and not args.no_fp32_leg:
        # the same steps with the FP32 element-Jacobi factored on MFMA
        opts32 = SolverOpts(lin=GmresOpts(m=20, rtol=1e-8), precond_precision=F32)
        U32 = U0.clone()
        disc.row_step(U32, args.scheme, args.dt, opts32)
        U32.copy_(U0)
        torch.cuda.synchronize()
        ev32 = it32 = 0
        t1 = time.perf_counter()
        for _ in range(args.steps):
            st = disc.row_step(U32, args.scheme, args.dt, opts32)
            ev32 += st["residual_evals"]
            it32 += st["gmres_iters"]
        torch.cuda.synchronize()
        w32 = time.perf_counter() - t1
        out["extra"]["fp32_precond"] = {
            "ms_per_step": w32 / args.steps * 1e3, "wall_s_per_time_unit": w32 / t_phys,
            "gmres_iters_per_step": it32 / args.steps, "dof_res_per_s": ndof * ev32 / w32,
            "l2_err_rho": disc.l2_error_vortex(U32, 0, t_phys, vortex),
            "rel_diff_vs_fp64_state": float(torch.linalg.norm(U32 - U) / torch.linalg.norm(U))}
        pc32 = disc.ejacobi_factor(U0, 1.0 / (0.4358665215084590 * args.dt), F32)
        z = disc.empty()
        v = torch.randn_like(U0)
        t_s32 = time_kernel(lambda: disc.ejacobi_solve(pc32, v, z))
        t_f32 = time_kernel(lambda: disc.ejacobi_factor(U0, 1.0 / (0.4358665215084590 * args.dt), F32, pc32),
                            reps=10, warm=2)
        nb = disc.nb
        b32 = disc.nel * nb * nb * 4 + 16 * ndof
        out["extra"]["kernels"]["ejacobi_solve_fp32"] = {"us": t_s32 * 1e6, "alg_bytes": b32,
                                                         "GBs": b32 / t_s32 / 1e9}
        fl = disc.nel * 2.0 * nb ** 3   # Gauss-Jordan inversion flops
        out["extra"]["kernels"]["ejacobi_factor_fp32_mfma(assemble+invert)"] = {
            "us": t_f32 * 1e6, "inversion_TFLOPs": fl / t_f32 / 1e12}

    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["extra"]["calib_copy_bytes"] = src.numel() * 8

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(nodes, U0_np.reshape(4, disc.nel, -1), args.dt)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
