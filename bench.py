"""Benchmark: Jacobian-free implicit time steps of FR/CPR flows on one MI355X.

Default workload (the combined-at-scale configuration): the isentropic vortex on
512x512 perturbed quads (mesh seed 5), P = 4, 26,214,400 DOFs, 100x100 element
blocks; a step is one ROW4 (RODASP) time step with dt = 0.0125, FGMRES(20) at rtol
1e-8, Rusanov flux.  Residual evaluations, Jacobian-free products, element-Jacobi
assembly/inversion/application, the Arnoldi/Givens loop and the learned warm start
all run in the HIP library; inputs are synthetic and resident in HBM before timing.

Phases: (1) untimed warm-up: `--warmup` steps from t = 0 (FP32 element-Jacobi) that
also log the stage solves (training data); (2) one network per ROW stage trained on
the GPU from those logs; (3) timed: `--steps` steps from the warm-up's end state with
the plain FP64 element-Jacobi (the headline `value`), then the same steps with the
FP32 MFMA element-Jacobi, then FP32 + learned warm start; all three legs end at the
same time with the same rho L2 error against the exact vortex (reported, and their
relative difference); (4) optional (`--schemes`): the ESDIRK and BDF2 legs from the
same state.

value = DOF-residuals/s = ndof x (residual evaluations incl. JF products) / wall time
of the FP64 leg.  The JSON line also carries wall-seconds per unit physical time of
every leg at the matched error, the learned leg's training and logging cost and its
break-even step count, the dominant kernel's roofline (live HIP-event timing on the
launch stream) and the FP64 oracle's rate on the host's cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "vortex64_p3": dict(nodes="vortex64_p3_perturbed", p=3, physics="euler", scheme=3, dt=0.1, state="vortex",
                        label="isentropic vortex, 64x64 perturbed quads (seed 2), P3, 262144 DOFs"),
    "shear256_p3_ns": dict(nodes="shear256_p3", p=3, physics="ns", scheme=4, dt=1e-3, state="shear",
                           label="Navier-Stokes shear layer (Re 1e4, M 0.1), 256x256 quads, P3, BR1, 4194304 DOFs"),
    "vortex512_p4": dict(nodes="vortex512_p4_perturbed", p=4, physics="euler", scheme=4, dt=0.0125, state="vortex",
                         label="isentropic vortex, 512x512 perturbed quads (seed 5), P4, 26214400 DOFs"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=6, help="untimed logging steps (training data for the warm start)")
    ap.add_argument("--workload", default="vortex512_p4", choices=sorted(WORKLOADS))
    ap.add_argument("--dt", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernels", action="store_true", help="skip the per-kernel timing block")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the per-kernel timing block, at the initial state (for profiler runs)")
    ap.add_argument("--no-learned", action="store_true", help="skip logging, training and the learned leg")
    ap.add_argument("--log-elems", type=int, default=1024, help="elements logged per stage solve (training samples)")
    ap.add_argument("--adam-steps", type=int, default=1500, help="Adam steps per stage network")
    ap.add_argument("--batch", type=int, default=1024, help="training batch (samples)")
    ap.add_argument("--no-fp32-leg", action="store_true", help="skip the FP32-preconditioner legs")
    ap.add_argument("--schemes", action="store_true", help="also run the ESDIRK and BDF2 legs")
    ap.add_argument("--allow-unconverged", action="store_true",
                    help="count GMRES solves that reach the iteration cap instead of stopping")
    ap.add_argument("--order-study", action="store_true",
                    help="instead of the bench line: ROW3, ESDIRK3 and BDF2 over t in [0, 10] at dt 0.2, 0.1, 0.05 "
                         "on the 64x64 P3 vortex; errors against the exact vortex and against a ROW4 run at "
                         "dt 0.0125, observed orders, wall seconds per unit time")
    ap.add_argument("--cpu-sample", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--paper-vortex", default=None,
                    help="instead of the bench line: the paper's vortex study (50x50 P6, Roe, GMRES(60)); a comma "
                         "list of SCHEME/STEPS entries of tests/golden/paper_vortex_tables.json, or 'all'")
    ap.add_argument("--cylinder", action="store_true",
                    help="instead of the bench line: the cylinder case's scheme comparison (120x48 P3 O-grid, "
                         "BR2, wall and far field, Re 1200, M 0.1)")
    ap.add_argument("--cyl-schemes", default="ROW3,ROW4,ESDIRK3,ESDIRK4,BDF2")
    ap.add_argument("--cyl-dts", default="0.2,0.1,0.05")
    ap.add_argument("--cyl-tdev", type=float, default=2.0)
    ap.add_argument("--cyl-devdt", type=float, default=0.05)
    ap.add_argument("--cyl-devtol", type=float, default=1e-3, help="nonlinear tolerance of the development run")
    ap.add_argument("--cyl-ref-save", default=None, help="save the reference C_d history (.json)")
    ap.add_argument("--cyl-ref-load", default=None, help="take the reference C_d history from a saved run")
    ap.add_argument("--cyl-settle", type=float, default=0.0, help="time units of ESDIRK4 at dt 0.01 after the development")
    ap.add_argument("--cyl-save", default=None, help="save the developed state (.npy)")
    ap.add_argument("--cyl-load", default=None, help="start from a saved developed state instead of developing")
    ap.add_argument("--cyl-trun", type=float, default=1.0)
    ap.add_argument("--cyl-dtref", type=float, default=0.00625)
    ap.add_argument("--cyl-tolnl", type=float, default=1e-6, help="ESDIRK / BDF2 nonlinear tolerance (the paper's 1e-6)")
    ap.add_argument("--cyl-tollin", type=float, default=1e-6, help="ROW linear tolerance (the paper's 1e-6)")
    ap.add_argument("--tgv", action="store_true",
                    help="instead of the bench line: the Taylor-Green vortex on 3D hexahedra (residual timing, "
                         "SSPRK3 steps with the dissipation diagnostics)")
    ap.add_argument("--tgv-n", type=int, default=64)
    ap.add_argument("--tgv-p", type=int, default=3)
    ap.add_argument("--tgv-steps", type=int, default=50)
    ap.add_argument("--tgv-dt", type=float, default=2e-4, help="SSPRK3 step in units of t_c (the paper's 2e-4)")
    ap.add_argument("--tgv-sample", type=int, default=10)
    ap.add_argument("--tgv-implicit", action="store_true",
                    help="instead of the bench line: the implicit schemes on the Taylor-Green vortex (Section 5.3), "
                         "Error(eps) against SSPRK3 over a window of t / t_c")
    ap.add_argument("--tgvi-n", type=int, default=16)
    ap.add_argument("--tgvi-schemes", default="ROW2,ROW3,ROW4,ESDIRK2,ESDIRK3,ESDIRK4,BDF2")
    ap.add_argument("--tgvi-steps-per-tc", default="25,50,100", help="dt = t_c / k for each k")
    ap.add_argument("--tgvi-t0", type=float, default=8.0)
    ap.add_argument("--tgvi-t1", type=float, default=9.0)
    ap.add_argument("--tgvi-ref-save", default=None, help="save the SSPRK3 reference (state at t0 and eps) (.npz)")
    ap.add_argument("--tgvi-ref-load", default=None)
    ap.add_argument("--mach-reading", default="magnitude", choices=["magnitude", "u"],
                    help="velocity of the paper's Mach number: |V| or u")
    ap.add_argument("--study-eps", default="rms", choices=["abs", "rms"],
                    help="JF perturbation of the paper-vortex study: the literal eps (abs) or eps / rms(v)")
    ap.add_argument("--study-precond", default="f64", choices=["f64", "f32"],
                    help="element-Jacobi precision of the paper-vortex study")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device-to-device copy (counter calibration for rocprofv3 --pmc runs)")
    return ap.parse_args()


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result line)."""
    print(f"# bench: {msg} ({time.strftime('%H:%M:%S')})", file=sys.stderr, flush=True)


def source_sha(rel):
    """Hash of the source file of a kernel: counter-derived traffic is reported only while
    the kernel is unchanged since the counters were taken."""
    with open(os.path.join(ROOT, rel), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def calib_copy(dev):
    """Three 1 GiB device-to-device copies: the counter readings of a plain copy of known
    size, to scale FETCH_SIZE / WRITE_SIZE of the kernels to bytes."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return src.numel() * 8


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


def cpu_sample(spec):
    """One bounded sample of the FP64 oracle on one host core (run in a child process that
    never touches the GPU): the first ROW stage of the workload's kind on a smaller mesh --
    R(U), the element-Jacobi blocks at q^n and `iters` FGMRES(20) iterations -- or, with
    iters = 0, one residual evaluation on the full mesh.  Prints one JSON line."""
    from threadpoolctl import threadpool_limits

    import fr_inputs as fi
    from oracle import integrators as I
    from oracle import linear
    from oracle.problem import make_euler, sample_state
    from oracle.tableaux import ROW
    nx, p, seed, iters, scheme, dt = (spec[k] for k in ("nx", "p", "seed", "iters", "scheme", "dt"))
    nodes = fi.workload_nodes(spec["nodes"]) if spec.get("nodes") else fi.perturbed_nodes(nx, nx, -5.0, -5.0, 10.0,
                                                                                          10.0, 0.1, seed)
    op = make_euler(nodes, p, flux="rusanov")
    vx = fi.Vortex()
    U = sample_state(op, lambda x, y: vx.conservative(x, y, 0.0))
    with threadpool_limits(1):
        R = I.Counted(op)
        t0 = time.perf_counter()
        R0 = R(U)
        if iters > 0:
            shift = 1.0 / (ROW[f"ROW{scheme}"].gamma * dt)
            pc = linear.ElementJacobi(op, U, shift)
            _, st = linear.fgmres(lambda v: linear.jf_matvec(R, U, R0, v, shift), pc.apply, R0, m=20, rtol=1e-8,
                                  max_iters=iters)
        wall = time.perf_counter() - t0
    print(json.dumps({"ndof": op.ndof, "evals": R.count, "wall": wall}), flush=True)


def _children(spec, n):
    """Run n concurrent single-thread oracle samples as child processes; returns their results."""
    import subprocess
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-sample", json.dumps(spec)]
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    procs = [subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
             for _ in range(n)]
    res = []
    for pr in procs:
        so, se = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError(f"oracle sample failed: {se[-2000:]}")
        res.append(json.loads(so.strip().splitlines()[-1]))
    return res


def cpu_baseline(W, dt, scheme):
    """The FP64 oracle (numpy, as it stands) on the host's cores.  Bounded samples: the first
    ROW stage of the same kind of workload on a 64x64 perturbed mesh at the same degree
    (R(U), element-Jacobi blocks, 20 FGMRES(20) iterations; every operation is linear in
    the number of elements, so the per-DOF rate carries over), once on one core and as
    concurrent single-thread processes on all cores (aggregate rate); plus one residual
    evaluation on the full mesh, which shows the per-DOF rate at full size."""
    import platform
    ncpu = os.cpu_count() or 1
    ncores = max(1, min(ncpu, 16))
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    spec = {"nx": 64, "p": W["p"], "seed": 5, "iters": 20, "scheme": scheme, "dt": dt}
    one = _children(spec, 1)[0]
    allc = _children(spec, ncores)
    full = _children({**spec, "nodes": W["nodes"], "iters": 0}, 1)[0]
    rate1 = one["ndof"] * one["evals"] / one["wall"]
    rate_all = sum(r["ndof"] * r["evals"] for r in allc) / max(r["wall"] for r in allc)
    return {"value": rate_all, "unit": "DOF-residuals/s", "cores": ncores, "kind": "oracle",
            "sample": f"ROW{scheme} stage-1 pipeline of the FP64 numpy oracle (R(U), element-Jacobi blocks at q^n, "
                      f"FGMRES(20) to rtol 1e-8, at most 20 iterations; {one['evals']} residual evaluations) on a 64x64 perturbed P{W['p']} "
                      f"vortex mesh ({one['ndof']} DOFs), {ncores} concurrent single-thread processes (aggregate "
                      f"rate, per-DOF rate taken as the full mesh's: every step is linear in the element count)",
            "one_core": {"value": rate1, "wall_s": one["wall"]},
            "full_mesh_residual": {"dof_res_per_s": full["ndof"] * full["evals"] / full["wall"],
                                   "ndof": full["ndof"], "wall_s": full["wall"], "cores": 1},
            "host": {"nproc": ncpu, "cpu_model": model}}


def kernel_block(disc, Ustart, dt, scheme, ndof, workload):
    """Per-kernel timings (HIP events on the launch stream) at state Ustart and the
    roofline object of the dominant kernel."""
    from paper_1904_04825_amd import F32, F64
    import torch
    out = {"extra": {}}
    # live per-kernel timing on the launch stream (torch's current stream)
    R0 = disc.residual(Ustart)
    v = torch.randn_like(Ustart) * 1e-3
    gam = {2: 0.25, 3: 0.4358665215084590, 4: 0.25}[scheme]
    shift = 1.0 / (gam * dt)
    nb = disc.nb
    kernels = {}
    t_res = time_kernel(lambda: disc.residual(Ustart, R0))
    res_bytes = 16 * ndof
    kernels["fr_residual"] = {"us": t_res * 1e6, "alg_bytes": res_bytes, "GBs": res_bytes / t_res / 1e9,
                              "dof_res_per_s": ndof / t_res}
    Av = disc.empty()
    t_mv = time_kernel(lambda: disc.jf_matvec(Ustart, R0, v, shift, out=Av))
    kernels["jf_matvec(norm+fused residual)"] = {"us": t_mv * 1e6, "alg_bytes": 40 * ndof,
                                                 "GBs": 40 * ndof / t_mv / 1e9}
    z = disc.empty()
    for prec, name, es in ((F64, "fp64", 8), (F32, "fp32", 4)):
        pc = disc.ejacobi_factor(Ustart, shift, prec)
        t_sol = time_kernel(lambda: disc.ejacobi_solve(pc, v, z))
        sb = disc.nel * nb * nb * es + 16 * ndof       # block inverse + r in + z out
        kernels[f"ejacobi_solve_{name}"] = {"us": t_sol * 1e6, "alg_bytes": sb, "GBs": sb / t_sol / 1e9}
        t_fac = time_kernel(lambda: disc.ejacobi_factor(Ustart, shift, prec, pc), reps=5, warm=1)
        kernels[f"ejacobi_factor_{name}(assemble+invert)"] = {
            "us": t_fac * 1e6, "inversion_TFLOPs": disc.nel * 2.0 * nb ** 3 / t_fac / 1e12}
        del pc
    out["extra"]["kernels"] = kernels
    dom = "ejacobi_solve_fp64"
    traffic = None
    tp = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tp):
        with open(tp) as fh:
            tj = json.load(fh)
        if tj.get("kernel") == dom and tj.get("workload") == workload \
                and tj.get("source_sha") == source_sha(tj["source"]):
            traffic = tj.get("bytes_per_launch")
    ach = kernels[dom]["GBs"]
    out["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom,
                       "alg_bytes_per_launch": kernels[dom]["alg_bytes"]}

    return out["extra"]["kernels"], out["roofline"]


def order_study(disc, U0, vortex):
    """Temporal order of ROW3, ESDIRK3 (PTC) and BDF2 (BDF1 start) on one mesh: every run
    goes from t = 0 to 10 (one period of the vortex), FP64 element-Jacobi.  E_exact is the
    rho L2 error against the exact vortex (it carries the spatial error); E_time is the rms
    rho difference to a ROW4 run at dt = 0.0125, i.e. the temporal error of the same
    spatial discretisation; the observed order is log2 of the ratio of E_time at dt and dt/2."""
    import math

    import torch

    from paper_1904_04825_amd import GmresOpts, SolverOpts
    T = 10.0
    lin = GmresOpts(m=20, rtol=1e-8)
    sopts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-8)

    def run(kind, dt):
        n = int(round(T / dt))
        tot = {"gmres_iters": 0, "ptc_iters": 0, "rejections": 0, "residual_evals": 0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind.startswith("ROW"):
            U = U0.clone()
            for _ in range(n):
                st = disc.row_step(U, int(kind[3]), dt, SolverOpts(lin=lin))
                if st["status"] != 0:
                    raise RuntimeError(f"row_step status {st['status']}")
                tot["gmres_iters"] += st["gmres_iters"]
                tot["residual_evals"] += st["residual_evals"]
        elif kind == "ESDIRK3":
            U = U0.clone()
            for _ in range(n):
                st = disc.esdirk_step(U, 3, dt, sopts)
                if st["status"] != 0:
                    raise RuntimeError(f"esdirk_step status {st['status']}")
                for k in tot:
                    tot[k] += st[k]
        else:
            Unm1, U = None, U0.clone()
            for _ in range(n):
                Unp1, st = disc.bdf2_step(Unm1, U, dt, sopts)
                if st["status"] != 0:
                    raise RuntimeError(f"bdf2_step status {st['status']}")
                for k in tot:
                    tot[k] += st[k]
                Unm1, U = U, Unp1
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        rec = {"dt": dt, "steps": n, "wall_s_per_time_unit": wall / T, "l2_err_rho_exact":
               disc.l2_error_vortex(U, 0, T, vortex), **{k: v / n for k, v in tot.items() if k != "rejections"},
               "rejections": tot["rejections"]}
        print(f"# {kind} dt={dt}: {n} steps in {wall:.1f} s", flush=True)
        return U, rec

    Uref, ref = run("ROW4", 0.0125)
    res = {"reference": {"scheme": "ROW4", **ref}}
    for kind in ("ROW3", "ESDIRK3", "BDF2"):
        rows = []
        for dt in (0.2, 0.1, 0.05):
            U, rec = run(kind, dt)
            rec["e_time_rho"] = float(torch.linalg.norm(U[0] - Uref[0]) / math.sqrt(U[0].numel()))
            if rows:
                rec["order"] = math.log2(rows[-1]["e_time_rho"] / rec["e_time_rho"])
            rows.append(rec)
        res[kind] = rows
    return res


def paper_vortex_study(select, speed, eps_mode="abs", pc_prec="f64", verbose=True):
    """The paper's own vortex study (Section 5.1): 50x50 uniform quads on [-10,10]^2, P6,
    Roe flux, GMRES(60) with the literal eps = 1e-8, FP64 element-Jacobi, one period
    (T = 20) at the table's step counts and tolerances; E(rho) and E(u) against the exact
    vortex beside the values the paper prints (tests/golden/paper_vortex_tables.json)."""
    import torch

    import fr_inputs as fi
    from paper_1904_04825_amd import EPS_ABS, EPS_RMS, F32, F64, Disc, GmresOpts, SolverOpts
    em = EPS_ABS if eps_mode == "abs" else EPS_RMS
    pp = F32 if pc_prec == "f32" else F64
    with open(os.path.join(ROOT, "tests", "golden", "paper_vortex_tables.json")) as fh:
        golden = json.load(fh)
    T = golden["workload"]["period"]
    vx = fi.paper_vortex(speed=speed)
    disc = Disc(fi.workload_nodes("vortex50_p6_paper"), 6, flux="roe")
    xy = disc.solution_points().cpu().numpy()
    U0 = torch.as_tensor(vx.conservative(xy[0], xy[1], 0.0), device=disc.device).contiguous()
    rows = []
    for ent in golden["entries"]:
        key = f"{ent['scheme']}/{ent['steps']}"
        if select != "all" and key not in select:
            continue
        sch, n = ent["scheme"], ent["steps"]
        dt = T / n
        U = U0.clone()
        tot = {"gmres_iters": 0, "ptc_iters": 0, "rejections": 0, "residual_evals": 0}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status = 0
        if sch.startswith("ROW"):
            o = SolverOpts(lin=GmresOpts(m=60, rtol=ent["tol_lin"], eps_mode=em), precond_precision=pp)
            for _ in range(n):
                st = disc.row_step(U, int(sch[3]), dt, o)
                status = status or st["status"]
                tot["gmres_iters"] += st["gmres_iters"]
                tot["residual_evals"] += st["residual_evals"]
        else:
            o = SolverOpts(lin=GmresOpts(m=60, rtol=ent["tol_lin"], eps_mode=em), tol_nl=ent["tol_nl"],
                           precond_precision=pp)
            Um1 = None
            for _ in range(n):
                if sch.startswith("ESDIRK"):
                    st = disc.esdirk_step(U, int(sch[6]), dt, o)
                else:
                    Un, st = disc.bdf2_step(Um1, U, dt, o)
                    Um1, U = U, Un
                status = status or st["status"]
                for k in tot:
                    tot[k] += st[k]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        e_rho = disc.l2_error_vortex(U, 0, T, vx)
        e_u = disc.l2_error_vortex(U, 1, T, vx)
        row = {"scheme": sch, "steps": n, "dt": dt, "tol_lin": ent["tol_lin"], "tol_nl": ent.get("tol_nl"),
               "status": status, "e_rho": e_rho, "e_rho_paper": ent["e_rho"], "ratio_rho": e_rho / ent["e_rho"],
               "e_u": e_u, "e_u_paper": ent["e_u"], "wall_s": wall, "wall_s_per_time_unit": wall / T,
               **{k: v / n for k, v in tot.items() if k != "rejections"}, "rejections": tot["rejections"]}
        if ent.get("note"):
            row["paper_scheme"] = ent["note"]
        rows.append(row)
        if verbose:
            print(f"# {sch} T/{n}: E(rho) {e_rho:.4e} (paper {ent['e_rho']:.4e}, ratio {e_rho / ent['e_rho']:.3f}), "
                  f"E(u) {e_u:.4e} (paper {ent['e_u']:.4e}), {wall:.1f} s", flush=True)
    return {"mode": "paper-vortex", "mach_reading": speed, "eps_mode": eps_mode, "precond_precision": pc_prec,
            "workload": golden["workload"], "rows": rows}


def cylinder_study(schemes, dts, t_dev, t_run, dt_ref, pc_prec="f32", tol_nl=1e-6, tol_lin_row=1e-6, dev_dt=0.01,
                   save=None, load=None, dev_tol=1e-3, ref_save=None, ref_load=None, settle_t=0.0, verbose=True):
    """The cylinder case's scheme comparison (Section 5.2) on a self-generated O-grid (the
    paper's 5,690-element mesh is not available): 120 x 48 P3 quads, first layer 0.0033,
    far field at radius 100; Re = 1200, M = 0.1, BR2, Roe, element-Jacobi.  From an
    impulsive start (with a small cross-stream bump that breaks the symmetry) the flow is
    developed for t_dev time units by ESDIRK3 at dev_dt with stage solves to dev_tol (ROW steps
    fail on the impulsive start's acoustic transient at these step sizes), then for settle_t
    more by ESDIRK4 at dt 0.01 with the study's tolerance (the state can be saved and loaded
    so that the study itself runs separately);
    from there every scheme runs t_run time units at each dt with the paper's tolerances
    (ROW: linear 1e-6; ESDIRK and BDF2: nonlinear 1e-6, linear 1e-1) and pseudo-time
    settings (dtau_init = 0.01, dtau_max = 1); a ROW stage whose GMRES(20) reaches the cap of
    1000 iterations commits what it has, and a run fails when a step fails or C_d stops
    being finite; Error(C_d) is the paper's root mean square
    of the drag-coefficient differences over the run's steps, against an ESDIRK4 run at
    dt_ref (in place of the paper's explicit SSPRK3 reference)."""
    import math

    import numpy as np
    import torch

    import fr_inputs as fi
    from paper_1904_04825_amd import F32, F64, Disc, GmresOpts, SolverOpts
    pp = F32 if pc_prec == "f32" else F64
    cyl = fi.Cylinder()
    disc = Disc(fi.workload_nodes("cylinder120x48_p3"), 3, physics="ns", flux="roe", mu=cyl.mu,
                prandtl=cyl.prandtl, viscous="br2", bc_south="wall", bc_north="farfield", q_far=cyl.far_state())
    xy = disc.solution_points().cpu().numpy()
    U0 = torch.as_tensor(cyl.conservative(xy[0], xy[1], perturb=0.05), device=disc.device).contiguous()
    qinf = 0.5 * cyl.speed ** 2         # rho u^2 / 2 with rho = 1, D = 1

    def cd(U):
        return disc.wall_force(U)[0] / qinf

    def run(sch, dt, nsteps, U, record, dev=False):
        """nsteps of scheme sch from U (in place); per-step totals and the C_d history.  dev:
        the development run (nonlinear tolerance dev_tol; the state is saved every 50 steps
        when save names a file)."""
        tot = {"gmres_iters": 0, "ptc_iters": 0, "rejections": 0, "residual_evals": 0, "failed_steps": 0,
               "unconverged": 0}
        hist = []
        lin_row = GmresOpts(m=20, rtol=tol_lin_row)
        # a ROW stage whose GMRES reaches its iteration cap (50 m) short of the tolerance still
        # commits its increment: the step fails only when the state stops being finite
        o_row = SolverOpts(lin=lin_row, precond_precision=pp, commit_unconverged=1)
        o_imp = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=dev_tol if dev else tol_nl, dtau_init=0.01,
                           dtau_max=1.0, precond_precision=pp)
        Um1 = None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(nsteps):
            if (it + 1) % 10 == 0:
                progress(f"cylinder: {sch} dt={dt} step {it + 1}/{nsteps}")
            if sch.startswith("ROW"):
                st = disc.row_step(U, int(sch[3]), dt, o_row)
            elif sch.startswith("ESDIRK"):
                st = disc.esdirk_step(U, int(sch[6]), dt, o_imp)
            else:
                Un, st = disc.bdf2_step(Um1, U, dt, o_imp)
                Um1 = U.clone()
                U.copy_(Un)
            if st["status"] != 0 and not (sch.startswith("ROW") and st["status"] == 1):
                tot["failed_steps"] += 1
                tot["fail_status"] = st["status"]
                break
            if dev and save is not None and (it + 1) % 50 == 0:
                np.save(save, U.cpu().numpy())
            for k in ("gmres_iters", "ptc_iters", "rejections", "residual_evals", "unconverged"):
                tot[k] += st.get(k, 0)
            if record:
                c = cd(U)
                if not math.isfinite(c):
                    tot["failed_steps"] += 1
                    break
                hist.append(c)
        torch.cuda.synchronize()
        return tot, hist, time.perf_counter() - t0

    U = U0.clone()
    if load is not None:
        U.copy_(torch.as_tensor(np.load(load), device=disc.device).reshape(U.shape))
        dev_tot, dev_s = {"rejections": 0, "failed_steps": 0}, 0.0
        progress(f"cylinder: developed state loaded from {load}")
    else:
        progress("cylinder: development run")
        dev_tot, _, dev_s = run("ESDIRK3", dev_dt, int(round(t_dev / dev_dt)), U, False, dev=True)
        if save is not None:
            np.save(save, U.cpu().numpy())
    settle_s = 0.0
    if settle_t > 0:
        # damp the acoustic content that the loosely converged development leaves behind
        progress(f"cylinder: settling for {settle_t} by ESDIRK4 at dt 0.01, tol_nl {tol_nl}")
        stot, _, settle_s = run("ESDIRK4", 0.01, int(round(settle_t / 0.01)), U, False)
        if stot["failed_steps"]:
            raise SystemExit("cylinder: the settling run failed")
        if save is not None:
            np.save(save, U.cpu().numpy())
    progress(f"cylinder: developed to t = {t_dev + settle_t}, C_d = {cd(U):.4f}")
    Ustart = U.clone()
    nref = int(round(t_run / dt_ref))
    if ref_load is not None:
        with open(ref_load) as f:
            ref = json.load(f)
        if ref["dt_ref"] != dt_ref or ref["steps"] != nref:
            raise SystemExit(f"{ref_load} holds a reference at dt {ref['dt_ref']} over {ref['steps']} steps")
        ref_hist, ref_s = ref["cd"], ref["wall_s"]
        progress(f"cylinder: reference loaded from {ref_load}")
    else:
        progress("cylinder: reference run")
        Ur = Ustart.clone()
        ref_tot, ref_hist, ref_s = run("ESDIRK4", dt_ref, nref, Ur, True)
        if ref_tot["failed_steps"]:
            raise SystemExit("cylinder: the reference run failed")
        if ref_save is not None:
            with open(ref_save, "w") as f:
                json.dump({"dt_ref": dt_ref, "steps": nref, "wall_s": ref_s, "cd": ref_hist, "totals": ref_tot}, f)
    rows = []
    for sch in schemes:
        for dt in dts:
            n = int(round(t_run / dt))
            stride = int(round(dt / dt_ref))
            Uc = Ustart.clone()
            tot, hist, wall = run(sch, dt, n, Uc, True)
            ok = tot["failed_steps"] == 0 and len(hist) == n
            dif = np.array([hist[i] - ref_hist[(i + 1) * stride - 1] for i in range(n)]) if ok else None
            err = float(np.sqrt(np.mean(dif ** 2))) if ok else None
            row = {"scheme": sch, "dt": dt, "steps": n, "completed": len(hist), "error_cd": err, "wall_s": wall,
                   "error_cd_max": float(np.abs(dif).max()) if ok else None,
                   "error_cd_first_tenth": float(np.sqrt(np.mean(dif[:max(n // 10, 1)] ** 2))) if ok else None,
                   "cd_end": hist[-1] if hist else None,
                   **{k: v / max(len(hist), 1) for k, v in tot.items()
                      if k not in ("rejections", "failed_steps", "unconverged", "fail_status")},
                   "fail_status": tot.get("fail_status"),
                   "rejections": tot["rejections"], "unconverged_solves": tot["unconverged"], "failed": not ok}
            rows.append(row)
            if verbose:
                print(f"# {sch} dt={dt}: Error(Cd) {err if err is None else f'{err:.3e}'}, {wall:.2f} s, "
                      f"GMRES/step {row['gmres_iters']:.1f}, PTC/step {row['ptc_iters']:.1f}, "
                      f"rejections {tot['rejections']}, unconverged solves {tot['unconverged']}"
                      f"{' FAILED at step %d' % (len(hist) + 1) if not ok else ''}", flush=True)
    return {"mode": "cylinder", "mesh": "O-grid 120x48, P3 (5760 elements, 368,640 DOFs)", "reynolds": cyl.reynolds,
            "mach": cyl.mach, "viscous": "BR2", "precond_precision": pc_prec, "tol_nl": tol_nl,
            "tol_lin_row": tol_lin_row,
            "development": {"scheme": f"ESDIRK3 at dt {dev_dt}, tol_nl {dev_tol}", "loaded_from": load,
                            "settle": {"scheme": "ESDIRK4 at dt 0.01", "t": settle_t, "wall_s": settle_s},
                            "t": t_dev, "wall_s": dev_s, "rejections": dev_tot["rejections"],
                            "failed_steps": dev_tot["failed_steps"]},
            "reference": {"scheme": "ESDIRK4", "dt": dt_ref, "steps": nref, "wall_s": ref_s, "loaded_from": ref_load,
                          "cd_start": ref_hist[0] if ref_hist else None, "cd_end": ref_hist[-1] if ref_hist else None},
            "rows": rows}


def tgv_study(n_el, P, steps, dt_tc, sample_every, verbose=True):
    """The Taylor-Green vortex of Section 5.3 on n_el^3 uniform P hexahedra (the paper's
    mesh is 64^3 P3: 83.9M DOFs), Re 1600, Ma 0.1, BR2, Roe.  Times the 3D residual with
    HIP events (DOF-residuals/s, and algorithmic bytes per second: the state in and the
    residual out, plus the face traces and raw face gradients the first kernel writes and
    the second reads), then runs `steps` SSPRK3 steps of dt_tc t_c (the paper's explicit
    reference integrator) from t = 0 with E_k, eps1 and eps3 every sample_every steps."""
    import math

    import torch

    import fr_inputs as fi
    from paper_1904_04825_amd import Disc3D
    tg = fi.TaylorGreen()
    L = tg.L
    disc = Disc3D(n_el, n_el, n_el, P, (-math.pi * L,) * 3, (2 * math.pi * L,) * 3, flux="roe", mu=tg.mu,
                  prandtl=tg.prandtl, gamma=tg.gamma, rgas=tg.rgas)
    xyz = disc.solution_points()
    U = torch.as_tensor(tg.conservative(xyz[0], xyz[1], xyz[2]), device=disc.device).reshape(disc.shape).contiguous()
    R = disc.empty()
    progress("tgv: residual timing")
    for _ in range(3):
        disc.residual(U, R)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 20
    e0.record(s)
    for _ in range(reps):
        disc.residual(U, R)
    e1.record(s)
    e1.synchronize()
    t_res = e0.elapsed_time(e1) / 1e3 / reps
    n2 = (P + 1) ** 2
    face = disc.nel * 6 * 5 * n2 * 8
    alg = 2 * 8 * disc.ndof + 2 * 4 * face          # state in, R out; traces and gradients (x, y, z) written and read
    tc = L / tg.V0
    dt = dt_tc * tc
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps + 1):
        if it % sample_every == 0:
            ek, e1_, e3 = disc.dissipation(U, tg.rho0)
            hist.append({"t_tc": it * dt_tc, "E_k": ek, "eps1": e1_, "eps3": e3})
            if verbose:
                print(f"# t/t_c {it * dt_tc:.4f}: E_k {ek:.6e}, eps1 {e1_:.6e}, eps3 {e3:.3e}", flush=True)
        if it < steps:
            disc.ssprk3_step(U, dt)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"mode": "tgv", "mesh": f"{n_el}^3 hexahedra, P{P}", "ndof": disc.ndof, "reynolds": 1600, "mach": 0.1,
            "viscous": "BR2", "flux": "Roe",
            "residual": {"us": t_res * 1e6, "dof_res_per_s": disc.ndof / t_res, "alg_bytes": alg,
                         "GBs": alg / t_res / 1e9},
            "ssprk3": {"dt_tc": dt_tc, "steps": steps, "wall_s": wall,
                       "ms_per_step": 1e3 * wall / max(steps, 1)},
            "history": hist}


def tgv_implicit_study(n_el, P, schemes, per_tc, t0, t1, dt_ref_tc, ref_save=None, ref_load=None, pc_prec="f64",
                       verbose=True):
    """The implicit schemes on the Taylor-Green vortex (Section 5.3) on n_el^3 P hexahedra:
    the reference is SSPRK3 at dt_ref_tc t_c from t = 0 (the paper's 2e-4 t_c), which also
    gives the state at t0; each scheme then runs from t0 to t1 at dt = t_c / k and
    Error(eps) is the paper's root mean square over its steps of eps - eps_ref, eps = eps1 +
    eps3 (eps2 = 0).  Tolerances as the paper's: ROW linear 1e-6; ESDIRK and BDF2 nonlinear
    1e-6 with linear 1e-1, dtau_init = dt, dtau_max = 1e20; GMRES(30), element-Jacobi in
    pc_prec ("f64", or "f32": blocks rounded to FP32, inverted and applied in FP32)."""
    import math

    import numpy as np
    import torch

    import fr_inputs as fi
    from paper_1904_04825_amd import F32, F64, Disc3D, GmresOpts, SolverOpts
    pp = F32 if pc_prec == "f32" else F64
    tg = fi.TaylorGreen()
    L = tg.L
    tc = L / tg.V0
    disc = Disc3D(n_el, n_el, n_el, P, (-math.pi * L,) * 3, (2 * math.pi * L,) * 3, flux="roe", mu=tg.mu,
                  prandtl=tg.prandtl, gamma=tg.gamma, rgas=tg.rgas)
    kmax = max(per_tc)
    stride = int(round(1.0 / (kmax * dt_ref_tc)))        # reference steps per finest implicit step
    if abs(stride * kmax * dt_ref_tc - 1.0) > 1e-9 or any(kmax % k for k in per_tc):
        raise SystemExit("tgv-implicit: every t_c / k must be a whole number of reference steps of the finest")

    def eps_of(U):
        _, e1, e3 = disc.dissipation(U, tg.rho0)
        return e1 + e3

    if ref_load is not None:
        z = np.load(ref_load)
        U0 = torch.as_tensor(z["U0"], device=disc.device).reshape(disc.shape).contiguous()
        ref_eps, ref_s = z["eps"], float(z["wall_s"])
        progress(f"tgv-implicit: reference loaded from {ref_load}")
    else:
        xyz = disc.solution_points()
        U = torch.as_tensor(tg.conservative(xyz[0], xyz[1], xyz[2]), device=disc.device).reshape(
            disc.shape).contiguous()
        n0 = int(round(t0 / dt_ref_tc))
        n1 = int(round(t1 / dt_ref_tc))
        ref_eps = []
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        U0 = None
        for it in range(n1 + 1):
            if it == n0:
                U0 = U.clone()
            if it >= n0 and (it - n0) % stride == 0:
                ref_eps.append(eps_of(U))
            if it % 5000 == 0:
                progress(f"tgv-implicit: reference step {it}/{n1}")
            if it < n1:
                disc.ssprk3_step(U, dt_ref_tc * tc)
        torch.cuda.synchronize()
        ref_s = time.perf_counter() - w0
        ref_eps = np.array(ref_eps)
        if ref_save is not None:
            np.savez(ref_save, U0=U0.cpu().numpy(), eps=ref_eps, wall_s=ref_s)
    rows = []
    for sch in schemes:
        for k in per_tc:
            dt = tc / k
            n = int(round((t1 - t0) * k))
            o = SolverOpts(lin=GmresOpts(m=30, rtol=1e-6), precond_precision=pp) if sch.startswith("ROW") else \
                SolverOpts(lin=GmresOpts(m=30, rtol=1e-1), tol_nl=1e-6, dtau_init=0.0, dtau_max=1e20,
                           precond_precision=pp)
            U = U0.clone()
            Um1 = None
            tot = {"gmres_iters": 0, "ptc_iters": 0, "rejections": 0, "residual_evals": 0}
            eps = []
            failed = None
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            for it in range(n):
                if sch.startswith("ROW"):
                    st = disc.row_step(U, int(sch[3]), dt, o)
                elif sch.startswith("ESDIRK"):
                    st = disc.esdirk_step(U, int(sch[6]), dt, o)
                else:
                    Un, st = disc.bdf2_step(Um1, U, dt, o)
                    Um1 = U.clone()
                    U.copy_(Un)
                if st["status"] != 0:
                    failed = st["status"]
                    break
                for key in tot:
                    tot[key] += st[key]
                eps.append(eps_of(U))
                if (it + 1) % 10 == 0:
                    progress(f"tgv-implicit: {sch} t_c/{k} step {it + 1}/{n}")
            torch.cuda.synchronize()
            wall = time.perf_counter() - w0
            err = None
            if failed is None:
                r = ref_eps[[(i + 1) * (kmax // k) for i in range(n)]]
                err = float(np.sqrt(np.mean((np.array(eps) - r) ** 2)))
            row = {"scheme": sch, "dt_tc": 1.0 / k, "steps": n, "error_eps": err, "wall_s": wall,
                   "fail_status": failed, **{key: v / max(len(eps), 1) for key, v in tot.items()},
                   "eps_end": eps[-1] if eps else None}
            rows.append(row)
            if verbose:
                print(f"# {sch} dt=t_c/{k}: Error(eps) {err if err is None else f'{err:.3e}'}, {wall:.1f} s, "
                      f"GMRES/step {row['gmres_iters']:.1f}, PTC/step {row['ptc_iters']:.1f}, "
                      f"rejections {tot['rejections']}{'' if failed is None else f' FAILED ({failed})'}", flush=True)
    return {"mode": "tgv-implicit", "mesh": f"{n_el}^3 hexahedra, P{P}", "ndof": disc.ndof, "reynolds": 1600,
            "precond_precision": pc_prec,
            "mach": 0.1, "window_tc": [t0, t1], "reference": {"scheme": "SSPRK3", "dt_tc": dt_ref_tc, "wall_s": ref_s,
                                                               "loaded_from": ref_load,
                                                               "eps_t0": float(ref_eps[0]),
                                                               "eps_t1": float(ref_eps[-1])},
            "rows": rows}


def precond_study(disc, W, U, dt, scheme, lin):
    """The first ROW stage's linear system at the timed legs' start state, solved to the
    same tolerance with each preconditioner on FP32 blocks: element-Jacobi (the paper's),
    LU-SGS and p-multigrid (coarse level P - 2, one pre-, one post- and one coarse sweep):
    GMRES iterations, Jacobian-free products and wall time of the factor + solve."""
    import torch
    from paper_1904_04825_amd import F32, PC_EJACOBI, PC_LUSGS, PC_PMG, GmresOpts, Pmg
    from paper_1904_04825_amd.api import scheme_table
    gam = scheme_table(0, scheme)[3]
    shift = 1.0 / (gam * dt)
    R0 = disc.residual(U)
    res = {}
    kinds = [("element-Jacobi", PC_EJACOBI), ("LU-SGS", PC_LUSGS)]
    if disc.p >= 4:
        kinds.append((f"p-multigrid P{disc.p}->P{disc.p - 2}", PC_PMG))
    mg = Pmg(disc, disc.p - 2, 1, 1, 1, F32) if disc.p >= 4 else None
    for name, pck in kinds:
        for rep in range(2):   # the second run is timed
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pc = disc.pmg_factor(U, shift, mg, F32) if pck == PC_PMG else disc.ejacobi_factor(U, shift, F32)
            x, st = disc.gmres_solve(pc, U, R0, shift, R0, opts=GmresOpts(m=lin.m, rtol=lin.rtol, precond=pck))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            del pc
        res[name] = {"gmres_iters": st["iters"], "jf_products": st["residual_evals"], "status": st["status"],
                     "wall_s": wall}
    return {"system": f"ROW{scheme} stage 1 at the legs' start, FGMRES({lin.m}) rtol {lin.rtol}, FP32 blocks",
            **res}


def run_leg(disc, U, steps, scheme, dt, opts, allow_unconverged=False):
    import torch
    evals = iters = 0
    extra = {"warm_used": 0, "warm_rejected": 0, "unconverged_solves": 0}
    opts.commit_unconverged = 1 if allow_unconverged else 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        st = disc.row_step(U, scheme, dt, opts)
        if st["status"] != 0 and not (allow_unconverged and st["status"] == 1):
            raise RuntimeError(f"row_step status {st['status']}")
        extra["unconverged_solves"] += st["unconverged"]
        evals += st["residual_evals"]
        iters += st["gmres_iters"]
        extra["warm_used"] += st["warm_used"]
        extra["warm_rejected"] += st["warm_rejected"]
    torch.cuda.synchronize()
    return time.perf_counter() - t0, evals, iters, extra


def main():
    args = parse()
    if args.cpu_sample is not None:
        cpu_sample(json.loads(args.cpu_sample))
        return
    if args.paper_vortex is not None:
        sel = "all" if args.paper_vortex == "all" else set(args.paper_vortex.split(","))
        print(json.dumps(paper_vortex_study(sel, args.mach_reading, args.study_eps, args.study_precond)), flush=True)
        return
    if args.tgv:
        print(json.dumps(tgv_study(args.tgv_n, args.tgv_p, args.tgv_steps, args.tgv_dt, args.tgv_sample)), flush=True)
        return
    if args.tgv_implicit:
        print(json.dumps(tgv_implicit_study(args.tgvi_n, args.tgv_p, args.tgvi_schemes.split(","),
                                            [int(k) for k in args.tgvi_steps_per_tc.split(",")], args.tgvi_t0,
                                            args.tgvi_t1, args.tgv_dt, args.tgvi_ref_save, args.tgvi_ref_load,
                                            args.study_precond)),
              flush=True)
        return
    if args.cylinder:
        print(json.dumps(cylinder_study(args.cyl_schemes.split(","), [float(x) for x in args.cyl_dts.split(",")],
                                        args.cyl_tdev, args.cyl_trun, args.cyl_dtref, args.study_precond,
                                        args.cyl_tolnl, args.cyl_tollin, args.cyl_devdt, args.cyl_save,
                                        args.cyl_load, args.cyl_devtol, args.cyl_ref_save,
                                        args.cyl_ref_load, args.cyl_settle)), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU: --gpus must be 1 (the sharding over several GPUs is a design, not a run)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import fr_inputs as fi
    from paper_1904_04825_amd import (F32, F64, PC_LUSGS, Disc, GmresOpts, MlpTrainer, SolverOpts, StageLog,
                                      StageLogs, WarmStart, fit_group)
    from paper_1904_04825_amd.api import scheme_table

    W = WORKLOADS[args.workload]
    dt = args.dt if args.dt is not None else W["dt"]
    scheme = W["scheme"]
    nstage = {2: 3, 3: 4, 4: 6}[scheme]
    dev = torch.device("cuda:0")
    nodes = fi.workload_nodes(W["nodes"])
    if W["physics"] == "ns":
        sl = fi.ShearLayer()
        disc = Disc(nodes, W["p"], physics="ns", mu=sl.mu, prandtl=sl.prandtl, device=dev)
        fn = lambda x, y: sl.conservative(x, y)  # noqa: E731
        vortex = None
    else:
        disc = Disc(nodes, W["p"], device=dev)
        vortex = fi.Vortex()
        fn = lambda x, y: vortex.conservative(x, y, 0.0)  # noqa: E731
    xy = disc.solution_points().cpu().numpy()
    U0_np = fn(xy[0], xy[1])
    U0 = torch.as_tensor(U0_np, device=dev).contiguous()
    ndof = disc.ndof
    lin = GmresOpts(m=20, rtol=1e-8)
    out = {"metric": "DOF-residuals/s", "unit": "DOF-residuals/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": f"{W['label']}; ROW{scheme} dt={dt}, FGMRES(20) rtol 1e-8, element-Jacobi FP64, "
                                  f"Rusanov, eps_rms 1e-8; timed steps start after {args.warmup} untimed steps",
                      "ndof": ndof, "dt": dt},
           "extra": {}}

    if args.order_study:
        if args.workload != "vortex64_p3":
            raise SystemExit("--order-study runs on the 64x64 P3 vortex")
        print(json.dumps({"mode": "order-study", "workload": W["label"],
                          "study": order_study(disc, U0, vortex)}), flush=True)
        return

    if args.kernels_only:
        kernels, roof = kernel_block(disc, U0, dt, scheme, ndof, args.workload)
        res = {"mode": "kernels-only", "config": out["config"], "kernels": kernels, "roofline": roof}
        if args.calib_copy:
            res["calib_copy_bytes"] = calib_copy(dev)
        print(json.dumps(res), flush=True)
        return

    progress("warm-up / logging steps")
    # ---- (1) warm-up steps, logging the stage solves
    rng = np.random.default_rng(40)
    learned = not args.no_learned
    per_stage = min(args.log_elems, disc.nel)
    logs = StageLogs([StageLog(disc, max(args.warmup, 1) * per_stage, rng.choice(disc.nel, per_stage, replace=False))
                      for _ in range(nstage)]) if learned else None
    yhist = torch.zeros((2, ndof), dtype=torch.float64, device=dev)
    U = U0.clone()
    t_w = time.perf_counter()
    for _ in range(args.warmup):
        if logs is not None:
            for lg in logs.logs:
                lg.set_elems(rng.choice(disc.nel, per_stage, replace=False))
        st = disc.row_step(U, scheme, dt, SolverOpts(lin=lin, log=logs, yhist=yhist, precond_precision=F32,
                                                     commit_unconverged=int(args.allow_unconverged)))
        if st["status"] != 0 and not (args.allow_unconverged and st["status"] == 1):
            raise RuntimeError(f"warm-up row_step status {st['status']}")
    torch.cuda.synchronize()
    out["extra"]["warmup_s"] = time.perf_counter() - t_w
    t_start = args.warmup * dt
    Ustart, hstart = U.clone(), yhist.clone()

    progress("training")
    # ---- (2) train one network per stage on the GPU
    def train(stage_logs, seed0):
        """One network per stage, all trained together on the GPU (fr_mlp_train_group: one
        launch per kernel for every network, cosine-decayed Adam), each from its stage's log.
        For reference, one more network is then trained alone through the per-step call
        (MlpTrainer.fit, the same arithmetic) and timed."""
        t_tr = time.perf_counter()
        trainers = []
        for i, lg in enumerate(stage_logs.logs):
            tr = MlpTrainer(disc, n_hidden=256, seed=seed0 + i, lr=1e-3)
            tr.fit_stats(lg)
            trainers.append(tr)
        final_loss = []
        for g0 in range(0, len(trainers), 8):
            ls = fit_group(trainers[g0:g0 + 8], stage_logs.logs[g0:g0 + 8], args.adam_steps, args.batch, lr=1e-3,
                           seeds=[seed0 + 100 + i for i in range(g0, min(g0 + 8, len(trainers)))], report_every=250)
            final_loss += [float(l[-1][1]) for l in ls]
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t_tr
        t_ref = time.perf_counter()
        ref = MlpTrainer(disc, n_hidden=256, seed=seed0, lr=1e-3)
        ref.fit_stats(stage_logs.logs[0])
        ref.fit(stage_logs.logs[0], args.adam_steps, args.batch, lr=1e-3, seed=seed0 + 100, report_every=250)
        torch.cuda.synchronize()
        ref_s = time.perf_counter() - t_ref
        del ref
        n = len(trainers)
        info = {"samples_per_stage": stage_logs.logs[0].count, "adam_steps_per_stage": args.adam_steps,
                "batch": args.batch, "networks": n, "final_mse_normalised": final_loss, "train_s": train_s,
                "train_s_per_network": train_s / n, "single_network_fit_s": ref_s,
                "note": "the networks are trained together (one launch per kernel for all of them); "
                        "single_network_fit_s is one network trained alone through the per-step call"}
        return WarmStart([t.net for t in trainers]), info

    warm = None
    if learned and args.warmup > 0:
        warm, out["extra"]["learned_training"] = train(logs, 4)

    progress("timed legs")
    # ---- (3) timed legs from the same state
    t_phys = args.steps * dt

    def err(Ux):
        return disc.l2_error_vortex(Ux, 0, t_start + t_phys, vortex) if vortex is not None else None

    U = Ustart.clone()
    wall, evals, iters, x1 = run_leg(disc, U, args.steps, scheme, dt, SolverOpts(lin=lin, yhist=hstart.clone()),
                                     args.allow_unconverged)
    U_fp64 = U
    out["value"] = ndof * evals / wall
    out["ms_per_step"] = wall / args.steps * 1e3
    out["extra"].update({"wall_s_per_time_unit": wall / t_phys, "gmres_iters_per_step": iters / args.steps,
                         "residual_evals_per_step": evals / args.steps, "l2_err_rho": err(U_fp64),
                         "t_start": t_start, "t_end": t_start + t_phys,
                         "unconverged_solves": x1["unconverged_solves"]})
    legs = {}
    if not args.no_fp32_leg:
        U = Ustart.clone()
        w2, e2, i2, _ = run_leg(disc, U, args.steps, scheme, dt,
                                SolverOpts(lin=lin, precond_precision=F32, yhist=hstart.clone()), args.allow_unconverged)
        legs["fp32_precond"] = {"wall_s_per_time_unit": w2 / t_phys, "ms_per_step": w2 / args.steps * 1e3,
                                "gmres_iters_per_step": i2 / args.steps, "l2_err_rho": err(U),
                                "rel_diff_vs_fp64": float(torch.linalg.norm(U - U_fp64) / torch.linalg.norm(U_fp64))}
        if warm is not None:
            U = Ustart.clone()
            w3, e3, i3, x3 = run_leg(disc, U, args.steps, scheme, dt,
                                     SolverOpts(lin=lin, precond_precision=F32, warm=warm, yhist=hstart.clone()))
            legs["fp32_precond_learned"] = {
                "wall_s_per_time_unit": w3 / t_phys, "ms_per_step": w3 / args.steps * 1e3,
                "gmres_iters_per_step": i3 / args.steps, "l2_err_rho": err(U), **x3,
                "rel_diff_vs_fp64": float(torch.linalg.norm(U - U_fp64) / torch.linalg.norm(U_fp64)),
                "speedup_vs_plain_fp64": wall / w3}
            # cost of the learned part: the logging warm-up and the training, against the
            # time it saves per step (over the FP32 leg, and over the plain FP64 leg)
            tr_s = out["extra"]["learned_training"]["train_s"]
            save32 = (w2 - w3) / args.steps
            save64 = (wall - w3) / args.steps
            legs["fp32_precond_learned"]["cost"] = {
                "logging_warmup_s": out["extra"]["warmup_s"], "train_s": tr_s,
                "saved_s_per_step_vs_fp32": save32, "saved_s_per_step_vs_fp64": save64,
                "break_even_steps_vs_fp32": (tr_s / save32) if save32 > 0 else None,
                "break_even_steps_vs_fp64": (tr_s / save64) if save64 > 0 else None,
                "note": "the logging steps are ordinary time steps of the run (FP32 element-Jacobi) that also "
                        "store training samples; training is the extra cost"}
        # the same steps with the matrix-free LU-SGS preconditioner on the FP32 blocks
        # (Section 4.5 names it beside element-Jacobi), and with the learned start on top
        if W["physics"] == "euler" and disc.nx % 2 == 0 and disc.ny % 2 == 0:
            lin_l = GmresOpts(m=lin.m, rtol=lin.rtol, precond=PC_LUSGS)
            for name, wnet in (("fp32_lusgs", None), ("fp32_lusgs_learned", warm)):
                if name.endswith("learned") and wnet is None:
                    continue
                U = Ustart.clone()
                w4, e4, i4, x4 = run_leg(disc, U, args.steps, scheme, dt,
                                         SolverOpts(lin=lin_l, precond_precision=F32, warm=wnet, yhist=hstart.clone()))
                legs[name] = {"wall_s_per_time_unit": w4 / t_phys, "ms_per_step": w4 / args.steps * 1e3,
                              "gmres_iters_per_step": i4 / args.steps, "residual_evals_per_step": e4 / args.steps,
                              "l2_err_rho": err(U), "speedup_vs_plain_fp64": wall / w4,
                              "rel_diff_vs_fp64": float(torch.linalg.norm(U - U_fp64) / torch.linalg.norm(U_fp64)),
                              **({k: x4[k] for k in ("warm_used", "warm_rejected")} if wnet is not None else {})}
    out["extra"]["legs"] = legs
    if not args.no_fp32_leg and W["physics"] == "euler":
        progress("preconditioner study")
        out["extra"]["preconditioners"] = precond_study(disc, W, Ustart, dt, scheme, lin)

    # ---- (4) the other implicit schemes of the same workload, FP64 element-Jacobi:
    # ESDIRK3 (ESDIRK4 beside ROW4) and BDF2 (BDF1 start), each also with the FP32
    # element-Jacobi, with pseudo-transient continuation, inexact
    # Newton (GMRES rtol 1e-1 per PTC iteration), nonlinear tolerance 1e-8
    if args.schemes:
        sopts = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-8)
        schemes = {}

        def scheme_leg(step):
            tot = {"gmres_iters": 0, "ptc_iters": 0, "rejections": 0, "residual_evals": 0, "warm_used": 0,
                   "warm_rejected": 0}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Ux = step(tot)
            torch.cuda.synchronize()
            w = time.perf_counter() - t0
            return {"ms_per_step": w / args.steps * 1e3, "wall_s_per_time_unit": w / t_phys,
                    "gmres_iters_per_step": tot["gmres_iters"] / args.steps,
                    "ptc_iters_per_step": tot["ptc_iters"] / args.steps, "rejections": tot["rejections"],
                    "residual_evals_per_step": tot["residual_evals"] / args.steps, "l2_err_rho": err(Ux),
                    "learned_starts_used": tot["warm_used"], "learned_starts_rejected": tot["warm_rejected"]}

        def add(tot, st, name):
            if st["status"] != 0:
                raise RuntimeError(f"{name} status {st['status']}")
            for k in tot:
                tot[k] += st[k]

        ek = 4 if scheme == 4 else 3   # the ESDIRK of the same order as the ROW scheme (3 or 4)

        def esdirk(o, hist=None):
            def run(tot):
                Ux = Ustart.clone()
                if hist is not None:
                    o.yhist = hist.clone()
                for _ in range(args.steps):
                    add(tot, disc.esdirk_step(Ux, ek, dt, o), "esdirk_step")
                return Ux
            return run

        def bdf2(o, hist=None):
            def run(tot):
                Unm1, Un = None, Ustart.clone()
                if hist is not None:
                    o.yhist = hist.clone()
                for _ in range(args.steps):
                    Unp1, st = disc.bdf2_step(Unm1, Un, dt, o)
                    add(tot, st, "bdf2_step")
                    Unm1, Un = Un, Unp1
                return Un
            return run

        # the same PTC with the FP32 MFMA element-Jacobi (formed at every pseudo-iterate)
        sopts32 = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-8, precond_precision=F32)
        schemes[f"ESDIRK{ek}"] = scheme_leg(esdirk(sopts))
        schemes[f"ESDIRK{ek}, FP32 element-Jacobi"] = scheme_leg(esdirk(sopts32))
        schemes["BDF2 (BDF1 start)"] = scheme_leg(bdf2(sopts))
        schemes["BDF2 (BDF1 start), FP32 element-Jacobi"] = scheme_leg(bdf2(sopts32))
        if learned and args.warmup > 0:
            # learned PTC starts: a logging run of each scheme from t = 0 (FP32 element-Jacobi),
            # one network per implicit stage trained on it, then the timed leg from the same
            # state as the other legs
            n_imp = len(scheme_table(1, ek)[2]) - 1
            for name, nst, kind in ((f"ESDIRK{ek}", n_imp, "esdirk"), ("BDF2 (BDF1 start)", 1, "bdf2")):
                slogs = StageLogs([StageLog(disc, args.warmup * per_stage, rng.choice(disc.nel, per_stage,
                                                                                     replace=False))
                                   for _ in range(nst)])
                h = torch.zeros((2, ndof), dtype=torch.float64, device=dev)
                o_log = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-8, precond_precision=F32, log=slogs,
                                   yhist=h)
                Ux, Um1 = U0.clone(), None
                for _ in range(args.warmup):
                    for lg in slogs.logs:
                        lg.set_elems(rng.choice(disc.nel, per_stage, replace=False))
                    if kind == "esdirk":
                        st = disc.esdirk_step(Ux, ek, dt, o_log)
                    else:
                        Unew, st = disc.bdf2_step(Um1, Ux, dt, o_log)
                        Um1, Ux = Ux, Unew
                    if st["status"] != 0:
                        raise RuntimeError(f"{kind} logging step status {st['status']}")
                wnet, info = train(slogs, 20 if kind == "esdirk" else 40)
                o_w = SolverOpts(lin=GmresOpts(m=20, rtol=1e-1), tol_nl=1e-8, precond_precision=F32, warm=wnet)
                leg = scheme_leg(esdirk(o_w, h) if kind == "esdirk" else bdf2(o_w, h))
                leg["speedup_vs_plain_fp64"] = schemes[name]["ms_per_step"] / leg["ms_per_step"]
                leg["learned_training"] = {"samples_per_stage": info["samples_per_stage"],
                                           "final_mse_normalised": info["final_mse_normalised"]}
                schemes[f"{name}, FP32 element-Jacobi + learned start"] = leg
        out["extra"]["schemes"] = schemes

    progress("kernel timing block")
    if not args.no_kernels:
        kernels, roof = kernel_block(disc, Ustart, dt, scheme, ndof, args.workload)
        out["extra"]["kernels"] = kernels
        out["roofline"] = roof

    if args.calib_copy:
        out["extra"]["calib_copy_bytes"] = calib_copy(dev)

    progress("CPU baseline")
    if not args.no_cpu_baseline and W["physics"] == "euler":
        out["cpu_baseline"] = cpu_baseline(W, dt, scheme)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
