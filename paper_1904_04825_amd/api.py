"""Torch-facing binding of the frjf C ABI: argument checks and marshalling only.

Every computation runs in the HIP library; tensors supply device memory and
the current torch stream supplies the HIP stream.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

EULER, NS_BR1 = 0, 1
RUSANOV, ROE = 0, 1
F64, F32 = 0, 1
EPS_ABS, EPS_RMS = 0, 1
PC_EJACOBI, PC_LUSGS, PC_PMG = 0, 1, 2
_PHYS = {"euler": EULER, "ns": NS_BR1, "ns_br1": NS_BR1}
_FLUX = {"rusanov": RUSANOV, "roe": ROE}
BR1, BR2 = 0, 1
BC_PERIODIC, BC_WALL, BC_FARFIELD = 0, 1, 2
_VISC = {"br1": BR1, "br2": BR2}
_BC = {None: BC_PERIODIC, "periodic": BC_PERIODIC, "wall": BC_WALL, "farfield": BC_FARFIELD}
_PREC = {"f64": F64, "fp64": F64, "f32": F32, "fp32": F32}


class FrError(RuntimeError):
    def __init__(self, fn, status):
        msg = L.lib().fr_last_error().decode()
        super().__init__(f"{fn} -> {L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(fn, st, allow_numerical=False):
    if st < 0 or (st > 0 and not allow_numerical):
        raise FrError(fn, st)
    return st


@dataclass
class GmresOpts:
    m: int = 20
    max_iters: int = 0
    rtol: float = 1e-8
    ref_norm: float = 0.0
    eps: float = 1e-8
    eps_mode: int = EPS_RMS
    precond: int = PC_EJACOBI

    def c(self):
        return L.GmresOptsC(self.m, self.max_iters, self.rtol, self.ref_norm, self.eps, self.eps_mode, self.precond)


@dataclass
class SolverOpts:
    lin: GmresOpts = None
    tol_nl: float = 1e-8
    dtau_init: float = 0.0
    dtau_max: float = 1e20
    max_ptc: int = 0
    max_reject: int = 0
    precond_precision: int = F64
    commit_unconverged: int = 0
    warm: "WarmStart" = None          # learned starts, one network per (implicit) stage
    log: "StageLogs" = None           # log training samples after each (implicit) stage solve
    yhist: torch.Tensor = None        # (2, ndof) previous step's last two increments (in/out)

    def c(self):
        lin = self.lin or GmresOpts()
        o = L.SolverOptsC(lin.c(), self.tol_nl, self.dtau_init, self.dtau_max, self.max_ptc, self.max_reject,
                          self.precond_precision, self.commit_unconverged)
        if self.warm is not None:
            o.warm = ctypes.cast(self.warm.array, ctypes.c_void_p)
            o.d_mlp_work = self.warm.work.data_ptr()
        if self.log is not None:
            o.log = ctypes.cast(self.log.array, ctypes.c_void_p)
        if self.yhist is not None:
            o.d_yhist = self.yhist.data_ptr()
        return o


def _stats(s):
    return {k: getattr(s, k) for k, _ in s._fields_}


class Ejacobi:
    """Element-Jacobi store (torch-owned) of one discretisation."""

    def __init__(self, disc, precision=F64):
        self.disc = disc
        self.precision = _PREC.get(precision, precision)
        nbytes = L.lib().fr_ejacobi_bytes(disc.handle, self.precision)
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=disc.device)
        self.c = L.EjacobiC(self.buf.data_ptr(), self.precision, 0.0, None)

    def inverse_blocks(self):
        dt = torch.float32 if self.precision == F32 else torch.float64
        nb = self.disc.nb
        # column-major per element: [e][col][row] -> return [e][row][col]
        return self.buf.view(dt).view(self.disc.nel, nb, nb).transpose(1, 2)


class Pmg:
    """The coarse level of a p-multigrid preconditioner: a discretisation of the same mesh
    at a lower degree, its element-Jacobi store and buffers (torch-owned)."""

    def __init__(self, fine, pc_coarse, nu1=1, nu2=1, nc=1, precision=F64):
        self.fine = fine
        self.coarse = fine.__class__(fine.nodes.cpu().numpy(), pc_coarse, flux={0: "rusanov", 1: "roe"}[fine.flux],
                                     gamma=fine.gamma, device=fine.device)
        self.cpc = Ejacobi(self.coarse, precision)
        self.Uc = self.coarse.empty()
        self.R0c = self.coarse.empty()
        self.work = torch.empty(4 * self.coarse.ndof + 32, dtype=torch.float64, device=fine.device)
        self.c = L.PmgC(self.coarse.handle, self.cpc.c, self.Uc.data_ptr(), self.R0c.data_ptr(),
                        self.work.data_ptr(), nu1, nu2, nc)


class Disc:
    """A structured quad mesh with FR degree p, bound to one GPU: doubly periodic, or (with
    Navier-Stokes) periodic in xi with a wall or far field on the eta = -1 / +1 sides."""

    def __init__(self, nodes, p, physics="euler", flux="rusanov", gamma=1.4, rgas=1.0, mu=0.0, prandtl=0.71,
                 device="cuda", viscous="br1", bc_south=None, bc_north=None, q_far=None):
        self.lib = L.lib()
        self.device = torch.device(device)
        self.nodes = torch.as_tensor(nodes, dtype=torch.float64).to(self.device).contiguous()
        self.ny, self.nx = self.nodes.shape[0] - 1, self.nodes.shape[1] - 1
        self.p = p
        self.n = p + 1
        self.np_ = self.n * self.n
        self.nb = 4 * self.np_
        self.nel = self.nx * self.ny
        self.physics = _PHYS.get(physics, physics)
        self.flux = _FLUX.get(flux, flux)
        self.gamma, self.rgas, self.mu, self.prandtl = gamma, rgas, mu, prandtl
        self.viscous = _VISC.get(viscous, viscous)
        self.bc_south, self.bc_north = _BC.get(bc_south, bc_south), _BC.get(bc_north, bc_north)
        qf = (ctypes.c_double * 4)(*([0.0] * 4 if q_far is None else [float(x) for x in q_far]))
        desc = L.DiscDesc(self.nx, self.ny, p, self.physics, self.flux, gamma, rgas, mu, prandtl,
                          self.nodes.data_ptr(), self.viscous, self.bc_south, self.bc_north, qf)
        h = ctypes.c_void_p()
        _check("fr_disc_create", self.lib.fr_disc_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.ndof = int(self.lib.fr_ndof(h))
        self.shape = (4, self.nel, self.np_)
        self._ws = {}

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.fr_disc_destroy(h)
            self.handle = None

    # ------------------------------------------------------------ helpers
    def _vec(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() \
                or t.device != self.nodes.device or t.numel() != self.ndof:
            raise ValueError(f"{name}: expected a contiguous float64 {self.device} tensor with {self.ndof} entries")
        return t

    def empty(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def zeros(self):
        return torch.zeros(self.shape, dtype=torch.float64, device=self.device)

    def workspace_mlp(self, n_hidden, batch):
        nbytes = int(self.lib.fr_mlp_work_bytes(self.handle, n_hidden, batch))
        key = ("mlp", n_hidden)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def workspace(self, what, m=20, precision=F64):
        nbytes = int(self.lib.fr_workspace_bytes(self.handle, what, m, precision))
        key = (what, m, precision)
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    # ------------------------------------------------------------ entry points
    def solution_points(self):
        xy = torch.empty((2, self.nel, self.np_), dtype=torch.float64, device=self.device)
        _check("fr_solution_points", self.lib.fr_solution_points(self.handle, _ptr(xy), _stream()))
        return xy

    def residual(self, U, R=None):
        self._vec(U, "U")
        R = self.empty() if R is None else self._vec(R, "R")
        ws = self.workspace(L.WS_RESIDUAL)
        _check("fr_residual", self.lib.fr_residual(self.handle, _ptr(U), _ptr(R), _ptr(ws), _stream()))
        return R

    def jf_matvec(self, U, R0, v, shift, eps=1e-8, eps_mode=EPS_RMS, out=None):
        for t, nm in ((U, "U"), (R0, "R0"), (v, "v")):
            self._vec(t, nm)
        out = self.empty() if out is None else self._vec(out, "out")
        ws = self.workspace(L.WS_MATVEC)
        _check("fr_jf_matvec", self.lib.fr_jf_matvec(self.handle, _ptr(U), _ptr(R0), _ptr(v), shift, eps, eps_mode,
                                                     _ptr(out), _ptr(ws), _stream()))
        return out

    def jf_matvec_noalloc(self, U, R0, v, shift, eps=1e-8, eps_mode=EPS_RMS, out=None):
        """fr_jf_matvec_noalloc: the JF product with the library's static scratch (no workspace)."""
        for t, nm in ((U, "U"), (R0, "R0"), (v, "v")):
            self._vec(t, nm)
        out = self.empty() if out is None else self._vec(out, "out")
        _check("fr_jf_matvec_noalloc", self.lib.fr_jf_matvec_noalloc(self.handle, _ptr(U), _ptr(R0), _ptr(v), shift,
                                                                     eps, eps_mode, _ptr(out), _stream()))
        return out

    def ejacobi_assemble(self, U, shift):
        """Raw FP64 blocks P_e = shift I - dR_e/dq_e as a [nel, Nb, Nb] (row, col) tensor."""
        self._vec(U, "U")
        blocks = torch.empty((self.nel, self.nb, self.nb), dtype=torch.float64, device=self.device)
        ws = self.workspace(L.WS_RESIDUAL)
        _check("fr_ejacobi_assemble", self.lib.fr_ejacobi_assemble(self.handle, _ptr(U), shift, _ptr(blocks),
                                                                   _ptr(ws), _stream()))
        return blocks.transpose(1, 2)   # stored column-major

    def ejacobi_factor(self, U, shift, precision=F64, pc=None):
        self._vec(U, "U")
        pc = Ejacobi(self, precision) if pc is None else pc
        ws = self.workspace(L.WS_RESIDUAL)
        _check("fr_ejacobi_factor", self.lib.fr_ejacobi_factor(self.handle, _ptr(U), shift, ctypes.byref(pc.c),
                                                               _ptr(ws), _stream()))
        return pc

    def ejacobi_factor_blocks(self, blocks_rowcol, precision=F64):
        """Invert caller-given blocks [nel, Nb, Nb] (row, col)."""
        colmajor = blocks_rowcol.to(self.device, torch.float64).transpose(1, 2).contiguous()
        pc = Ejacobi(self, precision)
        _check("fr_ejacobi_factor_blocks", self.lib.fr_ejacobi_factor_blocks(self.handle, _ptr(colmajor),
                                                                             ctypes.byref(pc.c), _stream()))
        torch.cuda.current_stream().synchronize()
        return pc

    def ejacobi_solve(self, pc, r, z=None):
        self._vec(r, "r")
        z = self.empty() if z is None else self._vec(z, "z")
        _check("fr_ejacobi_solve", self.lib.fr_ejacobi_solve(self.handle, ctypes.byref(pc.c), _ptr(r), _ptr(z),
                                                             _stream()))
        return z

    def pmg_factor(self, U, shift, mg, precision=F64, pc=None):
        """Fine element-Jacobi at (U, shift) plus the coarse level of mg (Pmg): returns the
        fine store, which carries mg for FR_PC_PMG solves."""
        self._vec(U, "U")
        pc = Ejacobi(self, precision) if pc is None else pc
        ws = self.workspace(L.WS_RESIDUAL)
        _check("fr_pmg_factor", self.lib.fr_pmg_factor(self.handle, _ptr(U), shift, ctypes.byref(pc.c),
                                                       ctypes.byref(mg.c), _ptr(ws), _stream()))
        pc.mg = mg   # keep the coarse level alive with the store
        return pc

    def pmg_apply(self, pc, U, R0, shift, r, eps=1e-8, eps_mode=EPS_RMS, z=None):
        """z = M^{-1} r for the p-multigrid preconditioner of pc (from pmg_factor)."""
        for t, nm in ((U, "U"), (R0, "R0"), (r, "r")):
            self._vec(t, nm)
        z = self.empty() if z is None else self._vec(z, "z")
        ws = self.workspace(L.WS_GMRES, 1)
        _check("fr_pmg_apply", self.lib.fr_pmg_apply(self.handle, ctypes.byref(pc.c), _ptr(U), _ptr(R0), shift, eps,
                                                     eps_mode, _ptr(r), _ptr(z), _ptr(ws), _stream()))
        return z

    def lusgs_apply(self, pc, U, R0, shift, r, eps=1e-8, eps_mode=EPS_RMS, z=None):
        """z = M^{-1} r for the LU-SGS preconditioner built on the element blocks of pc."""
        for t, nm in ((U, "U"), (R0, "R0"), (r, "r")):
            self._vec(t, nm)
        z = self.empty() if z is None else self._vec(z, "z")
        ws = self.workspace(L.WS_GMRES, 1)
        _check("fr_lusgs_apply", self.lib.fr_lusgs_apply(self.handle, ctypes.byref(pc.c), _ptr(U), _ptr(R0), shift,
                                                         eps, eps_mode, _ptr(r), _ptr(z), _ptr(ws), _stream()))
        return z

    def gmres_solve(self, pc, U, R0, shift, b, x=None, opts=None):
        opts = opts or GmresOpts()
        for t, nm in ((U, "U"), (R0, "R0"), (b, "b")):
            self._vec(t, nm)
        x = self.zeros() if x is None else self._vec(x, "x")
        ws = self.workspace(L.WS_GMRES, opts.m)
        st = L.GmresStatsC()
        oc = opts.c()
        status = self.lib.fr_gmres_solve(self.handle, ctypes.byref(pc.c), _ptr(U), _ptr(R0), shift, _ptr(b), _ptr(x),
                                         ctypes.byref(oc), ctypes.byref(st), _ptr(ws), _stream())
        _check("fr_gmres_solve", status, allow_numerical=True)
        return x, dict(_stats(st), status=status)

    def _step_ws(self, opts):
        lin = opts.lin or GmresOpts()
        return self.workspace(L.WS_STEP, lin.m, opts.precond_precision)

    def _check_hist(self, opts):
        if opts.yhist is not None:
            self._vec(opts.yhist.view(-1)[: self.ndof], "yhist")
            if opts.yhist.numel() != 2 * self.ndof or not opts.yhist.is_contiguous():
                raise ValueError("yhist: expected a contiguous (2, ndof) float64 tensor")

    def row_step(self, U, scheme, dt, opts=None):
        opts = opts or SolverOpts(lin=GmresOpts())
        self._vec(U, "U")
        st = L.StepStatsC()
        oc = opts.c()
        self._check_hist(opts)
        status = self.lib.fr_row_step(self.handle, int(scheme), dt, _ptr(U), ctypes.byref(oc), ctypes.byref(st),
                                      _ptr(self._step_ws(opts)), _stream())
        _check("fr_row_step", status, allow_numerical=True)
        if opts.log is not None:
            opts.log.pull()
        return dict(_stats(st), status=status)

    def esdirk_step(self, U, scheme, dt, opts=None):
        opts = opts or SolverOpts(lin=GmresOpts(rtol=1e-1))
        self._vec(U, "U")
        st = L.StepStatsC()
        oc = opts.c()
        self._check_hist(opts)
        status = self.lib.fr_esdirk_step(self.handle, int(scheme), dt, _ptr(U), ctypes.byref(oc), ctypes.byref(st),
                                         _ptr(self._step_ws(opts)), _stream())
        _check("fr_esdirk_step", status, allow_numerical=True)
        if opts.log is not None:
            opts.log.pull()
        return dict(_stats(st), status=status)

    def bdf2_step(self, Unm1, Un, dt, opts=None, out=None):
        opts = opts or SolverOpts(lin=GmresOpts(rtol=1e-1))
        self._vec(Un, "Un")
        if Unm1 is not None:
            self._vec(Unm1, "Unm1")
        out = self.empty() if out is None else self._vec(out, "out")
        st = L.StepStatsC()
        oc = opts.c()
        self._check_hist(opts)
        status = self.lib.fr_bdf2_step(self.handle, dt, _ptr(Unm1), _ptr(Un), _ptr(out), ctypes.byref(oc),
                                       ctypes.byref(st), _ptr(self._step_ws(opts)), _stream())
        _check("fr_bdf2_step", status, allow_numerical=True)
        if opts.log is not None:
            opts.log.pull()
        return out, dict(_stats(st), status=status)

    def l2_error_vortex(self, U, var, t, vortex):
        """vortex: object with the fields of fr_inputs.Vortex."""
        self._vec(U, "U")
        prm = (ctypes.c_double * 14)(vortex.rho_inf, vortex.u_inf, vortex.v_inf, vortex.p_inf, vortex.rgas,
                                     vortex.gamma, vortex.alpha, vortex.phi, vortex.xc, vortex.yc, vortex.xlo,
                                     vortex.ylo, vortex.lx, vortex.ly)
        err = ctypes.c_double()
        ws = self.workspace(L.WS_MATVEC)
        _check("fr_l2_error_vortex", self.lib.fr_l2_error_vortex(self.handle, _ptr(U), var, t, prm,
                                                                 ctypes.byref(err), _ptr(ws), _stream()))
        return err.value

    def wall_force(self, U):
        """(F_x, F_y): force of the fluid on the wall of the eta = -1 side (fr_wall_force)."""
        self._vec(U, "U")
        f = (ctypes.c_double * 2)()
        ws = self.workspace(L.WS_RESIDUAL)
        _check("fr_wall_force", self.lib.fr_wall_force(self.handle, _ptr(U), f, _ptr(ws), _stream()))
        return f[0], f[1]


# ---------------------------------------------------------------- 3D hexahedra
class Disc3D:
    """Uniform hexahedra of a triply periodic box with FR degree p, bound to one GPU
    (fr3d_* of the C ABI); mu > 0 gives Navier-Stokes with the BR2 gradient, mu = 0 Euler."""

    def __init__(self, nx, ny, nz, p, lo, length, flux="roe", gamma=1.4, rgas=1.0, mu=0.0, prandtl=0.71,
                 device="cuda"):
        self.lib = L.lib()
        self.device = torch.device(device)
        self.nx, self.ny, self.nz, self.p, self.n = nx, ny, nz, p, p + 1
        self.np_ = self.n ** 3
        self.nel = nx * ny * nz
        desc = L.Desc3C(nx, ny, nz, p, _FLUX.get(flux, flux), (ctypes.c_double * 3)(*lo),
                        (ctypes.c_double * 3)(*length), gamma, rgas, mu, prandtl)
        h = ctypes.c_void_p()
        _check("fr3d_create", self.lib.fr3d_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        self.ndof = int(self.lib.fr3d_ndof(h))
        self.shape = (5, self.nel, self.np_)
        self.work = torch.empty(int(self.lib.fr3d_workspace_bytes(h)), dtype=torch.uint8, device=self.device)
        self.device = self.work.device        # with its index (cuda:0)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.fr3d_destroy(h)
            self.handle = None

    def _vec(self, t, name):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_contiguous() \
                or t.device != self.device or t.numel() != self.ndof:
            raise ValueError(f"{name}: expected a contiguous float64 {self.device} tensor with {self.ndof} entries")
        return t

    def empty(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def solution_points(self):
        import numpy as np
        xyz = np.empty((3, self.nel * self.np_))
        _check("fr3d_solution_points", self.lib.fr3d_solution_points(self.handle, xyz.ctypes.data))
        return xyz

    def residual(self, U, out=None):
        self._vec(U, "U")
        out = self.empty() if out is None else out
        _check("fr3d_residual", self.lib.fr3d_residual(self.handle, _ptr(U), _ptr(out), _ptr(self.work), _stream()))
        return out

    def jf_matvec(self, U, R0, v, shift, eps=1e-8, eps_mode=EPS_RMS, out=None):
        for t, nm in ((U, "U"), (R0, "R0"), (v, "v")):
            self._vec(t, nm)
        out = self.empty() if out is None else out
        _check("fr3d_jf_matvec", self.lib.fr3d_jf_matvec(self.handle, _ptr(U), _ptr(R0), _ptr(v), shift, eps, eps_mode,
                                                         _ptr(out), _ptr(self.work), _stream()))
        return out

    def ssprk3_step(self, U, dt):
        self._vec(U, "U")
        _check("fr3d_ssprk3_step", self.lib.fr3d_ssprk3_step(self.handle, _ptr(U), dt, _ptr(self.work), _stream()))

    # ---- implicit steps (FP64 element-Jacobi on 5 (p+1)^3-row blocks, p = 2 or 3)
    @property
    def nb(self):
        return 5 * self.np_

    def step_workspace(self, m):
        """The workspace of the implicit calls for restart length m, kept between calls."""
        ws = getattr(self, "_ws3", {})
        self._ws3 = ws
        if m not in ws:
            nbytes = int(self.lib.fr3d_step_workspace_bytes(self.handle, m))
            if nbytes == 0:
                raise ValueError("fr3d_step_workspace_bytes: m must be 1 .. 64")
            ws.clear()      # one workspace at a time: they hold two block stores each
            ws[m] = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return ws[m]

    def ejacobi_assemble(self, U, shift):
        """The element blocks shift I - dR_e/dq_e, returned as [nel, Nb, Nb] (row, column)."""
        self._vec(U, "U")
        B = torch.empty((self.nel, self.nb, self.nb), dtype=torch.float64, device=self.device)
        _check("fr3d_ejacobi_assemble", self.lib.fr3d_ejacobi_assemble(self.handle, _ptr(U), shift, _ptr(B),
                                                                       _ptr(self.step_workspace(1)), _stream()))
        return B.transpose(1, 2)        # stored column-major per element

    def ejacobi_factor(self, U, shift):
        """The inverse blocks (the library's column-major store) at (U, shift)."""
        self._vec(U, "U")
        inv = torch.empty((self.nel, self.nb, self.nb), dtype=torch.float64, device=self.device)
        _check("fr3d_ejacobi_factor", self.lib.fr3d_ejacobi_factor(self.handle, _ptr(U), shift, _ptr(inv),
                                                                   _ptr(self.step_workspace(1)), _stream()))
        return inv

    def ejacobi_apply(self, inv, r, out=None):
        self._vec(r, "r")
        out = self.empty() if out is None else self._vec(out, "out")
        _check("fr3d_ejacobi_apply", self.lib.fr3d_ejacobi_apply(self.handle, _ptr(inv), _ptr(r), _ptr(out),
                                                                 _stream()))
        return out

    def gmres_solve(self, inv, U, R0, shift, b, x=None, opts=None):
        opts = opts or GmresOpts()
        for t, nm in ((U, "U"), (R0, "R0"), (b, "b")):
            self._vec(t, nm)
        x = torch.zeros(self.shape, dtype=torch.float64, device=self.device) if x is None else self._vec(x, "x")
        st = L.GmresStatsC()
        oc = opts.c()
        status = self.lib.fr3d_gmres_solve(self.handle, _ptr(inv), _ptr(U), _ptr(R0), shift, _ptr(b), _ptr(x),
                                           ctypes.byref(oc), ctypes.byref(st), _ptr(self.step_workspace(opts.m)),
                                           _stream())
        _check("fr3d_gmres_solve", status, allow_numerical=True)
        return x, dict(_stats(st), status=status)

    def _step(self, name, opts, *args):
        st = L.StepStatsC()
        oc = opts.c()
        ws = self.step_workspace((opts.lin or GmresOpts()).m)
        status = getattr(self.lib, name)(self.handle, *args, ctypes.byref(oc), ctypes.byref(st), _ptr(ws), _stream())
        _check(name, status, allow_numerical=True)
        return dict(_stats(st), status=status)

    def row_step(self, U, scheme, dt, opts=None):
        opts = opts or SolverOpts(lin=GmresOpts())
        self._vec(U, "U")
        return self._step("fr3d_row_step", opts, int(scheme), dt, _ptr(U))

    def esdirk_step(self, U, scheme, dt, opts=None):
        opts = opts or SolverOpts(lin=GmresOpts(rtol=1e-1))
        self._vec(U, "U")
        return self._step("fr3d_esdirk_step", opts, int(scheme), dt, _ptr(U))

    def bdf2_step(self, Unm1, Un, dt, opts=None, out=None):
        opts = opts or SolverOpts(lin=GmresOpts(rtol=1e-1))
        self._vec(Un, "Un")
        if Unm1 is not None:
            self._vec(Unm1, "Unm1")
        out = self.empty() if out is None else self._vec(out, "out")
        return out, self._step("fr3d_bdf2_step", opts, dt, _ptr(Unm1), _ptr(Un), _ptr(out))

    def dissipation(self, U, rho0=1.0):
        """(E_k, eps1, eps3) of the Taylor-Green diagnostics."""
        self._vec(U, "U")
        h = (ctypes.c_double * 3)()
        _check("fr3d_dissipation", self.lib.fr3d_dissipation(self.handle, _ptr(U), rho0, h, _ptr(self.work),
                                                             _stream()))
        return h[0], h[1], h[2]


# ---------------------------------------------------------------- learned warm start
class Mlp:
    """Per-element MLP (BF16 weights) on the device; sizes fixed by the disc's degree."""

    def __init__(self, disc, n_hidden=256):
        lib = L.lib()
        self.disc = disc
        self.n_in, self.n_hidden, self.n_out = 16 * disc.np_, n_hidden, 4 * disc.np_
        nw = lib.fr_mlp_weight_bytes(self.n_in, n_hidden, self.n_out) // 2
        self.w = torch.zeros(nw, dtype=torch.bfloat16, device=disc.device)
        self.b = torch.zeros(2 * n_hidden + self.n_out, dtype=torch.float32, device=disc.device)
        self.norm = torch.tensor([0.0, 1.0] * 20, dtype=torch.float32, device=disc.device)
        self.c = L.MlpC(self.n_in, n_hidden, self.n_out, self.w.data_ptr(), self.b.data_ptr(), self.norm.data_ptr())

    def forward(self, x_bf16, y=None):
        """Raw forward pass on standardised bf16 features [batch, n_in] -> [batch, n_out] float32."""
        B = x_bf16.shape[0]
        y = torch.empty((B, self.n_out), dtype=torch.float32, device=self.disc.device) if y is None else y
        ws = self.disc.workspace_mlp(self.n_hidden, B)
        _check("fr_mlp_forward", L.lib().fr_mlp_forward(ctypes.byref(self.c), _ptr(x_bf16.contiguous()), B, _ptr(y),
                                                        _ptr(ws), _stream()))
        return y

    def infer(self, U, R, Y1, Y2, dt, out=None):
        d = self.disc
        out = d.empty() if out is None else out
        ws = d.workspace_mlp(self.n_hidden, 1)
        _check("fr_mlp_infer", L.lib().fr_mlp_infer(d.handle, ctypes.byref(self.c), _ptr(U), _ptr(R), _ptr(Y1),
                                                    _ptr(Y2), dt, _ptr(out), _ptr(ws), _stream()))
        return out


class MlpTrainer:
    """FP32 master parameters + Adam state of one network; initial weights uniform in
    +-1/sqrt(fan_in) from a seeded generator, biases zero."""

    def __init__(self, disc, n_hidden=256, seed=4, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        import numpy as np
        self.net = Mlp(disc, n_hidden)
        n = L.lib().fr_mlp_param_count(self.net.n_in, n_hidden, self.net.n_out)
        rng = np.random.default_rng(seed)
        parts = []
        for o, i in ((n_hidden, self.net.n_in), (n_hidden, n_hidden), (self.net.n_out, n_hidden)):
            lim = 1.0 / np.sqrt(i)
            parts += [rng.uniform(-lim, lim, size=o * i), np.zeros(o)]
        init = np.concatenate(parts).astype(np.float32)
        assert init.size == n
        dev = disc.device
        self.master = torch.as_tensor(init, device=dev)
        self.grad = torch.zeros(n, dtype=torch.float32, device=dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        self.c = L.MlpTrainerC(self.net.c, self.master.data_ptr(), self.grad.data_ptr(), self.m.data_ptr(),
                               self.v.data_ptr(), 0, lr, beta1, beta2, eps)
        self.sync()

    def set_master(self, flat):
        self.master.copy_(torch.as_tensor(flat, dtype=torch.float32))
        self.sync()

    def sync(self):
        _check("fr_mlp_sync", L.lib().fr_mlp_sync(ctypes.byref(self.c), _stream()))

    def fit_stats(self, log):
        _check("fr_mlp_fit_stats", L.lib().fr_mlp_fit_stats(self.net.disc.handle, ctypes.byref(log.c),
                                                            ctypes.byref(self.c.net), _stream()))

    def step(self, log, idx, lr=None, read_loss=True):
        """One Adam step on the logged rows idx (int32 device tensor); returns the batch
        loss, or None without a host read when read_loss is False."""
        if lr is not None:
            self.c.lr = lr
        loss = ctypes.c_double()
        ws = self.net.disc.workspace_mlp(self.net.n_hidden, idx.numel())
        _check("fr_mlp_train_step", L.lib().fr_mlp_train_step(self.net.disc.handle, ctypes.byref(self.c),
                                                              ctypes.byref(log.c), _ptr(idx), idx.numel(),
                                                              ctypes.byref(loss) if read_loss else None, _ptr(ws),
                                                              _stream()))
        return loss.value if read_loss else None

    def fit(self, log, steps, batch, lr=1e-3, seed=0, report_every=100):
        """`steps` Adam steps with a cosine-decayed learning rate on random batches of the
        log (each batch drawn without replacement, seeded; all batches copied to the device
        at once).  The loss is read back only every `report_every` steps and at the end:
        returns the list of those (step, loss) pairs."""
        idx = _fit_batches(log.count, steps, batch, seed)
        lrs = _cosine_lr(lr, steps)
        didx = torch.as_tensor(idx, device=self.net.disc.device)
        out = []
        for it in range(steps):
            rd = (it + 1) % report_every == 0 or it + 1 == steps or it == 0
            l = self.step(log, didx[it], lr=lrs[it], read_loss=rd)
            if rd:
                out.append((it, l))
        return out


def _fit_batches(n, steps, batch, seed):
    """The batches of MlpTrainer.fit: per step `batch` logged rows drawn without replacement."""
    import numpy as np
    rng = np.random.default_rng(seed)
    b = min(batch, n)
    return np.stack([rng.choice(n, b, replace=False) for _ in range(steps)]).astype(np.int32)


def _cosine_lr(lr, steps):
    import numpy as np
    return [lr * 0.5 * (1 + np.cos(np.pi * it / steps)) for it in range(steps)]


def fit_group(trainers, logs, steps, batch, lr=1e-3, seeds=None, report_every=100):
    """Train several networks of equal sizes together (fr_mlp_train_group): `steps` Adam
    steps of trainers[q] on logs[q], with the batches and cosine-decayed learning rate that
    MlpTrainer.fit draws from seeds[q], so every network ends bitwise where its own fit
    would have left it.  The step loop runs in the library; the losses are read after the
    first step, every report_every steps and at the end: returns per trainer the list of
    those (step, loss) pairs."""
    import numpy as np
    count = len(trainers)
    if count != len(logs) or not 1 <= count <= 8:
        raise ValueError("fit_group: one log per trainer, 1..8 trainers")
    seeds = list(seeds) if seeds is not None else [0] * count
    disc = trainers[0].net.disc
    idx = np.stack([_fit_batches(lg.count, steps, batch, sd) for lg, sd in zip(logs, seeds)])  # [count][steps][b]
    b = idx.shape[2]
    didx = torch.as_tensor(idx, device=disc.device)
    lrs = np.asarray(_cosine_lr(lr, steps), dtype=np.float32)
    nbytes = int(L.lib().fr_mlp_group_work_bytes(disc.handle, trainers[0].net.n_hidden, b, count))
    if nbytes == 0:
        raise ValueError("fit_group: invalid sizes")
    work = torch.empty(nbytes, dtype=torch.uint8, device=disc.device)
    arr = (L.MlpTrainerC * count)(*[t.c for t in trainers])
    larr = (L.StageLogC * count)(*[lg.c for lg in logs])
    bounds = sorted({0, 1, steps} | set(range(report_every, steps, report_every)))
    out = [[] for _ in range(count)]
    loss = (ctypes.c_double * count)()
    for a, e in zip(bounds[:-1], bounds[1:]):
        chunk = didx[:, a:e, :].contiguous()
        lr_c = (ctypes.c_float * (e - a))(*lrs[a:e])
        _check("fr_mlp_train_group", L.lib().fr_mlp_train_group(disc.handle, arr, larr, count, _ptr(chunk), e - a, b,
                                                                lr_c, loss, _ptr(work), _stream()))
        for q in range(count):
            out[q].append((e - 1, loss[q]))
    for q, t in enumerate(trainers):
        t.c.t, t.c.lr = arr[q].t, arr[q].lr
    return out


class StageLog:
    """Device buffer of logged (inputs, converged increment) samples of one stage."""

    def __init__(self, disc, capacity, elems):
        self.disc = disc
        self.stride = 20 * disc.np_
        self.samples = torch.zeros((capacity, self.stride), dtype=torch.float32, device=disc.device)
        self.elems = torch.as_tensor(elems, dtype=torch.int32, device=disc.device).contiguous()
        self.c = L.StageLogC(self.samples.data_ptr(), self.elems.data_ptr(), self.elems.numel(), capacity, 0)

    @property
    def count(self):
        return self.c.count

    def set_elems(self, elems):
        self.elems.copy_(torch.as_tensor(elems, dtype=torch.int32))


class StageLogs:
    """One StageLog per stage of a scheme, as the C ABI expects (contiguous array)."""

    def __init__(self, logs):
        self.logs = logs
        self.array = (L.StageLogC * len(logs))(*[lg.c for lg in logs])

    def pull(self):
        for i, lg in enumerate(self.logs):
            lg.c.count = self.array[i].count


class WarmStart:
    """One network per stage, contiguous for the C ABI, plus the inference workspace."""

    def __init__(self, nets):
        self.nets = nets
        self.array = (L.MlpC * len(nets))(*[n.c for n in nets])
        d = nets[0].disc
        self.work = d.workspace_mlp(nets[0].n_hidden, 1)


def scheme_table(kind, scheme):
    """Coefficients compiled into the library: kind 0 = ROW (a, c, m, gamma), 1 = ESDIRK (a, b, gamma)."""
    a = (ctypes.c_double * 36)()
    c = (ctypes.c_double * 36)()
    b = (ctypes.c_double * 6)()
    g = ctypes.c_double()
    s = L.lib().fr_scheme_table(kind, scheme, a, c, b, ctypes.byref(g))
    if s < 0:
        raise ValueError("unknown scheme")
    import numpy as np
    A = np.array(a[:s * s]).reshape(s, s)
    C = np.array(c[:s * s]).reshape(s, s)
    return A, C, np.array(b[:s]), g.value
