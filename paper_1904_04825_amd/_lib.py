"""ctypes declarations of the frjf C ABI (include/frjf.h)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, Structure, c_double, c_int, c_long, c_size_t, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfrjf.so")

FR_OK, FR_EINVAL, FR_EHIP, FR_ESIZE = 0, -1, -2, -3
FR_NOTCONV, FR_BREAKDOWN, FR_ENAN, FR_REJECTED = 1, 2, 3, 4
STATUS_NAMES = {0: "FR_OK", -1: "FR_EINVAL", -2: "FR_EHIP", -3: "FR_ESIZE", 1: "FR_NOTCONV",
                2: "FR_BREAKDOWN", 3: "FR_ENAN", 4: "FR_REJECTED"}
WS_RESIDUAL, WS_MATVEC, WS_GMRES, WS_STEP = 0, 1, 2, 3


class DiscDesc(Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("p", c_int), ("physics", c_int), ("flux", c_int),
                ("gamma", c_double), ("rgas", c_double), ("mu", c_double), ("prandtl", c_double),
                ("d_nodes", c_void_p), ("viscous", c_int), ("bc_south", c_int), ("bc_north", c_int),
                ("q_far", c_double * 4)]


class Desc3C(Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("nz", c_int), ("p", c_int), ("flux", c_int),
                ("lo", c_double * 3), ("len", c_double * 3), ("gamma", c_double), ("rgas", c_double),
                ("mu", c_double), ("prandtl", c_double)]


class EjacobiC(Structure):
    _fields_ = [("d_factors", c_void_p), ("precision", c_int), ("shift", c_double), ("mg", c_void_p)]


class PmgC(Structure):
    _fields_ = [("coarse", c_void_p), ("coarse_pc", EjacobiC), ("d_Uc", c_void_p), ("d_R0c", c_void_p),
                ("d_work_c", c_void_p), ("nu1", c_int), ("nu2", c_int), ("nc", c_int)]


class GmresOptsC(Structure):
    _fields_ = [("m", c_int), ("max_iters", c_int), ("rtol", c_double), ("ref_norm", c_double),
                ("eps", c_double), ("eps_mode", c_int), ("precond", c_int)]


class GmresStatsC(Structure):
    _fields_ = [("iters", c_int), ("restarts", c_int), ("converged", c_int), ("r_ref", c_double),
                ("r_final", c_double), ("residual_evals", c_long)]


class MlpC(Structure):
    _fields_ = [("n_in", c_int), ("n_hidden", c_int), ("n_out", c_int), ("d_w", c_void_p), ("d_b", c_void_p),
                ("d_norm", c_void_p)]


class MlpTrainerC(Structure):
    _fields_ = [("net", MlpC), ("d_master", c_void_p), ("d_grad", c_void_p), ("d_m", c_void_p), ("d_v", c_void_p),
                ("t", c_int), ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


class StageLogC(Structure):
    _fields_ = [("d_samples", c_void_p), ("d_elems", c_void_p), ("per_stage", c_int), ("capacity", c_int),
                ("count", c_int)]


class SolverOptsC(Structure):
    _fields_ = [("lin", GmresOptsC), ("tol_nl", c_double), ("dtau_init", c_double), ("dtau_max", c_double),
                ("max_ptc", c_int), ("max_reject", c_int), ("precond_precision", c_int),
                ("commit_unconverged", c_int), ("warm", c_void_p), ("log", c_void_p), ("d_yhist", c_void_p),
                ("d_mlp_work", c_void_p)]


class StepStatsC(Structure):
    _fields_ = [("gmres_iters", c_int), ("ptc_iters", c_int), ("rejections", c_int), ("linear_solves", c_int),
                ("unconverged", c_int), ("warm_used", c_int), ("warm_rejected", c_int), ("residual_evals", c_long),
                ("wall_s", c_double)]


_SIGS = {
    "fr_disc_create": (c_int, [POINTER(DiscDesc), POINTER(c_void_p)]),
    "fr_disc_destroy": (None, [c_void_p]),
    "fr_ndof": (c_size_t, [c_void_p]),
    "fr_workspace_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int]),
    "fr_ejacobi_bytes": (c_size_t, [c_void_p, c_int]),
    "fr_solution_points": (c_int, [c_void_p, c_void_p, c_void_p]),
    "fr_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "fr_jf_matvec": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_int, c_void_p,
                             c_void_p, c_void_p]),
    "fr_lusgs_apply": (c_int, [c_void_p, POINTER(EjacobiC), c_void_p, c_void_p, c_double, c_double, c_int, c_void_p,
                               c_void_p, c_void_p, c_void_p]),
    "fr_pmg_factor": (c_int, [c_void_p, c_void_p, c_double, POINTER(EjacobiC), POINTER(PmgC), c_void_p, c_void_p]),
    "fr_pmg_apply": (c_int, [c_void_p, POINTER(EjacobiC), c_void_p, c_void_p, c_double, c_double, c_int, c_void_p,
                             c_void_p, c_void_p, c_void_p]),
    "fr_jf_matvec_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_int, c_void_p,
                                     c_void_p]),
    "fr_ejacobi_assemble": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "fr_ejacobi_factor": (c_int, [c_void_p, c_void_p, c_double, POINTER(EjacobiC), c_void_p, c_void_p]),
    "fr_ejacobi_factor_blocks": (c_int, [c_void_p, c_void_p, POINTER(EjacobiC), c_void_p]),
    "fr_ejacobi_solve": (c_int, [c_void_p, POINTER(EjacobiC), c_void_p, c_void_p, c_void_p]),
    "fr_gmres_solve": (c_int, [c_void_p, POINTER(EjacobiC), c_void_p, c_void_p, c_double, c_void_p, c_void_p,
                               POINTER(GmresOptsC), POINTER(GmresStatsC), c_void_p, c_void_p]),
    "fr_row_step": (c_int, [c_void_p, c_int, c_double, c_void_p, POINTER(SolverOptsC), POINTER(StepStatsC),
                            c_void_p, c_void_p]),
    "fr_esdirk_step": (c_int, [c_void_p, c_int, c_double, c_void_p, POINTER(SolverOptsC), POINTER(StepStatsC),
                               c_void_p, c_void_p]),
    "fr_bdf2_step": (c_int, [c_void_p, c_double, c_void_p, c_void_p, c_void_p, POINTER(SolverOptsC),
                             POINTER(StepStatsC), c_void_p, c_void_p]),
    "fr_l2_error_vortex": (c_int, [c_void_p, c_void_p, c_int, c_double, POINTER(c_double), POINTER(c_double),
                                   c_void_p, c_void_p]),
    "fr_scheme_table": (c_int, [c_int, c_int, POINTER(c_double), POINTER(c_double), POINTER(c_double),
                                POINTER(c_double)]),
    "fr_mlp_weight_bytes": (c_size_t, [c_int, c_int, c_int]),
    "fr_mlp_param_count": (c_size_t, [c_int, c_int, c_int]),
    "fr_mlp_work_bytes": (c_size_t, [c_void_p, c_int, c_int]),
    "fr_mlp_infer": (c_int, [c_void_p, POINTER(MlpC), c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p,
                             c_void_p, c_void_p]),
    "fr_mlp_forward": (c_int, [POINTER(MlpC), c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "fr_mlp_fit_stats": (c_int, [c_void_p, POINTER(StageLogC), POINTER(MlpC), c_void_p]),
    "fr_mlp_sync": (c_int, [POINTER(MlpTrainerC), c_void_p]),
    "fr_mlp_train_step": (c_int, [c_void_p, POINTER(MlpTrainerC), POINTER(StageLogC), c_void_p, c_int,
                                  POINTER(c_double), c_void_p, c_void_p]),
    "fr_mlp_group_work_bytes": (c_size_t, [c_void_p, c_int, c_int, c_int]),
    "fr_mlp_train_group": (c_int, [c_void_p, POINTER(MlpTrainerC), POINTER(StageLogC), c_int, c_void_p, c_int, c_int,
                                   POINTER(ctypes.c_float), POINTER(c_double), c_void_p, c_void_p]),
    "fr_wall_force": (c_int, [c_void_p, c_void_p, POINTER(c_double), c_void_p, c_void_p]),
    "fr3d_create": (c_int, [POINTER(Desc3C), POINTER(c_void_p)]),
    "fr3d_destroy": (None, [c_void_p]),
    "fr3d_ndof": (c_size_t, [c_void_p]),
    "fr3d_workspace_bytes": (c_size_t, [c_void_p]),
    "fr3d_solution_points": (c_int, [c_void_p, c_void_p]),
    "fr3d_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "fr3d_jf_matvec": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_int, c_void_p,
                               c_void_p, c_void_p]),
    "fr3d_ssprk3_step": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_void_p]),
    "fr3d_dissipation": (c_int, [c_void_p, c_void_p, c_double, POINTER(c_double), c_void_p, c_void_p]),
    "fr3d_ejacobi_bytes": (c_size_t, [c_void_p]),
    "fr3d_step_workspace_bytes": (c_size_t, [c_void_p, c_int]),
    "fr3d_ejacobi_assemble": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "fr3d_ejacobi_factor": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_void_p, c_void_p]),
    "fr3d_ejacobi_apply": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "fr3d_gmres_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_void_p, c_void_p,
                                 POINTER(GmresOptsC), POINTER(GmresStatsC), c_void_p, c_void_p]),
    "fr3d_row_step": (c_int, [c_void_p, c_int, c_double, c_void_p, POINTER(SolverOptsC), POINTER(StepStatsC),
                              c_void_p, c_void_p]),
    "fr3d_esdirk_step": (c_int, [c_void_p, c_int, c_double, c_void_p, POINTER(SolverOptsC), POINTER(StepStatsC),
                                 c_void_p, c_void_p]),
    "fr3d_bdf2_step": (c_int, [c_void_p, c_double, c_void_p, c_void_p, c_void_p, POINTER(SolverOptsC),
                               POINTER(StepStatsC), c_void_p, c_void_p]),
    "fr_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libfrjf.so (built in-tree by paper_1904_04825_amd/build.py).  Raises if absent:
    there is no fallback path."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"frjf HIP library not built: {LIB_PATH} is missing "
                              "(run python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib
