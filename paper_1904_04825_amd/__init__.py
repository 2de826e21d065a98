"""MI355X (gfx950) Jacobian-free implicit solver for FR/CPR discretisations.

The compute path is the HIP library libfrjf.so behind the C ABI in
include/frjf.h; this package is a thin binding that marshals torch tensors
(device memory, streams) into those calls.
"""
from .api import (Disc, Ejacobi, GmresOpts, SolverOpts, FrError, Mlp, MlpTrainer, StageLog, StageLogs, WarmStart,
                  EULER, NS_BR1, RUSANOV, ROE, F64, F32, EPS_ABS, EPS_RMS, PC_EJACOBI, PC_LUSGS, PC_PMG, Pmg, fit_group, Disc3D)

__all__ = ["Disc", "Ejacobi", "GmresOpts", "SolverOpts", "FrError", "Mlp", "MlpTrainer", "StageLog", "StageLogs",
           "WarmStart", "EULER", "NS_BR1", "RUSANOV", "ROE",
           "F64", "F32", "EPS_ABS", "EPS_RMS", "PC_EJACOBI", "PC_LUSGS", "PC_PMG", "Pmg", "fit_group", "Disc3D"]
