"""MI355X Newton-step library for quadratic-objective SOCP interior-point
methods (the problem class of QOCO-GPU, arXiv 2603.29197).

The numeric work lives in the HIP library ``libqg.so`` (C ABI in
include/qg.h); this package only marshals arguments to it.
"""
from ._lib import QG_FP32_IR, QG_FP64, QG_ORDER_MD, QG_ORDER_ND, QGError, lib  # noqa: F401
from .api import BatchSolver, QGSolve, QGSolveAll, Solver, analyze, default_settings  # noqa: F401
