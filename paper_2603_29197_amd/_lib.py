"""ctypes binding of the C ABI in include/qg.h (argument marshalling only).

The shared library ``libqg.so`` is built in this directory by ``build.py``;
importing this module fails loudly if it is missing -- there is no other
implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqg.so")

c_int32_p = ctypes.POINTER(ctypes.c_int32)
c_int64_p = ctypes.POINTER(ctypes.c_int64)
c_double_p = ctypes.POINTER(ctypes.c_double)

QG_OK = 0
ERRORS = {-1: "QG_ERR_ARG", -2: "QG_ERR_PATTERN", -3: "QG_ERR_NONFINITE", -4: "QG_ERR_OOM",
          -5: "QG_ERR_HIP", -6: "QG_ERR_STATE", -7: "QG_ERR_DEVICE", -8: "QG_ERR_SIZE"}
STATUS = {0: "unsolved", 1: "solved", 2: "solved_inaccurate", -1: "max_iter", -2: "numerical_error"}
QG_FP64 = 0
QG_FP32_IR = 1
QG_ORDER_MD = 0
QG_ORDER_ND = 1
QG_STEP_MS_MAX = 256


class QGError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = code
        super().__init__(f"{where}: {ERRORS.get(code, code)}")


class qg_csc(ctypes.Structure):
    _fields_ = [("nrow", ctypes.c_int32), ("ncol", ctypes.c_int32), ("colptr", c_int64_p),
                ("rowind", c_int32_p), ("val", c_double_p)]


class qg_settings(ctypes.Structure):
    _fields_ = [("eps_abs", ctypes.c_double), ("eps_rel", ctypes.c_double), ("eps_inacc", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("precision", ctypes.c_int), ("switch_gap", ctypes.c_double),
                ("static_reg", ctypes.c_double), ("dyn_eps", ctypes.c_double), ("dyn_delta", ctypes.c_double),
                ("static_reg32", ctypes.c_double), ("dyn_eps32", ctypes.c_double),
                ("dyn_delta32", ctypes.c_double), ("ir_max", ctypes.c_int), ("ir_max32", ctypes.c_int),
                ("ir_tol", ctypes.c_double), ("step_frac", ctypes.c_double), ("differentiable", ctypes.c_int),
                ("verbose", ctypes.c_int), ("profile", ctypes.c_int), ("chains", ctypes.c_int),
                ("fp32_min_flops", ctypes.c_double), ("ordering", ctypes.c_int),
                ("cone_lanes", ctypes.c_int), ("tiny_groups", ctypes.c_int), ("graphs", ctypes.c_int),
                ("ruiz_iters", ctypes.c_int)]


class qg_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("switch_iter", ctypes.c_int),
                ("ir_steps", ctypes.c_int), ("nreg", ctypes.c_int), ("nfactor", ctypes.c_int),
                ("nsolve", ctypes.c_int), ("pobj", ctypes.c_double), ("dobj", ctypes.c_double),
                ("pres", ctypes.c_double), ("dres", ctypes.c_double), ("gap", ctypes.c_double),
                ("ms_setup", ctypes.c_double), ("ms_analyze", ctypes.c_double), ("ms_solve", ctypes.c_double),
                ("ms_factor", ctypes.c_double), ("ms_trisolve", ctypes.c_double), ("ms_cone", ctypes.c_double),
                ("ms_step_median", ctypes.c_double), ("ms_step_median_fp32", ctypes.c_double),
                ("ms_step_median_fp64", ctypes.c_double), ("nnz_L", ctypes.c_int64),
                ("factor_flops", ctypes.c_double), ("kern_launches", ctypes.c_int64 * 4),
                ("kern_ms", ctypes.c_double * 4), ("kern_flops", ctypes.c_double * 4),
                ("ms_step_p90", ctypes.c_double), ("ntrisolve", ctypes.c_int64 * 2), ("nresidual", ctypes.c_int64),
                ("nstep_ms", ctypes.c_int32), ("step_fp32", ctypes.c_int32 * QG_STEP_MS_MAX),
                ("step_ms", ctypes.c_double * QG_STEP_MS_MAX)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        for k in ("kern_launches", "kern_ms", "kern_flops", "ntrisolve"):
            d[k] = list(d[k])
        d["step_ms"] = list(d["step_ms"])[:self.nstep_ms]
        d["step_fp32"] = list(d["step_fp32"])[:self.nstep_ms]
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class qg_pattern(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nsuper_fund", ctypes.c_int32), ("nsuper", ctypes.c_int32),
                ("perm", c_int32_p), ("iperm", c_int32_p), ("parent", c_int32_p), ("colcount", c_int64_p),
                ("super_fund", c_int32_p), ("super_ptr", c_int32_p), ("rows_ptr", c_int64_p),
                ("rows", c_int32_p), ("nfront", ctypes.c_int32), ("front_perm", c_int32_p),
                ("front_ptr", c_int32_p), ("front_rows_ptr", c_int64_p), ("front_rows", c_int32_p),
                ("nchain_front", ctypes.c_int32)]


# Device-memory hooks of qg_setup (include/qg.h: qg_alloc_fn, qg_free_fn).
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

EXPORTS = [
    "qg_default_settings", "qg_analyze", "qg_symbolic_pattern", "qg_symbolic_free", "qg_setup", "qg_update",
    "qg_update_vectors", "qg_set_settings", "qg_solve", "qg_backward", "qg_backward_full", "qg_backward_batch", "qg_get_pattern", "qg_last_hip_error", "qg_cleanup",
    "qg_strerror", "qg_step_scaling", "qg_step_get_kkt", "qg_step_factor", "qg_step_get_factor",
    "qg_step_solve", "qg_step_max_step", "qg_step_cone_op", "qg_step_corrector", "qg_max_step_noalloc",
    "qg_setup_batch", "qg_solve_batch",
]
QG_NOALLOC_MAX_UNITS = 4194304

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2603_29197_amd/build.py "
                          "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.qg_default_settings.argtypes = [ctypes.POINTER(qg_settings)]
    L.qg_analyze.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             ctypes.POINTER(qg_csc), ctypes.POINTER(qg_csc), ctypes.POINTER(qg_csc),
                             ctypes.c_int32, ctypes.c_int32, c_int32_p, ctypes.c_int]
    L.qg_symbolic_pattern.argtypes = [vp, ctypes.POINTER(qg_pattern)]
    L.qg_symbolic_free.argtypes = [vp]
    L.qg_symbolic_free.restype = None
    L.qg_setup.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                           ctypes.POINTER(qg_csc), c_double_p, ctypes.POINTER(qg_csc), c_double_p,
                           ctypes.POINTER(qg_csc), c_double_p, ctypes.c_int32, ctypes.c_int32, c_int32_p,
                           ctypes.POINTER(qg_settings), vp, ALLOC_FN, FREE_FN, vp]
    L.qg_setup_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.POINTER(qg_csc), c_double_p, ctypes.POINTER(qg_csc),
                                 c_double_p, ctypes.POINTER(qg_csc), c_double_p, ctypes.c_int32, ctypes.c_int32,
                                 c_int32_p, ctypes.POINTER(qg_settings), vp, ALLOC_FN, FREE_FN, vp]
    L.qg_solve_batch.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(qg_info)]
    L.qg_update.argtypes = [vp, c_double_p, c_double_p, c_double_p, c_double_p, c_double_p, c_double_p]
    L.qg_update_vectors.argtypes = [vp, vp, vp, vp]
    L.qg_set_settings.argtypes = [vp, ctypes.POINTER(qg_settings)]
    L.qg_solve.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(qg_info)]
    L.qg_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.qg_backward_full.argtypes = [vp] * 11
    L.qg_backward_batch.argtypes = [vp, ctypes.c_int32] + [vp] * 10
    L.qg_get_pattern.argtypes = [vp, ctypes.POINTER(qg_pattern)]
    L.qg_last_hip_error.argtypes = [vp]
    L.qg_cleanup.argtypes = [vp]
    L.qg_cleanup.restype = None
    L.qg_strerror.argtypes = [ctypes.c_int]
    L.qg_strerror.restype = ctypes.c_char_p
    L.qg_step_scaling.argtypes = [vp, vp, vp, vp, ctypes.c_int]
    L.qg_step_get_kkt.argtypes = [vp, c_double_p, c_int64_p]
    L.qg_step_factor.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.qg_step_get_factor.argtypes = [vp, c_int64_p, c_int32_p, c_double_p, c_double_p]
    L.qg_step_solve.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    L.qg_step_max_step.argtypes = [vp, vp, vp, c_double_p]
    L.qg_step_cone_op.argtypes = [vp, ctypes.c_int, vp, vp, vp]
    L.qg_step_corrector.argtypes = [vp, vp, vp, ctypes.c_double, vp]
    L.qg_max_step_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, vp, vp, vp, c_double_p, vp]
    _lib = L
    return L


def check(rc: int, where: str) -> None:
    if rc != QG_OK:
        raise QGError(rc, where)
