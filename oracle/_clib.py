"""Builds and loads the oracle's C core (``oracle/csrc/oracle.c``) with ctypes.

Test infrastructure only: the product library never loads this.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile the oracle's C core with gcc (always recompiles)."""
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build()
    L = ctypes.CDLL(_SO)
    L.or_min_degree.argtypes = [ctypes.c_int32, i64p, i32p, ctypes.c_int32, ctypes.c_int32, i32p,
                                ctypes.POINTER(ctypes.c_int64)]
    L.or_min_degree.restype = ctypes.c_int
    L.or_etree.argtypes = [ctypes.c_int32, i64p, i32p, i32p]
    L.or_etree.restype = ctypes.c_int
    L.or_lpattern.argtypes = [ctypes.c_int32, i64p, i32p, i32p, ctypes.c_void_p, i64p, ctypes.c_void_p]
    L.or_lpattern.restype = ctypes.c_int
    L.or_row_work.argtypes = [ctypes.c_int32, i64p, i32p, i32p, i64p, f64p]
    L.or_ldl_numeric_rows_marked.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, i64p, i32p, f64p,
                                             i32p, i64p, i32p, i8p, ctypes.c_double, ctypes.c_double, f64p,
                                             f64p, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    L.or_ldl_numeric_rows_marked.restype = ctypes.c_int
    L.or_row_work.restype = ctypes.c_int
    L.or_ldl_numeric.argtypes = [ctypes.c_int32, i64p, i32p, f64p, i32p, i64p, i32p, i8p,
                                 ctypes.c_double, ctypes.c_double, f64p, f64p,
                                 ctypes.POINTER(ctypes.c_int64)]
    L.or_ldl_numeric.restype = ctypes.c_int
    L.or_ldl_numeric_rows.argtypes = [ctypes.c_int32, ctypes.c_int32, i64p, i32p, f64p, i32p, i64p, i32p,
                                      i8p, ctypes.c_double, ctypes.c_double, f64p, f64p,
                                      ctypes.POINTER(ctypes.c_int64)]
    L.or_ldl_numeric_rows.restype = ctypes.c_int
    L.or_ldl_solve.argtypes = [ctypes.c_int32, i64p, i32p, f64p, f64p, f64p]
    L.or_ldl_solve.restype = ctypes.c_int
    _lib = L
    return L
