"""Oracle factor/solve of the KKT system (paper Sec. 2.2, eq. 2): one LDL'
factorization per interior-point iteration, solves reusing it, and FP64
iterative refinement against the unregularized matrix.

Regularization (our reading; the paper is silent): the factored matrix is
K + diag(+delta 1_n, -delta 1_p, 0_m), which is quasi-definite so that LDL'
exists for any symmetric permutation without pivoting; a pivot whose sign
disagrees with the expected one (+ for x, - for y and z) or whose magnitude
is at most ``dyn_eps`` is replaced by sign * ``dyn_delta``.

Iterative refinement (our reading): x0 = solve(r); for k < ir_max:
res = r - K x_k with the unregularized K; stop when
||res||_inf <= ir_tol (1 + ||r||_inf); else x_{k+1} = x_k + solve(res).

Test infrastructure only.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from ._clib import lib
from . import kkt as _kkt
from . import symbolic as _sym


@dataclass
class RegSettings:
    static_reg: float = 1e-8
    dyn_eps: float = 1e-13
    dyn_delta: float = 1e-7
    ir_max: int = 3
    ir_tol: float = 1e-12


class KKTFactor:
    """Symbolic analysis once per pattern; numeric LDL' per call to factor()."""

    def __init__(self, prob, pattern: _sym.Pattern | None = None, reg: RegSettings | None = None):
        self.prob = prob
        self.reg = reg or RegSettings()
        self.asm = _kkt.KKTAssembler(prob)
        self.Kpat = _kkt.kkt_pattern(prob)
        self.pat = pattern if pattern is not None else _sym.analyze(self.Kpat)
        self.Up_indptr, self.Up_indices, self.Up_pos = _sym.permute_map(self.Kpat, self.pat.perm)
        self.N = self.pat.N
        self.sign_perm = _kkt.pivot_signs(prob)[self.pat.perm].astype(np.int8)
        self.Lx = np.zeros(len(self.pat.Li))
        self.D = np.zeros(self.N)
        self.K_unreg = None
        self.nreg = 0
        self.nfactor = 0
        self.nsolve = 0

    def factor(self, orth_diag, soc_blocks):
        """Factor K with (3,3) block given by ``orth_diag`` (orthant diagonal,
        the -W'W entries) and ``soc_blocks`` (dense -W'W per SOC)."""
        r = self.reg
        Kreg = self.asm.upper(orth_diag, soc_blocks, r.static_reg, r.static_reg)
        self.K_upper_unreg = self.asm.upper(orth_diag, soc_blocks, 0.0, 0.0)
        self.K_unreg = _kkt.full_from_upper(self.K_upper_unreg)
        Upx = np.empty(len(self.Up_indices))
        Upx[self.Up_pos] = Kreg.data
        nreg = ctypes.c_int64(0)
        rc = lib().or_ldl_numeric(self.N, self.Up_indptr, self.Up_indices,
                                  Upx, self.pat.parent, self.pat.Lp, self.pat.Li,
                                  self.sign_perm, r.dyn_eps, r.dyn_delta, self.Lx, self.D,
                                  ctypes.byref(nreg))
        if rc != 0:
            raise FloatingPointError(f"oracle LDL failed ({rc})")
        self.nreg = int(nreg.value)
        self.nfactor += 1

    def solve_factor(self, rhs: np.ndarray) -> np.ndarray:
        """x = Pi' L^-T D^-1 L^-1 Pi rhs (no refinement)."""
        x = np.ascontiguousarray(rhs[self.pat.perm], dtype=np.float64)
        lib().or_ldl_solve(self.N, self.pat.Lp, self.pat.Li, self.Lx, self.D, x)
        out = np.empty_like(x)
        out[self.pat.perm] = x
        return out

    def solve(self, rhs: np.ndarray, ir_max: int | None = None):
        """Solve the unregularized K x = rhs with refinement; returns (x, steps)."""
        ir_max = self.reg.ir_max if ir_max is None else ir_max
        self.nsolve += 1
        x = self.solve_factor(rhs)
        bnd = self.reg.ir_tol * (1.0 + np.max(np.abs(rhs), initial=0.0))
        steps = 0
        for _ in range(ir_max):
            res = rhs - self.K_unreg @ x
            if np.max(np.abs(res), initial=0.0) <= bnd:
                break
            x = x + self.solve_factor(res)
            steps += 1
        return x, steps

    def L_dense(self) -> np.ndarray:
        """Unit lower L as a dense array (permuted ordering), for small tests."""
        N = self.N
        L = np.eye(N)
        for j in range(N):
            for u in range(self.pat.Lp[j], self.pat.Lp[j + 1]):
                L[self.pat.Li[u], j] = self.Lx[u]
        return L
