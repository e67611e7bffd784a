"""Oracle cone algebra on K = C_1 x ... x C_K (paper Sec. 1 and Sec. 2.1:
Jordan products, projection onto K and Nesterov-Todd scalings, computed per
cone).  Orthant rows come first (``l`` of them), then second-order cones of
dimensions ``q`` in row order.

Notation (standard Jordan algebra of the second-order cone, Alizadeh and
Goldfarb 2003; NT scaling as in Vandenberghe 2010, the paper's reference for
its interior-point method):

  SOC  C = {u = (u0, u1) : u0 >= ||u1||},  J = diag(1, -I),  e = (1, 0, ..., 0)
  orthant: u o v = (u_i v_i), e = 1
  SOC:     u o v = (u'v, u0 v1 + v0 u1)
  lambda \\ v (the x with lambda o x = v):
     orthant x_i = v_i / lambda_i
     SOC     rho = lambda0^2 - ||lambda1||^2,
             x0 = (lambda0 v0 - lambda1'v1) / rho,  x1 = (v1 - x0 lambda1) / lambda0
  NT scaling W with W'W z = s and lambda = W z = W^-T s:
     orthant w_i = sqrt(s_i / z_i), lambda_i = sqrt(s_i z_i)
     SOC     s_n = sqrt(s'Js), z_n = sqrt(z'Jz), sb = s/s_n, zb = z/z_n,
             gamma = sqrt((1 + zb'sb)/2), wb = (sb + J zb) / (2 gamma),
             beta = sqrt(s_n / z_n),  W = beta * Wb with
             Wb = [[wb0, wb1'], [wb1, I + wb1 wb1'/(1 + wb0)]],
             W'W = W^2 = beta^2 (2 wb wb' - J),  W^-1 = (1/beta) J Wb J.
     The J-norms are computed as sqrt((u0 - ||u1||)(u0 + ||u1||)).

Everything is FP64 numpy, vectorised over all cones of one dimension.

Test infrastructure only.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List

import numpy as np


class Cones:
    def __init__(self, l: int, q: List[int]):
        self.l = int(l)
        self.q = [int(x) for x in q]
        self.m = self.l + sum(self.q)
        self.nu = self.l + len(self.q)           # degree of the cone
        offs = []
        off = self.l
        for qk in self.q:
            offs.append(off)
            off += qk
        self.offsets = np.array(offs, dtype=np.int64)
        # group second-order cones by dimension: index matrices (k x q)
        self.groups: Dict[int, np.ndarray] = {}
        self.group_cones: Dict[int, np.ndarray] = {}
        for qd in sorted(set(self.q)):
            ks = np.array([k for k, qk in enumerate(self.q) if qk == qd], dtype=np.int64)
            self.group_cones[qd] = ks
            self.groups[qd] = self.offsets[ks][:, None] + np.arange(qd)[None, :]

    # --- elementary pieces ---------------------------------------------------
    def identity(self) -> np.ndarray:
        e = np.zeros(self.m)
        e[:self.l] = 1.0
        e[self.offsets] = 1.0
        return e

    def lambda_min(self, u: np.ndarray) -> np.ndarray:
        """Per-cone minimum eigenvalue: u_i (orthant), u0 - ||u1|| (SOC)."""
        out = [u[:self.l]]
        vals = np.empty(len(self.q))
        for qd, idx in self.groups.items():
            U = u[idx]
            vals[self.group_cones[qd]] = U[:, 0] - np.linalg.norm(U[:, 1:], axis=1)
        out.append(vals)
        return np.concatenate(out)

    def jordan(self, u: np.ndarray, v: np.ndarray) -> np.ndarray:
        out = np.empty(self.m)
        out[:self.l] = u[:self.l] * v[:self.l]
        for qd, idx in self.groups.items():
            U, V = u[idx], v[idx]
            R = np.empty_like(U)
            R[:, 0] = np.sum(U * V, axis=1)
            R[:, 1:] = U[:, :1] * V[:, 1:] + V[:, :1] * U[:, 1:]
            out[idx] = R
        return out

    def inv_jordan(self, lam: np.ndarray, v: np.ndarray) -> np.ndarray:
        """lam \\ v : the x with lam o x = v."""
        out = np.empty(self.m)
        out[:self.l] = v[:self.l] / lam[:self.l]
        for qd, idx in self.groups.items():
            Lm, V = lam[idx], v[idx]
            rho = Lm[:, 0] ** 2 - np.sum(Lm[:, 1:] ** 2, axis=1)
            x0 = (Lm[:, 0] * V[:, 0] - np.sum(Lm[:, 1:] * V[:, 1:], axis=1)) / rho
            X = np.empty_like(V)
            X[:, 0] = x0
            X[:, 1:] = (V[:, 1:] - x0[:, None] * Lm[:, 1:]) / Lm[:, :1]
            out[idx] = X
        return out

    # --- maximum step --------------------------------------------------------
    def max_step_per_cone(self, u: np.ndarray, du: np.ndarray) -> np.ndarray:
        """sup{a >= 0 : u + a du in C_k} for each cone (inf when unbounded).

        Orthant: -u_i/du_i when du_i < 0.  SOC (u interior): with
        uJ = sqrt(u'Ju), ub = u/uJ, rho0 = ub'J du / uJ and
        rho1 = (du1 - ((rho0 uJ + du0) / (1 + ub0)) ub1) / uJ, the step is
        1 / max(0, ||rho1|| - rho0)  (Wb(ub) maps e to ub and preserves C, so
        u + a du in C  iff  e + a rho in C)."""
        out = np.empty(self.l + len(self.q))
        ul, dl = u[:self.l], du[:self.l]
        with np.errstate(divide="ignore", invalid="ignore"):
            out[:self.l] = np.where(dl < 0, -ul / dl, np.inf)
        for qd, idx in self.groups.items():
            U, D = u[idx], du[idx]
            n1 = np.linalg.norm(U[:, 1:], axis=1)
            uJ = np.sqrt((U[:, 0] - n1) * (U[:, 0] + n1))
            Ub = U / uJ[:, None]
            rho0 = (Ub[:, 0] * D[:, 0] - np.sum(Ub[:, 1:] * D[:, 1:], axis=1)) / uJ
            coef = (rho0 * uJ + D[:, 0]) / (1.0 + Ub[:, 0])
            rho1 = (D[:, 1:] - coef[:, None] * Ub[:, 1:]) / uJ[:, None]
            den = np.linalg.norm(rho1, axis=1) - rho0
            with np.errstate(divide="ignore"):
                a = np.where(den > 0, 1.0 / np.where(den > 0, den, 1.0), np.inf)
            out[self.l + self.group_cones[qd]] = a
        return out

    def max_step(self, u: np.ndarray, du: np.ndarray) -> float:
        a = self.max_step_per_cone(u, du)
        return float(np.min(a)) if a.size else np.inf

    # --- interior shift (initial point) --------------------------------------
    def shift_interior(self, u: np.ndarray) -> np.ndarray:
        """alpha = -min_k lambda_min(u_k); keep u if alpha < 0, else u + (1 + alpha) e."""
        lm = self.lambda_min(u)
        if lm.size == 0:
            return u.copy()
        alpha = -float(np.min(lm))
        if alpha < 0:
            return u.copy()
        return u + (1.0 + alpha) * self.identity()


@dataclass
class NTScaling:
    cones: Cones
    w: np.ndarray                                   # orthant: sqrt(s/z)
    wbar: Dict[int, np.ndarray] = field(default_factory=dict)   # per group: (k, q)
    beta: Dict[int, np.ndarray] = field(default_factory=dict)   # per group: (k,)
    lam: np.ndarray = None

    def _wb_apply(self, WB, X):
        """Wb X row-wise for a group (hyperbolic reflection form)."""
        w0 = WB[:, 0]
        w1 = WB[:, 1:]
        x0 = X[:, 0]
        x1 = X[:, 1:]
        R = np.empty_like(X)
        R[:, 0] = w0 * x0 + np.sum(w1 * x1, axis=1)
        R[:, 1:] = x1 + w1 * (x0 + np.sum(w1 * x1, axis=1) / (1.0 + w0))[:, None]
        return R

    def W(self, v: np.ndarray) -> np.ndarray:
        c = self.cones
        out = np.empty(c.m)
        out[:c.l] = self.w * v[:c.l]
        for qd, idx in c.groups.items():
            out[idx] = self.beta[qd][:, None] * self._wb_apply(self.wbar[qd], v[idx])
        return out

    def Winv(self, v: np.ndarray) -> np.ndarray:
        """W^-1 = (1/beta) J Wb J on each SOC (W is symmetric, so W^-T = W^-1)."""
        c = self.cones
        out = np.empty(c.m)
        out[:c.l] = v[:c.l] / self.w
        for qd, idx in c.groups.items():
            X = v[idx].copy()
            X[:, 1:] *= -1.0
            R = self._wb_apply(self.wbar[qd], X)
            R[:, 1:] *= -1.0
            out[idx] = R / self.beta[qd][:, None]
        return out

    def WtW(self, v: np.ndarray) -> np.ndarray:
        return self.W(self.W(v))

    def block33(self):
        """(3,3) block of eq. (2): -W'W as (orthant diagonal, dense SOC blocks
        in cone order)."""
        c = self.cones
        orth = -(self.w ** 2)
        blocks = [None] * len(c.q)
        for qd, idx in c.groups.items():
            WB = self.wbar[qd]
            Jm = np.diag(np.concatenate([[1.0], -np.ones(qd - 1)]))
            for t, k in enumerate(c.group_cones[qd]):
                wb = WB[t]
                blocks[k] = -(self.beta[qd][t] ** 2) * (2.0 * np.outer(wb, wb) - Jm)
        return orth, blocks


def _jnorm(U: np.ndarray) -> np.ndarray:
    n1 = np.linalg.norm(U[:, 1:], axis=1)
    return np.sqrt((U[:, 0] - n1) * (U[:, 0] + n1))


def nt_scaling(cones: Cones, s: np.ndarray, z: np.ndarray) -> NTScaling:
    sc = NTScaling(cones=cones, w=np.sqrt(s[:cones.l] / z[:cones.l]))
    lam = np.empty(cones.m)
    lam[:cones.l] = np.sqrt(s[:cones.l] * z[:cones.l])
    for qd, idx in cones.groups.items():
        S, Z = s[idx], z[idx]
        sn, zn = _jnorm(S), _jnorm(Z)
        Sb, Zb = S / sn[:, None], Z / zn[:, None]
        gamma = np.sqrt((1.0 + np.sum(Zb * Sb, axis=1)) / 2.0)
        JZb = Zb.copy()
        JZb[:, 1:] *= -1.0
        WB = (Sb + JZb) / (2.0 * gamma[:, None])
        sc.wbar[qd] = WB
        sc.beta[qd] = np.sqrt(sn / zn)
    sc.lam = sc.W(z) if cones.q else lam
    sc.lam[:cones.l] = lam[:cones.l]
    return sc
