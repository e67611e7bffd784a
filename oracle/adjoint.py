"""Oracle gradients of a loss L(x*) with respect to the problem data, by
implicit differentiation of the KKT conditions of problem (1).

Our reading (the paper itself has no differentiation).  At the final iterate
(x, s, y, z) the optimality conditions of problem (1) are

    Px + A'y + G'z + c = 0,   Ax = b,   Gx + s = h,   s o z = 0

(o the Jordan product).  Their linearisation, with ds eliminated through
the linearised complementarity  Arw(z) ds + Arw(s) dz = 0  (Arw(u) the
arrow matrix of u: u_i on the orthant, [[u0, u1'], [u1, u0 I]] on an SOC),
is

    K_fin [dx; dy; dz] = [-dc - dP x - dA'y - dG'z; db - dA x; dh - dG x],
    K_fin = [[P, A', G'], [A, 0, 0], [G, 0, -H]],   H = Arw(z)^-1 Arw(s),

i.e. eq. (2) with -W'W replaced by -H: H = s_i/z_i on the orthant (which is
W'W at the final iterate) and, per SOC, the symmetric part of
Arw(z)^-1 Arw(s) (s and z nearly operator-commute at the final iterate, so
the skew part is of the order of the duality gap).  The NT-scaled Newton
block W'W would not do for second-order cones: it linearises the scaled
complementarity (W^-T s) o (W z), whose sensitivities differ from those of
s o z at boundary solutions.

K_fin is factored once after convergence (FP64, same pattern as every
Newton step) and reused by every backward call.  For g = dL/dx*, solve
K_fin u = [g; 0; 0] (K_fin is symmetric); then

    dL/dc = -u_x,  dL/db = u_y,  dL/dh = u_z,
    dL/dP_ij = -(u_x,i x_j + u_x,j x_i)  (i < j),   dL/dP_ii = -u_x,i x_i

on the stored upper pattern of P, and on the patterns of A and G (from
dL = u'[rhs] with the dA and dG terms above)

    dL/dA_ij = -(y_i u_x,j + u_y,i x_j),   dL/dG_ij = -(z_i u_x,j + u_z,i x_j).

A loss of the whole solution L(x*, y*, z*, s*) enters through g = [g_x; g_y;
g_z] and g_s: the primal equality gives ds = dh - G dx - dG x exactly, so
g_s' ds = g_s' dh - (G' g_s)' dx - g_s' dG x; with u solving
K_fin u = [g_x - G' g_s; g_y; g_z] the formulas above hold, plus g_s in
dL/dh and -g_s,i x_j in dL/dG_ij.

``backward`` uses the sparse factorization with FP64 refinement;
``backward_dense`` forms K_fin densely and calls numpy's dense solver.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np

from . import kkt as _kkt
from .cones import Cones
from .ldl import KKTFactor


def arrow_inv_times_arrow(z: np.ndarray, s: np.ndarray) -> np.ndarray:
    """Arw(z)^-1 Arw(s) for one SOC, with the closed-form inverse
    Arw(z)^-1 = (1/d) [[z0, -z1'], [-z1, (d/z0) I + z1 z1'/z0]], d = z0^2 - |z1|^2."""
    q = len(z)
    z0, z1 = z[0], z[1:]
    d = z0 * z0 - z1 @ z1
    Ai = np.empty((q, q))
    Ai[0, 0] = z0
    Ai[0, 1:] = -z1
    Ai[1:, 0] = -z1
    Ai[1:, 1:] = (d / z0) * np.eye(q - 1) + np.outer(z1, z1) / z0
    Ai /= d
    As = s[0] * np.eye(q)
    As[0, 1:] = s[1:]
    As[1:, 0] = s[1:]
    return Ai @ As


def final_block(prob, s, z):
    """(3,3) block -H of K_fin: orthant diagonal and dense SOC blocks."""
    cn = Cones(prob.l, prob.q)
    orth = -(s[:prob.l] / z[:prob.l])
    blocks = []
    for k, off in enumerate(cn.offsets):
        q = cn.q[k]
        H = arrow_inv_times_arrow(z[off:off + q], s[off:off + q])
        blocks.append(-0.5 * (H + H.T))
    return orth, blocks


def final_factor(prob, result) -> KKTFactor:
    if getattr(result, "_final_factor", None) is None:
        F = KKTFactor(prob, pattern=result.factor.pat, reg=result.factor.reg)
        F.factor(*final_block(prob, result.s, result.z))
        result._final_factor = F
    return result._final_factor


def _grads(prob, x, y, z, u, gs=None):
    n, p = prob.n, prob.p
    ux, uy, uz = u[:n], u[n:n + p], u[n + p:]
    if gs is not None:
        uz = uz + gs                 # ds = dh - G dx - dG x: g_s joins u_z in dL/dh and dL/dG
    Pu = prob.P.tocoo()              # tocoo() of a CSC matrix keeps the CSC entry order
    dP = np.where(Pu.row == Pu.col, -ux[Pu.row] * x[Pu.col],
                  -(ux[Pu.row] * x[Pu.col] + ux[Pu.col] * x[Pu.row]))
    Au, Gu = prob.A.tocoo(), prob.G.tocoo()
    dA = -(y[Au.row] * ux[Au.col] + uy[Au.row] * x[Au.col])
    dG = -(z[Gu.row] * ux[Gu.col] + uz[Gu.row] * x[Gu.col])
    return dict(dc=-ux, db=uy.copy(), dh=uz.copy(), dP=dP, dA=dA, dG=dG, u=u)


def _rhs(prob, g, gy, gz, gs):
    gx = np.asarray(g, dtype=float)
    if gs is not None:
        gx = gx - prob.G.T @ gs
    return np.concatenate([gx, np.zeros(prob.p) if gy is None else gy, np.zeros(prob.m) if gz is None else gz])


def backward(prob, result, g, ir_max: int = 10, gy=None, gz=None, gs=None):
    """Adjoint solve on the stored final factorization (+ FP64 refinement);
    g = dL/dx*, and optionally gy, gz, gs = dL/dy*, dL/dz*, dL/ds*."""
    F = final_factor(prob, result)
    u, _ = F.solve(_rhs(prob, g, gy, gz, gs), ir_max=ir_max)
    return _grads(prob, result.x, result.y, result.z, u, gs)


def backward_dense(prob, result, g, gy=None, gz=None, gs=None):
    """Same gradients from a dense FP64 solve with K_fin."""
    orth, blocks = final_block(prob, result.s, result.z)
    K = _kkt.full_from_upper(_kkt.kkt_upper(prob, orth, blocks)).toarray()
    u = np.linalg.solve(K, _rhs(prob, g, gy, gz, gs))
    return _grads(prob, result.x, result.y, result.z, u, gs)
