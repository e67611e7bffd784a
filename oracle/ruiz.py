"""Oracle Ruiz equilibration of the problem data (a preprocessing that the paper does not state;
the library offers it as an option, and this module is what its scaled data are checked against).

Scaled problem, with positive diagonal D (n), E (p), F (m) and a scalar k > 0:

    minimize 1/2 x^'(k D P D) x^ + (k D c)'x^  s.t.  (F h) - (F G D) x^ in K,  (E A D) x^ = (E b)

whose solution maps back as x = D x^, y = E y^ / k, z = F z^ / k, s = s^ / F.  F is constant on
each second-order cone, so F K = K.

Each pass takes the data matrix M = [P A' G'; A 0 0; G 0 0] as scaled so far (P as the full
symmetric matrix) and multiplies D_j by 1/sqrt of the largest magnitude in column j of its x part,
E_i and F_i by 1/sqrt of the largest magnitude in row i of A D and G D; the rows of one
second-order cone all take the largest of their rows' values (an all-zero column or row keeps its
factor).  After the passes k = 1 / max(1, |D c|_inf).

Dense FP64 numpy, for the small problems of the tests.  Test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def _inv_sqrt(v):
    out = np.ones_like(v)
    pos = v > 0
    out[pos] = 1.0 / np.sqrt(v[pos])
    return out


def equilibrate(prob, passes: int):
    """D, E, F, k after `passes` passes."""
    n, p, m = prob.n, prob.p, prob.m
    Pu = prob.P.toarray()
    Pf = Pu + Pu.T - np.diag(np.diag(Pu))
    A = prob.A.toarray().reshape(p, n)
    G = prob.G.toarray().reshape(m, n)
    D, E, F = np.ones(n), np.ones(p), np.ones(m)
    for _ in range(passes):
        Ps = np.abs(D[:, None] * Pf * D[None, :])
        As = np.abs(E[:, None] * A * D[None, :])
        Gs = np.abs(F[:, None] * G * D[None, :])
        col = np.max(np.vstack([Ps, As, Gs]), axis=0) if n > 0 else np.zeros(0)
        rowA = As.max(axis=1) if n > 0 else np.zeros(p)
        rowG = Gs.max(axis=1) if n > 0 else np.zeros(m)
        off = prob.l
        for q in prob.q:
            rowG[off:off + q] = rowG[off:off + q].max()
            off += q
        D = D * _inv_sqrt(col)
        E = E * _inv_sqrt(rowA)
        F = F * _inv_sqrt(rowG)
    k = 1.0 / max(1.0, float(np.max(np.abs(D * prob.c), initial=0.0)))
    return D, E, F, k


def _scale(M, r, c):
    """diag(r) M diag(c) on M's own pattern and entry order."""
    M = M.tocsc(copy=True)
    cols = np.repeat(np.arange(M.shape[1]), np.diff(M.indptr))
    M.data = r[M.indices] * M.data * c[cols]
    return M


def scaled_problem(prob, D, E, F, k):
    """The problem with the scaled data (the same patterns, P kept as its upper triangle)."""
    import copy
    q = copy.copy(prob)
    q.P = _scale(prob.P, k * D, D)
    q.c = k * D * prob.c
    q.A = _scale(prob.A, E, D)
    q.b = E * prob.b
    q.G = _scale(prob.G, F, D)
    q.h = F * prob.h
    return q


def unscale(D, E, F, k, x, s, y, z):
    """The original problem's (x, s, y, z) from the scaled problem's."""
    return D * x, s / F, E * y / k, F * z / k
