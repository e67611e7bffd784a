"""Seeded synthetic problem generators for problem (1) of the paper (Sec. 1).

Each generator returns a :class:`Problem` holding the data of

    minimize 1/2 x'Px + c'x   s.t.  h - Gx in K,  Ax = b

exactly as the paper states it (Sec. 1, eq. 1): P is given as its upper
triangle (the paper's size count uses nnz of the upper half of P, Sec. 3),
A is p x n, G is m x n, and the cone K is described by ``l`` (dimension of
the nonnegative orthant, whose rows come first), ``nsoc`` and ``q`` (the
second-order cone dimensions, in row order after the orthant).

This module draws inputs only.  It holds none of the solver's arithmetic:
the products used here (b = A x0, h = G x0 + s0, the lasso weight) only place
a known feasible point inside the cone so that every instance is feasible
and bounded, as the paper assumes (Sec. 1).  Both the oracle and the device
path consume these problems; neither is imported here.

Density rule: "density d" means exactly round(d * rows * cols) distinct
positions drawn uniformly without replacement, each with an N(0, 1) value.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

BASE_SEED = 29197


@dataclass
class Problem:
    n: int
    m: int
    p: int
    P: sp.csc_matrix          # n x n, upper triangle incl. diagonal (may have no entries)
    c: np.ndarray             # n
    A: sp.csc_matrix          # p x n
    b: np.ndarray             # p
    G: sp.csc_matrix          # m x n
    h: np.ndarray             # m
    l: int                    # orthant dimension (rows 0..l-1 of G)
    q: List[int] = field(default_factory=list)   # SOC dimensions, rows after the orthant
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nsoc(self) -> int:
        return len(self.q)

    @property
    def size(self) -> int:
        """Problem size as the paper counts it: nnz(A) + nnz(G) + nnz(triu(P))."""
        return int(self.A.nnz + self.G.nnz + self.P.nnz)

    def check(self) -> None:
        assert self.P.shape == (self.n, self.n)
        assert self.A.shape == (self.p, self.n)
        assert self.G.shape == (self.m, self.n)
        assert self.c.shape == (self.n,) and self.b.shape == (self.p,) and self.h.shape == (self.m,)
        assert self.l + sum(self.q) == self.m
        assert all(qk >= 1 for qk in self.q)
        Pc = self.P.tocoo()
        assert np.all(Pc.row <= Pc.col), "P must be upper triangular"


def _csc(M) -> sp.csc_matrix:
    """Canonical CSC: sorted row indices, no duplicates, no explicit zeros."""
    M = sp.csc_matrix(M)
    M.sum_duplicates()
    M.eliminate_zeros()
    M.sort_indices()
    return M


def random_sparse(rng: np.random.Generator, rows: int, cols: int, density: float) -> sp.csc_matrix:
    """Exactly round(density*rows*cols) distinct uniform positions with N(0,1) values."""
    k = int(round(density * rows * cols))
    pos = rng.choice(rows * cols, size=k, replace=False)
    vals = rng.standard_normal(k)
    r = (pos // cols).astype(np.int64)
    cc = (pos % cols).astype(np.int64)
    return _csc(sp.coo_matrix((vals, (r, cc)), shape=(rows, cols)))


def random_sparse_per_row(rng: np.random.Generator, rows: int, cols: int, per_row: int) -> sp.csc_matrix:
    """Each row gets exactly ``per_row`` distinct uniform columns with N(0,1) values."""
    cidx = np.empty((rows, per_row), dtype=np.int64)
    for i in range(rows):
        cidx[i] = rng.choice(cols, size=per_row, replace=False)
    vals = rng.standard_normal(rows * per_row)
    r = np.repeat(np.arange(rows, dtype=np.int64), per_row)
    return _csc(sp.coo_matrix((vals, (r, cidx.ravel())), shape=(rows, cols)))


# --------------------------------------------------------------------------------------
# Workload 1: small dense-ish QP (n=200, p=50, m=200 orthant)
# --------------------------------------------------------------------------------------
def small_qp(seed: int = BASE_SEED + 1, n: int = 200, p: int = 50, m: int = 200,
             mrows: int = 100, density: float = 0.1) -> Problem:
    rng = np.random.default_rng(seed)
    M = random_sparse(rng, mrows, n, density)
    P = (M.T @ M + 0.01 * sp.identity(n)).tocsc()
    A = random_sparse(rng, p, n, density)
    G = random_sparse(rng, m, n, density)
    x0 = rng.standard_normal(n)
    s0 = rng.uniform(0.1, 1.0, m)
    b = A @ x0
    h = G @ x0 + s0
    c = rng.standard_normal(n)
    prob = Problem(n=n, m=m, p=p, P=_csc(sp.triu(P)), c=c, A=A, b=b, G=G, h=h, l=m, q=[],
                   name=f"small_qp_n{n}", meta=dict(seed=seed))
    prob.check()
    return prob


# --------------------------------------------------------------------------------------
# Workload 2 / 5: lasso as a sparse QP, variables (x, y, t)
#   minimize 1/2||y||^2 + lam 1't  s.t.  y = F x - g,  -t <= x <= t
# --------------------------------------------------------------------------------------
def lasso(rows: int = 20000, cols: int = 10000, density: float = 0.005,
          seed: int = BASE_SEED + 2, sparsity: float = 0.01, noise: float = 0.01) -> Problem:
    rng = np.random.default_rng(seed)
    F = random_sparse(rng, rows, cols, density)
    k = max(1, int(round(sparsity * cols)))
    x_true = np.zeros(cols)
    support = rng.choice(cols, size=k, replace=False)
    x_true[support] = rng.standard_normal(k)
    g = F @ x_true + noise * rng.standard_normal(rows)
    lam = 0.1 * float(np.max(np.abs(F.T @ g)))
    nx, ny, nt = cols, rows, cols
    n = nx + ny + nt
    I_y = sp.identity(ny, format="csc")
    I_x = sp.identity(nx, format="csc")
    P = sp.block_diag([sp.csc_matrix((nx, nx)), I_y, sp.csc_matrix((nt, nt))], format="csc")
    c = np.concatenate([np.zeros(nx), np.zeros(ny), lam * np.ones(nt)])
    A = sp.hstack([F, -I_y, sp.csc_matrix((rows, nt))], format="csc")
    b = g.copy()
    G = sp.hstack([sp.vstack([I_x, -I_x]), sp.csc_matrix((2 * nx, ny)),
                   sp.vstack([-I_x, -I_x])], format="csc")
    h = np.zeros(2 * nx)
    prob = Problem(n=n, m=2 * nx, p=rows, P=_csc(P), c=c, A=_csc(A), b=b, G=_csc(G), h=h,
                   l=2 * nx, q=[], name=f"lasso_{rows}x{cols}_d{density}",
                   meta=dict(seed=seed, lam=lam, F_nnz=int(F.nnz), x_true=x_true))
    prob.check()
    return prob


# --------------------------------------------------------------------------------------
# Workload 3: many small second-order cones ||F_i x + g_i|| <= d_i'x + e_i, plus bounds
# --------------------------------------------------------------------------------------
def many_soc(n: int = 300000, ncones: int = 100000, q=4, nbounds: int = 100000,
             seed: int = BASE_SEED + 3, windowed: bool = True, per_row: int = 2,
             window: int = 12) -> Problem:
    """``q`` is one cone dimension for all ``ncones`` cones, or a list of
    dimensions (one per cone; ``ncones`` is then ignored)."""
    qs = [int(q)] * ncones if np.isscalar(q) else [int(v) for v in q]
    ncones = len(qs)
    offs = np.concatenate([[0], np.cumsum(qs)]).astype(np.int64)
    rng = np.random.default_rng(seed)
    x0 = rng.standard_normal(n)
    Pdiag = rng.uniform(0.1, 1.0, n)
    c = rng.standard_normal(n)
    rows_i, cols_i, vals_i = [], [], []
    h_soc = np.empty(int(offs[-1]))
    for i in range(ncones):
        q_i = qs[i]
        nf = q_i - 1
        base = int(offs[i])
        if windowed:
            pool = (3 * i + np.arange(window)) % n
        else:
            pool = None
        # row 0 of the cone: t-row  (-d_i' x, h = e_i)
        # rows 1..q-1: (-F_i x, h = g_i)
        Fcols = []
        for r in range(nf):
            cols = rng.choice(pool, size=per_row, replace=False) if windowed else \
                rng.choice(n, size=per_row, replace=False)
            Fcols.append(cols)
        dcols = rng.choice(pool, size=per_row, replace=False) if windowed else \
            rng.choice(n, size=per_row, replace=False)
        Fvals = rng.standard_normal((nf, per_row))
        dvals = rng.standard_normal(per_row)
        gi = rng.standard_normal(nf)
        Fx0 = np.array([Fvals[r] @ x0[Fcols[r]] for r in range(nf)])
        ei = np.linalg.norm(Fx0 + gi) - dvals @ x0[dcols] + rng.uniform(0.1, 1.0)
        rows_i.append(np.full(per_row, base)); cols_i.append(dcols); vals_i.append(-dvals)
        for r in range(nf):
            rows_i.append(np.full(per_row, base + 1 + r)); cols_i.append(Fcols[r]); vals_i.append(-Fvals[r])
        h_soc[base] = ei
        h_soc[base + 1:base + q_i] = gi
    Gsoc = sp.coo_matrix((np.concatenate(vals_i), (np.concatenate(rows_i), np.concatenate(cols_i))),
                         shape=(int(offs[-1]), n))
    bidx = np.sort(rng.choice(n, size=nbounds, replace=False))
    slack = rng.uniform(0.1, 1.0, nbounds)
    Gb = sp.coo_matrix((-np.ones(nbounds), (np.arange(nbounds), bidx)), shape=(nbounds, n))
    hb = slack - x0[bidx]
    G = sp.vstack([Gb, Gsoc], format="csc")
    h = np.concatenate([hb, h_soc])
    P = sp.diags(Pdiag, format="csc")
    qname = f"q{qs[0]}" if np.isscalar(q) else f"qmix{max(qs)}"
    prob = Problem(n=n, m=nbounds + int(offs[-1]), p=0, P=_csc(P), c=c,
                   A=_csc(sp.csc_matrix((0, n))), b=np.zeros(0), G=_csc(G), h=h,
                   l=nbounds, q=list(qs),
                   name=f"many_soc_n{n}_k{ncones}_{qname}{'' if windowed else '_random'}",
                   meta=dict(seed=seed, windowed=windowed))
    prob.check()
    return prob


# --------------------------------------------------------------------------------------
# Workload 4: Huber-style regression, variables (x, u, v, w)
#   minimize 1/2||u||^2 + 1'w  s.t.  F x - u - v = g,  -w <= v <= w
# --------------------------------------------------------------------------------------
def huber(rows: int = 500000, cols: int = 200000, per_row: int = 40,
          seed: int = BASE_SEED + 4, outlier_frac: float = 0.05) -> Problem:
    rng = np.random.default_rng(seed)
    F = random_sparse_per_row(rng, rows, cols, per_row)
    x_true = rng.standard_normal(cols)
    g = F @ x_true + rng.standard_normal(rows)
    nout = int(round(outlier_frac * rows))
    oi = rng.choice(rows, size=nout, replace=False)
    g[oi] += rng.choice([-1.0, 1.0], size=nout) * rng.uniform(5.0, 10.0, nout)
    nx, nu = cols, rows
    n = nx + 3 * nu
    I_u = sp.identity(nu, format="csc")
    Z = lambda r, c_: sp.csc_matrix((r, c_))
    P = sp.block_diag([Z(nx, nx), I_u, Z(nu, nu), Z(nu, nu)], format="csc")
    c = np.concatenate([np.zeros(nx + 2 * nu), np.ones(nu)])
    A = sp.hstack([F, -I_u, -I_u, Z(rows, nu)], format="csc")
    G = sp.bmat([[Z(nu, nx), Z(nu, nu), I_u, -I_u], [Z(nu, nx), Z(nu, nu), -I_u, -I_u]], format="csc")
    prob = Problem(n=n, m=2 * nu, p=rows, P=_csc(P), c=c, A=_csc(A), b=g, G=_csc(G),
                   h=np.zeros(2 * nu), l=2 * nu, q=[],
                   name=f"huber_{rows}x{cols}_r{per_row}", meta=dict(seed=seed))
    prob.check()
    return prob


# --------------------------------------------------------------------------------------
# Named workloads at full size and at oracle-scale
# --------------------------------------------------------------------------------------
def workload(name: str) -> Problem:
    """Named workloads: the five full-size configurations and their scaled variants."""
    table = {
        "small_qp": lambda: small_qp(),
        "lasso": lambda: lasso(),
        "many_soc": lambda: many_soc(),
        "huber": lambda: huber(),
        "lasso_diff": lambda: lasso(50000, 20000, 0.002, seed=BASE_SEED + 5),
        # the largest Huber instance of the same generator used in the device tests (the full one
        # needs a ~2e5-wide dense root front: more than one GPU's memory)
        "huber_m": lambda: huber(50000, 20000, 40, seed=BASE_SEED + 4),
        # the benchmark's Huber instance: the same generator at F 100000 x 40000 (40 entries per row)
        "huber_l": lambda: huber(100000, 40000, 40, seed=BASE_SEED + 4),
        # oracle-scaled variants drawn from the same generators
        "lasso_s": lambda: lasso(2000, 1000, 0.02, seed=BASE_SEED + 12),
        "many_soc_s": lambda: many_soc(3000, 1000, 4, 1000, seed=BASE_SEED + 13),
        "huber_s": lambda: huber(10000, 4000, 40, seed=BASE_SEED + 14),
        "huber_t": lambda: huber(2500, 1000, 40, seed=BASE_SEED + 17),
        "lasso_diff_s": lambda: lasso(2500, 1000, 0.016, seed=BASE_SEED + 15),
        # large second-order cones: 3000 of 64 entries, 300 of 256, 30 of 1024 (m = 304520)
        "big_cones": lambda: many_soc(20000, q=[64] * 3000 + [256] * 300 + [1024] * 30, nbounds=5000,
                                      seed=BASE_SEED + 16),
    }
    return table[name]()


def family(prob: Problem, k: int, seed: int) -> List[Problem]:
    """k problems on the sparsity pattern of ``prob`` with drawn values (a parametric family):
    P scaled by U(0.5, 1.5) (stays positive semidefinite), every entry of A and G multiplied by
    1 + 0.05 N(0,1), c + 0.1 N(0,1); b and h from a fresh point x0 ~ N(0,1) and slack s0 strictly
    inside the cones (orthant U(0.1, 1); each SOC (|u| + U(0.1, 1), u), u ~ N(0,1)), so each
    problem is feasible.  Problem 0 is drawn like the others (it is not ``prob`` itself)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        P = prob.P.copy()
        P.data = P.data * rng.uniform(0.5, 1.5)
        A = prob.A.copy()
        A.data = A.data * (1.0 + 0.05 * rng.standard_normal(A.nnz))
        G = prob.G.copy()
        G.data = G.data * (1.0 + 0.05 * rng.standard_normal(G.nnz))
        c = prob.c + 0.1 * rng.standard_normal(prob.n)
        x0 = rng.standard_normal(prob.n)
        s0 = np.empty(prob.m)
        s0[:prob.l] = rng.uniform(0.1, 1.0, prob.l)
        off = prob.l
        for qk in prob.q:
            u = rng.standard_normal(qk - 1)
            s0[off] = np.linalg.norm(u) + rng.uniform(0.1, 1.0)
            s0[off + 1:off + qk] = u
            off += qk
        out.append(Problem(n=prob.n, m=prob.m, p=prob.p, P=P, c=c, A=A, b=A @ x0, G=G, h=G @ x0 + s0,
                           l=prob.l, q=list(prob.q), name=f"{prob.name}_family{i}", meta=dict(seed=seed, index=i)))
    return out


def random_point(prob: Problem, seed: int):
    """A strictly interior (s, z) pair and random (x, y) for step-level tests.

    Orthant entries are U(0.5, 2); each SOC block is (t, u) with u ~ N(0,1) and
    t = ||u|| + U(0.5, 2), so both s and z lie in the interior of K.
    """
    rng = np.random.default_rng(seed)

    def interior():
        v = np.empty(prob.m)
        v[:prob.l] = rng.uniform(0.5, 2.0, prob.l)
        off = prob.l
        for qk in prob.q:
            u = rng.standard_normal(qk - 1)
            v[off] = np.linalg.norm(u) + rng.uniform(0.5, 2.0)
            v[off + 1:off + qk] = u
            off += qk
        return v

    x = rng.standard_normal(prob.n)
    y = rng.standard_normal(prob.p)
    s = interior()
    z = interior()
    return x, s, y, z
