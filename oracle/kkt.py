"""The KKT matrix of the paper's eq. (2), assembled plainly with scipy.

    K = [ P    A'   G'     ]      unknowns ordered [x (n); y (p); z (m)]
        [ A    0    0      ]
        [ G    0   -W'W    ]

Stored as its upper triangle in CSC with sorted rows.  The pattern is fixed
by the problem's sparsity alone (never by values): the whole diagonal is
always present, the (3,3) block holds one diagonal entry per orthant row and
the full upper triangle of a dense q x q block per second-order cone
(eq. 2 shows -W'W; for an SOC it is dense, for the orthant diagonal).

Static regularization (our reading; the paper is silent): +delta on the
(1,1) diagonal and -delta on the (2,2) diagonal make K quasi-definite.

Test infrastructure only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def block33_entries(prob, orth_diag, soc_blocks):
    """COO entries (local row, local col, value) of the upper triangle of the
    (3,3) block: ``orth_diag`` (length l) on the orthant diagonal and, for
    SOC k, the upper triangle of the dense matrix ``soc_blocks[k]``."""
    rows = [np.arange(prob.l)]
    cols = [np.arange(prob.l)]
    vals = [np.asarray(orth_diag, dtype=np.float64)]
    off = prob.l
    for k, qk in enumerate(prob.q):
        iu, ju = np.triu_indices(qk)
        rows.append(off + iu)
        cols.append(off + ju)
        vals.append(np.asarray(soc_blocks[k], dtype=np.float64)[iu, ju])
        off += qk
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def _coo_entries(prob, orth_diag, soc_blocks, delta_x, delta_y):
    """All entries of the upper triangle of K as COO triples, always in the
    same order for a given problem (duplicates allowed: P's diagonal and the
    regularization land on the same position and are summed)."""
    n, p = prob.n, prob.p
    parts_r, parts_c, parts_v = [], [], []
    Pu = sp.triu(prob.P).tocoo()
    parts_r.append(Pu.row); parts_c.append(Pu.col); parts_v.append(Pu.data)
    # full diagonal of the (1,1) and (2,2) blocks
    parts_r.append(np.arange(n)); parts_c.append(np.arange(n)); parts_v.append(np.full(n, float(delta_x)))
    parts_r.append(n + np.arange(p)); parts_c.append(n + np.arange(p)); parts_v.append(np.full(p, -float(delta_y)))
    # A' in rows 0..n-1, columns n..n+p-1 ; G' in columns n+p..
    Ac = prob.A.tocoo()
    parts_r.append(Ac.col); parts_c.append(n + Ac.row); parts_v.append(Ac.data)
    Gc = prob.G.tocoo()
    parts_r.append(Gc.col); parts_c.append(n + p + Gc.row); parts_v.append(Gc.data)
    r3, c3, v3 = block33_entries(prob, orth_diag, soc_blocks)
    parts_r.append(n + p + r3); parts_c.append(n + p + c3); parts_v.append(v3)
    r = np.concatenate(parts_r).astype(np.int64)
    c = np.concatenate(parts_c).astype(np.int64)
    v = np.concatenate(parts_v).astype(np.float64)
    return r, c, v


class KKTAssembler:
    """Fixed upper-CSC pattern of K and the map from COO entries to it."""

    def __init__(self, prob):
        self.prob = prob
        self.N = prob.n + prob.p + prob.m
        r, c, _ = _coo_entries(prob, np.ones(prob.l), [np.ones((qk, qk)) for qk in prob.q], 1.0, 1.0)
        key = c * self.N + r                      # column-major order
        uniq, inv = np.unique(key, return_inverse=True)
        self.map = inv                            # COO entry -> CSC data position
        self.indices = (uniq % self.N).astype(np.int32)
        cols = uniq // self.N
        self.indptr = np.zeros(self.N + 1, dtype=np.int64)
        np.cumsum(np.bincount(cols, minlength=self.N), out=self.indptr[1:])

    def upper(self, orth_diag, soc_blocks, delta_x: float = 0.0, delta_y: float = 0.0) -> sp.csc_matrix:
        _, _, v = _coo_entries(self.prob, orth_diag, soc_blocks, delta_x, delta_y)
        data = np.zeros(len(self.indices))
        np.add.at(data, self.map, v)
        return sp.csc_matrix((data, self.indices.copy(), self.indptr.copy()), shape=(self.N, self.N))


def kkt_upper(prob, orth_diag, soc_blocks, delta_x: float = 0.0, delta_y: float = 0.0) -> sp.csc_matrix:
    """Upper triangle of K (eq. 2) with the given (3,3) block and static
    regularization; explicit zeros are kept so the pattern never depends on
    values."""
    return KKTAssembler(prob).upper(orth_diag, soc_blocks, delta_x, delta_y)


def kkt_pattern(prob) -> sp.csc_matrix:
    """The fixed upper-triangular pattern of K (values all 1)."""
    A = KKTAssembler(prob)
    return sp.csc_matrix((np.ones(len(A.indices)), A.indices, A.indptr), shape=(A.N, A.N))


def full_from_upper(Ku: sp.csc_matrix) -> sp.csr_matrix:
    """Both triangles of the symmetric matrix whose upper triangle is Ku."""
    return (Ku + sp.triu(Ku, k=1).T).tocsr()


def pivot_signs(prob) -> np.ndarray:
    """Expected sign of each pivot of the quasi-definite K: + for x, - for y and z."""
    return np.concatenate([np.ones(prob.n), -np.ones(prob.p + prob.m)]).astype(np.int8)
