"""Oracle symbolic analysis of the KKT pattern (paper Sec. 2.2: reordering,
permutation and symbolic factorization, run once per sparsity pattern).

The paper delegates this phase to its sparse solver and fixes no algorithm,
so the integers below follow our own written rule, which the device library
implements independently; the two must agree bit for bit:

 1. graph: off-diagonal pattern of K, both triangles;
 2. dense nodes: degree > max(16, floor(10 sqrt(N))) are set aside and
    ordered last, by increasing index;
 3. minimum degree on the quotient graph with supervariables and the
    approximate (upper-bound) external degree of Amestoy, Davis and Duff
    (rule written out in ``or_min_degree``); or, as the alternative ordering,
    nested dissection by breadth-first level structures with minimum degree
    on its pieces (``nested_dissection``);
 4. postorder of the elimination tree of the minimum-degree order (depth
    first, children and roots by increasing index), composed with it;
 5. elimination tree, column counts and the strictly-lower pattern of L for
    the final permutation, by explicit row-subtree traversal;
 6. fundamental supernodes: j+1 joins j's supernode iff parent[j] = j+1,
    colcount[j] = colcount[j+1] + 1 and j is the only child of j+1;
 7. relaxed supernodes: walking fundamental supernodes in order, the current
    group G is merged with the next supernode T when T holds G's parent
    column and the merged block satisfies  zeros <= 0.1 * stored  or
    (width <= 8 and zeros <= 64), where stored = w*r - w(w-1)/2 with
    r = width(G) + colcount[first(T)], and zeros = stored - sum of colcounts;
 8. row list of each relaxed supernode: the sorted union of the structures of
    its columns (diagonal included).

Test infrastructure only.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from ._clib import lib

ZREL = 0.1          # relaxed-supernode zero fraction
RELAX_W = 8         # small-width clause: width limit ...
RELAX_Z = 64        # ... and absolute zero limit


@dataclass
class Pattern:
    N: int
    perm: np.ndarray        # perm[k] = original index of pivot k
    iperm: np.ndarray       # iperm[perm[k]] = k
    parent: np.ndarray      # etree of the permuted matrix (-1 = root)
    colcount: np.ndarray    # nnz of each column of L incl. diagonal
    super_fund: np.ndarray  # fundamental supernode start columns (+ N)
    super_ptr: np.ndarray   # relaxed supernode start columns (+ N)
    rows_ptr: np.ndarray    # int64, per relaxed supernode offsets into rows
    rows: np.ndarray        # int32, sorted row lists (permuted indices)
    Lp: np.ndarray          # strictly-lower pattern of L (CSC), int64
    Li: np.ndarray          # int32

    @property
    def nnz_L(self) -> int:
        return int(self.colcount.sum())


def dense_cut(N: int) -> int:
    return max(16, int(math.floor(10.0 * math.sqrt(N))))


def sym_graph(Ku: sp.csc_matrix) -> sp.csc_matrix:
    """Off-diagonal pattern of the symmetric matrix with upper triangle Ku."""
    S = sp.csc_matrix((np.ones(Ku.nnz), Ku.indices, Ku.indptr), shape=Ku.shape)
    S = (S + S.T).tocsc()
    S.setdiag(0)
    S.eliminate_zeros()
    S.sort_indices()
    return S


def permute_map(Ku: sp.csc_matrix, perm: np.ndarray):
    """Pattern of the upper triangle of (Pi K Pi'), row/col k being perm[k],
    and pos with Up.data[pos[t]] = Ku.data[t] (pure index arithmetic, so
    explicit zeros keep their place)."""
    N = Ku.shape[0]
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    cols = np.repeat(np.arange(N, dtype=np.int64), np.diff(Ku.indptr))
    a = iperm[Ku.indices.astype(np.int64)]
    b = iperm[cols]
    r, c = np.minimum(a, b), np.maximum(a, b)
    key = c * N + r
    order = np.argsort(key, kind="stable")
    pos = np.empty(len(key), dtype=np.int64)
    pos[order] = np.arange(len(key))
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(c, minlength=N), out=indptr[1:])
    indices = r[order].astype(np.int32)
    return indptr, indices, pos


def permute_upper(Ku: sp.csc_matrix, perm: np.ndarray) -> sp.csc_matrix:
    """Upper triangle of (Pi K Pi') where row/col k of the result is perm[k]."""
    indptr, indices, pos = permute_map(Ku, perm)
    data = np.empty(len(indices))
    data[pos] = Ku.data
    N = Ku.shape[0]
    return sp.csc_matrix((data, indices, indptr), shape=(N, N))


def min_degree(graph: sp.csc_matrix, merge: bool = True, exact: bool = False,
               check: bool = False):
    """Minimum-degree order of ``graph`` (see ``or_min_degree`` for the rule).

    With ``check`` the exact external degree is computed alongside the
    approximate one and the number of updates where the bound fell below it
    is returned as a second value."""
    N = graph.shape[0]
    order = np.empty(N, dtype=np.int32)
    Gp = graph.indptr.astype(np.int64)
    Gi = graph.indices.astype(np.int32)
    chk = ctypes.c_int64(0)
    rc = lib().or_min_degree(N, Gp, Gi, 1 if merge else 0, 1 if exact else 0, order,
                             ctypes.byref(chk) if check else None)
    if rc != 0:
        raise RuntimeError(f"or_min_degree failed ({rc})")
    return (order, int(chk.value)) if check else order


def etree(Up: sp.csc_matrix) -> np.ndarray:
    N = Up.shape[0]
    parent = np.empty(N, dtype=np.int32)
    lib().or_etree(N, Up.indptr.astype(np.int64), Up.indices.astype(np.int32), parent)
    return parent


def postorder(parent: np.ndarray) -> np.ndarray:
    """Depth-first postorder; children and roots visited by increasing index."""
    N = len(parent)
    children = [[] for _ in range(N)]
    roots = []
    for j in range(N):
        (roots if parent[j] < 0 else children[parent[j]]).append(j)
    post = np.empty(N, dtype=np.int64)
    k = 0
    for r in roots:
        stack = [(r, 0)]
        while stack:
            node, ci = stack[-1]
            if ci < len(children[node]):
                stack[-1] = (node, ci + 1)
                stack.append((children[node][ci], 0))
            else:
                stack.pop()
                post[k] = node
                k += 1
    return post


def l_pattern(Up: sp.csc_matrix, parent: np.ndarray):
    """Strictly lower pattern of L by row subtrees; returns (Lp, Li, colcount)."""
    N = Up.shape[0]
    Upp = Up.indptr.astype(np.int64)
    Upi = Up.indices.astype(np.int32)
    cnt = np.zeros(N, dtype=np.int64)
    L = lib()
    L.or_lpattern(N, Upp, Upi, parent, None, cnt, None)
    Lp = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(cnt, out=Lp[1:])
    Li = np.empty(int(Lp[-1]), dtype=np.int32)
    cnt2 = np.zeros(N, dtype=np.int64)
    L.or_lpattern(N, Upp, Upi, parent, Lp.ctypes.data_as(ctypes.c_void_p), cnt2,
                  Li.ctypes.data_as(ctypes.c_void_p))
    return Lp, Li, (cnt + 1).astype(np.int64)


def row_work(Up: sp.csc_matrix, parent: np.ndarray, nrows: int | None = None):
    """Per row k of the up-looking factorization: entries of row k of L (strictly lower) and its
    multiply-add count (see or_row_work); only rows < nrows (default all)."""
    N = Up.shape[0] if nrows is None else int(nrows)
    rowcnt = np.zeros(N, dtype=np.int64)
    rowops = np.zeros(N, dtype=np.float64)
    lib().or_row_work(N, Up.indptr.astype(np.int64), Up.indices.astype(np.int32),
                      np.ascontiguousarray(parent, dtype=np.int32), rowcnt, rowops)
    return rowcnt, rowops


def l_pattern_rows(Up: sp.csc_matrix, parent: np.ndarray, nrows: int):
    """Strictly lower pattern of the leading nrows x nrows block of L (columns and rows < nrows):
    the rows of the row subtrees of rows 0..nrows-1 only; returns (Lp, Li)."""
    Upp = Up.indptr.astype(np.int64)
    Upi = Up.indices.astype(np.int32)
    cnt = np.zeros(nrows, dtype=np.int64)
    L = lib()
    L.or_lpattern(nrows, Upp, Upi, np.ascontiguousarray(parent, dtype=np.int32), None, cnt, None)
    Lp = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(cnt, out=Lp[1:])
    Li = np.empty(int(Lp[-1]), dtype=np.int32)
    cnt2 = np.zeros(nrows, dtype=np.int64)
    L.or_lpattern(nrows, Upp, Upi, np.ascontiguousarray(parent, dtype=np.int32),
                  Lp.ctypes.data_as(ctypes.c_void_p), cnt2, Li.ctypes.data_as(ctypes.c_void_p))
    return Lp, Li


def fundamental_supernodes(parent: np.ndarray, colcount: np.ndarray) -> np.ndarray:
    N = len(parent)
    nchild = np.zeros(N, dtype=np.int64)
    for j in range(N):
        if parent[j] >= 0:
            nchild[parent[j]] += 1
    starts = [0] if N > 0 else []
    for j in range(N - 1):
        joins = parent[j] == j + 1 and colcount[j] == colcount[j + 1] + 1 and nchild[j + 1] == 1
        if not joins:
            starts.append(j + 1)
    starts.append(N)
    return np.array(starts, dtype=np.int32)


def relaxed_supernodes(parent, colcount, sfund) -> np.ndarray:
    ns = len(sfund) - 1
    if ns <= 0:
        return np.array(sfund, dtype=np.int32)
    starts = []
    cf, cl = int(sfund[0]), int(sfund[1]) - 1          # current group [cf, cl]
    csum = int(colcount[cf:cl + 1].sum())
    for s in range(1, ns):
        tf, tl = int(sfund[s]), int(sfund[s + 1]) - 1
        merged = False
        if parent[cl] == tf:
            w = tl - cf + 1
            r = (cl - cf + 1) + int(colcount[tf])
            stored = w * r - w * (w - 1) // 2
            actual = csum + int(colcount[tf:tl + 1].sum())
            zeros = stored - actual
            if zeros <= ZREL * stored or (w <= RELAX_W and zeros <= RELAX_Z):
                cl = tl
                csum = actual
                merged = True
        if not merged:
            starts.append(cf)
            cf, cl = tf, tl
            csum = int(colcount[tf:tl + 1].sum())
    starts.append(cf)
    starts.append(int(sfund[-1]))
    return np.array(starts, dtype=np.int32)


def supernode_rows(sptr, Lp, Li):
    """Row list of each supernode: union of its columns' structures."""
    ns = len(sptr) - 1
    ptr = np.zeros(ns + 1, dtype=np.int64)
    chunks = []
    for s in range(ns):
        f, l = int(sptr[s]), int(sptr[s + 1])
        parts = [np.arange(f, l, dtype=np.int32)] + [Li[Lp[c]:Lp[c + 1]] for c in range(f, l)]
        rows = np.unique(np.concatenate(parts))
        chunks.append(rows.astype(np.int32))
        ptr[s + 1] = ptr[s] + len(rows)
    rows = np.concatenate(chunks) if chunks else np.zeros(0, dtype=np.int32)
    return ptr, rows


ND_LEAF = 256      # nested dissection: pieces of at most this many nodes go to minimum degree


def induced(graph: sp.csc_matrix, S: np.ndarray) -> sp.csc_matrix:
    """Subgraph induced by the ascending node list S; local node i is S[i]."""
    N = graph.shape[0]
    loc = np.full(N, -1, dtype=np.int64)
    loc[S] = np.arange(len(S))
    rows, cols = [], []
    for i, v in enumerate(S):
        nb = loc[graph.indices[graph.indptr[v]:graph.indptr[v + 1]]]
        nb = nb[nb >= 0]
        rows.append(nb)
        cols.append(np.full(len(nb), i, dtype=np.int64))
    r = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, dtype=np.int64)
    sub = sp.csc_matrix((np.ones(len(r)), (r, c)), shape=(len(S), len(S)))
    sub.sort_indices()
    return sub


def bfs_levels(graph: sp.csc_matrix, inside: np.ndarray, root: int) -> list:
    """Breadth-first level structure from ``root`` within the nodes where
    ``inside`` is true: a list of ascending arrays, level 0 = [root]."""
    seen = np.zeros(graph.shape[0], dtype=bool)
    seen[root] = True
    levels = [np.array([root], dtype=np.int64)]
    while True:
        nxt = []
        for v in levels[-1]:
            nb = graph.indices[graph.indptr[v]:graph.indptr[v + 1]]
            nb = nb[inside[nb] & ~seen[nb]]
            seen[nb] = True
            nxt.append(nb)
        nxt = np.sort(np.concatenate(nxt)) if nxt else np.zeros(0, dtype=np.int64)
        if len(nxt) == 0:
            return levels
        levels.append(nxt.astype(np.int64))


def nested_dissection(graph: sp.csc_matrix) -> np.ndarray:
    """Automatic nested dissection by breadth-first level structures (George
    and Liu, Computer Solution of Large Sparse Positive Definite Systems,
    1981, ch. 8) with minimum degree on the small pieces.  ND(S), S ascending:

      a. |S| <= ND_LEAF: minimum degree on the subgraph induced by S;
      b. S not connected: ND of each component, by increasing least node;
      c. level structure from the least node of S; while the node of its
         last level with least (degree within S, index) roots a structure
         with more levels, that one replaces it;
      d. h levels, h < 3: as a; else m = h // 2, separator = nodes of level m
         with a neighbour in level m + 1, A = levels < m and the rest of
         level m, B = levels > m; order ND(A), ND(B), separator ascending.
    """
    N = graph.shape[0]
    out = []

    def leaf(S):
        out.extend(S[min_degree(induced(graph, S))].tolist())

    def nd(S):
        if len(S) == 0:
            return
        if len(S) <= ND_LEAF:
            leaf(S)
            return
        inside = np.zeros(N, dtype=bool)
        inside[S] = True
        levels = bfs_levels(graph, inside, int(S[0]))
        if sum(len(x) for x in levels) < len(S):
            done = np.zeros(N, dtype=bool)
            comps = []
            for v in S:
                if not done[v]:
                    comp = np.sort(np.concatenate(bfs_levels(graph, inside, int(v))))
                    done[comp] = True
                    comps.append(comp)
            for comp in comps:
                nd(comp)
            return
        while True:
            last = levels[-1]
            deg = np.array([np.count_nonzero(inside[graph.indices[graph.indptr[v]:graph.indptr[v + 1]]])
                            for v in last])
            v = int(last[np.lexsort((last, deg))[0]])
            cand = bfs_levels(graph, inside, v)
            if len(cand) > len(levels):
                levels = cand
            else:
                break
        h = len(levels)
        if h < 3:
            leaf(S)
            return
        m = h // 2
        nextlev = np.zeros(N, dtype=bool)
        nextlev[levels[m + 1]] = True
        touches = np.array([nextlev[graph.indices[graph.indptr[v]:graph.indptr[v + 1]]].any()
                            for v in levels[m]], dtype=bool)
        sep = levels[m][touches]
        A = np.sort(np.concatenate(levels[:m] + [levels[m][~touches]]))
        B = np.sort(np.concatenate(levels[m + 1:]))
        nd(A)
        nd(B)
        out.extend(np.sort(sep).tolist())

    nd(np.arange(N, dtype=np.int64))
    return np.array(out, dtype=np.int64)


def order(Ku: sp.csc_matrix, ordering: str = "md") -> np.ndarray:
    """Steps 1-4: the final fill-reducing permutation (perm[k] = original node).
    ``ordering`` "nd" replaces step 3 by ``nested_dissection``."""
    N = Ku.shape[0]
    g = sym_graph(Ku)
    deg = np.diff(g.indptr)
    dense = deg > dense_cut(N)
    keep = np.flatnonzero(~dense)
    sub = g[keep][:, keep].tocsc()
    sub.sort_indices()
    md_sub = nested_dissection(sub) if ordering == "nd" else min_degree(sub)
    md = np.concatenate([keep[md_sub], np.flatnonzero(dense)]).astype(np.int64)
    par = etree(permute_upper(Ku, md))
    post = postorder(par)
    return md[post]


def analyze(Ku: sp.csc_matrix, ordering: str = "md") -> Pattern:
    N = Ku.shape[0]
    perm = order(Ku, ordering)
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    Up = permute_upper(Ku, perm)
    parent = etree(Up)
    Lp, Li, colcount = l_pattern(Up, parent)
    sfund = fundamental_supernodes(parent, colcount)
    sptr = relaxed_supernodes(parent, colcount, sfund)
    rptr, rows = supernode_rows(sptr, Lp, Li)
    return Pattern(N=N, perm=perm.astype(np.int32), iperm=iperm.astype(np.int32), parent=parent,
                   colcount=colcount, super_fund=sfund, super_ptr=sptr, rows_ptr=rptr, rows=rows,
                   Lp=Lp, Li=Li)
