"""Pins of the oracle's symbolic analysis against brute force and closed forms.

The elimination tree, column counts and L pattern are fixed by the matrix
alone; they are checked against dense boolean symbolic elimination.  The
ordering rule is checked (i) in its exact/no-merge form against brute-force
minimum degree on the explicit elimination graph, (ii) in its product form
for the upper-bound property of the approximate degree, and (iii) on graphs
whose order is known in closed form.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import kkt, symbolic
from synth import problems


def random_sym_upper(N, density, seed):
    rng = np.random.default_rng(seed)
    M = sp.random(N, N, density=density, random_state=rng, format="csc")
    U = sp.triu(M + M.T, k=1) + sp.identity(N)
    U = sp.csc_matrix(U)
    U.data[:] = 1.0
    U.sort_indices()
    return U


def brute_symbolic(Up):
    """Dense boolean elimination: returns (L pattern as bool matrix, parent, colcount)."""
    N = Up.shape[0]
    A = Up.toarray() != 0
    A = A | A.T
    np.fill_diagonal(A, True)
    L = np.zeros((N, N), dtype=bool)
    for j in range(N):
        col = A[j:, j].copy()
        L[j:, j] = col
        nz = np.flatnonzero(col) + j
        nz = nz[nz > j]
        for a in nz:                      # fill: clique among the remaining neighbours
            A[nz, a] = True
    parent = np.full(N, -1)
    for j in range(N):
        below = np.flatnonzero(L[j + 1:, j])
        if below.size:
            parent[j] = j + 1 + below[0]
    return L, parent, L.sum(axis=0)


def brute_md(G):
    """Plain minimum degree on the explicit elimination graph, ties to the smallest index."""
    N = G.shape[0]
    adj = [set(G.indices[G.indptr[i]:G.indptr[i + 1]].tolist()) - {i} for i in range(N)]
    alive = set(range(N))
    order = []
    while alive:
        p = min(alive, key=lambda v: (len(adj[v]), v))
        order.append(p)
        nb = adj[p]
        for u in nb:
            adj[u] |= nb
            adj[u].discard(u)
            adj[u].discard(p)
        alive.remove(p)
        adj[p] = set()
    return np.array(order)


@pytest.mark.parametrize("seed", range(12))
def test_etree_colcount_lpattern_vs_brute_force(seed):
    N = 20 + 7 * seed
    U = random_sym_upper(N, 0.06, seed)
    parent = symbolic.etree(U)
    Lp, Li, colcount = symbolic.l_pattern(U, parent)
    Lb, pb, cb = brute_symbolic(U)
    assert np.array_equal(parent, pb)
    assert np.array_equal(colcount, cb)
    for j in range(N):
        assert np.array_equal(Li[Lp[j]:Lp[j + 1]], np.flatnonzero(Lb[j + 1:, j]) + j + 1)


@pytest.mark.parametrize("seed", range(10))
def test_exact_md_without_merging_is_brute_force_md(seed):
    N = 25 + 5 * seed
    U = random_sym_upper(N, 0.08, 100 + seed)
    g = symbolic.sym_graph(U)
    got = symbolic.min_degree(g, merge=False, exact=True)
    assert np.array_equal(got, brute_md(g))


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "many_soc_s"])
def test_approximate_degree_is_an_upper_bound(name):
    prob = problems.workload(name)
    g = symbolic.sym_graph(kkt.kkt_pattern(prob))
    order, below = symbolic.min_degree(g, check=True)
    assert below == 0
    assert np.array_equal(np.sort(order), np.arange(g.shape[0]))


def test_md_closed_forms():
    # clique K_n: every node has degree n-1; node 0 is picked, the rest become
    # one supervariable (represented by node 1) and are eliminated in order.
    n = 9
    K = sp.csc_matrix(np.ones((n, n)) - np.eye(n))
    assert np.array_equal(symbolic.min_degree(K), np.arange(n))
    # path 0-1-2-...-7: the leaves have degree 1; node 0 goes first, which
    # leaves node 1 as the new leaf, and so on down the path.
    n = 8
    P = sp.diags([np.ones(n - 1), np.ones(n - 1)], [-1, 1], shape=(n, n), format="csc")
    assert np.array_equal(symbolic.min_degree(P), np.arange(n))
    # star with centre 0 and leaves 1..6: leaves (degree 1) go first while the
    # centre's degree (leaves left) exceeds 1; with one leaf left the centre
    # ties at degree 1 and wins on index.
    S = sp.lil_matrix((7, 7))
    for i in range(1, 7):
        S[0, i] = S[i, 0] = 1
    assert np.array_equal(symbolic.min_degree(S.tocsc()), [1, 2, 3, 4, 5, 0, 6])
    # disconnected nodes (degree 0) are taken first, by index
    D = sp.csc_matrix((5, 5))
    assert np.array_equal(symbolic.min_degree(D), np.arange(5))


def _check_postorder(parent):
    N = len(parent)
    # every node comes after all its descendants and subtrees are contiguous
    first = np.arange(N)
    for j in range(N):
        if parent[j] >= 0:
            assert parent[j] > j
            first[parent[j]] = min(first[parent[j]], first[j])
    for j in range(N):
        if parent[j] >= 0:
            assert first[parent[j]] <= first[j]


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "many_soc_s"])
def test_analysis_invariants_on_kkt_patterns(name):
    prob = problems.workload(name)
    Kp = kkt.kkt_pattern(prob)
    pat = symbolic.analyze(Kp)
    N = pat.N
    assert np.array_equal(np.sort(pat.perm), np.arange(N))
    assert np.array_equal(pat.iperm[pat.perm], np.arange(N))
    _check_postorder(pat.parent)
    # dense nodes (none in these workloads) would come last
    # fundamental supernodes: nested structures and single-child chains
    sf = pat.super_fund
    for s in range(len(sf) - 1):
        for j in range(sf[s], sf[s + 1] - 1):
            a = pat.Li[pat.Lp[j]:pat.Lp[j + 1]]
            b = pat.Li[pat.Lp[j + 1]:pat.Lp[j + 2]]
            assert a[0] == j + 1 and np.array_equal(a[1:], b)
    # relaxed supernodes refine nothing: every fundamental boundary not merged stays
    assert set(pat.super_ptr.tolist()) <= set(sf.tolist())
    # row lists: own columns first, then sorted rows below, and the rule
    for s in range(len(pat.super_ptr) - 1):
        f, l = pat.super_ptr[s], pat.super_ptr[s + 1]
        rows = pat.rows[pat.rows_ptr[s]:pat.rows_ptr[s + 1]]
        assert np.array_equal(rows[:l - f], np.arange(f, l))
        assert np.all(np.diff(rows) > 0)
        # structure of the last column equals the rows at and below it
        last = pat.Li[pat.Lp[l - 1]:pat.Lp[l]]
        assert np.array_equal(rows[l - f:], last)


def test_counts_and_row_lists_on_brute_force_pattern():
    prob = problems.workload("small_qp")
    Kp = kkt.kkt_pattern(prob)
    pat = symbolic.analyze(Kp)
    Up = symbolic.permute_upper(Kp, pat.perm)
    Lb, pb, cb = brute_symbolic(Up)
    assert np.array_equal(pat.parent, pb)
    assert np.array_equal(pat.colcount, cb)
    sptr = pat.super_ptr
    for s in range(len(sptr) - 1):
        f, l = sptr[s], sptr[s + 1]
        union = np.flatnonzero(Lb[:, f:l].any(axis=1))
        assert np.array_equal(pat.rows[pat.rows_ptr[s]:pat.rows_ptr[s + 1]], union)


def test_kkt_pattern_matches_dense_eq2():
    prob = problems.many_soc(n=30, ncones=4, q=3, nbounds=5, seed=7)
    n, p, m = prob.n, prob.p, prob.m
    Pd = prob.P.toarray(); Pd = Pd + np.triu(Pd, 1).T
    rng = np.random.default_rng(0)
    orth = -rng.uniform(1, 2, prob.l)
    blocks = []
    for qk in prob.q:
        B = rng.standard_normal((qk, qk)); blocks.append(-(B @ B.T) - np.eye(qk))
    H = np.zeros((m, m))
    H[:prob.l, :prob.l] = np.diag(orth)
    off = prob.l
    for qk, B in zip(prob.q, blocks):
        H[off:off + qk, off:off + qk] = B
        off += qk
    A = prob.A.toarray(); G = prob.G.toarray()
    Kd = np.block([[Pd + 1e-3 * np.eye(n), A.T, G.T],
                   [A, -1e-3 * np.eye(p), np.zeros((p, m))],
                   [G, np.zeros((m, p)), H]])
    Ku = kkt.kkt_upper(prob, orth, blocks, 1e-3, 1e-3)
    assert np.allclose(np.triu(Kd), Ku.toarray(), rtol=0, atol=1e-15)
    # the pattern holds every diagonal entry and every SOC block entry
    pat = kkt.kkt_pattern(prob).toarray() != 0
    assert np.all(np.diag(pat))


def test_dense_nodes_are_ordered_last():
    # an arrow matrix: node 0 touches everything -> dense when N is large enough
    N = 300
    rows = np.concatenate([np.zeros(N - 1, dtype=int), np.arange(N)])
    cols = np.concatenate([np.arange(1, N), np.arange(N)])
    U = sp.csc_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N))
    U.sort_indices()
    assert symbolic.dense_cut(N) < N - 1
    perm = symbolic.order(U)
    assert perm[-1] == 0


def _relax_ok(rows_of_group, cols, colcount):
    """The relaxation test on a candidate block: explicit zeros of its stored lower trapezoid,
    counted from the union of the columns' row sets (brute force, not the colcount formula)."""
    w = len(cols)
    r = len(rows_of_group)
    stored = w * r - w * (w - 1) // 2
    zeros = stored - int(sum(colcount[c] for c in cols))
    return zeros <= symbolic.ZREL * stored or (w <= symbolic.RELAX_W and zeros <= symbolic.RELAX_Z)


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "many_soc_s", "rand"])
def test_relaxed_supernodes_are_the_greedy_partition(name):
    """The relaxed partition is pinned by two properties that determine a greedy left-to-right
    grouping uniquely: every extension of a group's prefix by its next fundamental supernode
    passes the test (T holds the parent of the prefix's last column, zeros within bounds), and
    every group boundary fails it.  Row sets come from the explicit L pattern."""
    if name == "rand":
        Ku = random_sym_upper(150, 0.03, 5)
    else:
        Ku = kkt.kkt_pattern(problems.workload(name))
    pat = symbolic.analyze(Ku)
    cc, par = pat.colcount, pat.parent
    struct = [set([j]) | set(pat.Li[pat.Lp[j]:pat.Lp[j + 1]].tolist()) for j in range(pat.N)]

    def extends(group_cols, t_cols):
        if par[group_cols[-1]] != t_cols[0]:
            return False
        cols = list(group_cols) + list(t_cols)
        rows = set().union(*(struct[c] for c in cols))
        return _relax_ok(rows, cols, cc)

    sf = pat.super_fund.tolist()
    fund = [list(range(sf[s], sf[s + 1])) for s in range(len(sf) - 1)]
    start_of = {f[0]: k for k, f in enumerate(fund)}
    sp_ = pat.super_ptr.tolist()
    merges = 0
    for g in range(len(sp_) - 1):
        k0, k1 = start_of[sp_[g]], start_of.get(sp_[g + 1], len(fund))
        group = list(fund[k0])
        for k in range(k0 + 1, k1):
            assert extends(group, fund[k]), (g, k)
            group += fund[k]
            merges += 1
        if k1 < len(fund):
            assert not extends(group, fund[k1]), (g, k1)
    assert merges > 0


# ----------------------------------------------------------------------------------------------
# nested dissection
# ----------------------------------------------------------------------------------------------
def path_graph(N):
    i = np.arange(N - 1)
    return symbolic.sym_graph(sp.csc_matrix((np.ones(N - 1), (i, i + 1)), shape=(N, N)))


def grid_graph(k):
    """k x k grid, node i*k + j, 4-neighbour edges."""
    r, c = [], []
    for i in range(k):
        for j in range(k):
            v = i * k + j
            if j + 1 < k:
                r.append(v); c.append(v + 1)
            if i + 1 < k:
                r.append(v); c.append(v + k)
    return symbolic.sym_graph(sp.csc_matrix((np.ones(len(r)), (r, c)), shape=(k * k, k * k)))


def etree_height(graph, order):
    """Height of the elimination tree of the graph's matrix in the given order."""
    N = graph.shape[0]
    pos = np.empty(N, dtype=np.int64)
    pos[order] = np.arange(N)
    G = graph.tocoo()
    keep = pos[G.row] < pos[G.col]
    U = sp.csc_matrix((np.ones(int(keep.sum())), (pos[G.row[keep]], pos[G.col[keep]])), shape=(N, N))
    U = (U + sp.identity(N)).tocsc()
    U.sort_indices()
    parent = symbolic.etree(U)
    h = np.zeros(N, dtype=np.int64)
    for j in range(N):
        if parent[j] >= 0:
            h[parent[j]] = max(h[parent[j]], h[j] + 1)
    return int(h.max()), parent


def test_nd_on_a_path_is_recursive_bisection():
    """On the path 0-1-...-(N-1) the level structure from node 0 is the path itself (the far end
    roots no longer one), so each piece [a, b) splits at its middle node a + (b-a)//2, which is
    ordered after both halves; pieces of at most ND_LEAF nodes are paths ordered by minimum
    degree."""
    def expected(a, b):
        n = b - a
        if n == 0:
            return []
        if n <= symbolic.ND_LEAF:
            return [a + int(i) for i in symbolic.min_degree(path_graph(n))]
        m = n // 2
        return expected(a, a + m) + expected(a + m + 1, b) + [a + m]

    for N in (257, 600, 3001):
        got = symbolic.nested_dissection(path_graph(N))
        assert got.tolist() == expected(0, N)


def test_nd_balanced_tree_on_a_path(monkeypatch):
    """With pieces of one node, the path of 2^t - 1 nodes is cut into halves t - 1 times: its
    elimination tree is the complete binary tree of height t - 1 with 2^(t-1) leaves (pieces of
    two nodes have fewer than 3 levels and go to minimum degree: a 2-node chain)."""
    monkeypatch.setattr(symbolic, "ND_LEAF", 1)
    t = 10
    N = 2 ** t - 1
    g = path_graph(N)
    order = symbolic.nested_dissection(g)
    assert sorted(order.tolist()) == list(range(N))
    h, parent = etree_height(g, order)
    assert h == t - 1
    nchild = np.bincount(parent[parent >= 0], minlength=N)
    assert int(np.count_nonzero(nchild == 0)) == 2 ** (t - 1)
    # minimum degree on the same path gives a deeper tree
    assert etree_height(g, symbolic.min_degree(g))[0] > h


def test_nd_grid_top_separator_is_the_antidiagonal():
    """k x k grid with k*k > ND_LEAF: the levels from corner 0 are the anti-diagonals i + j = d
    (the opposite corner roots as many, 2k - 1), so the middle level is i + j = k - 1, every node
    of which touches the next level: it is the separator, ordered last; the two triangles before
    it are pieces of k(k-1)/2 <= ND_LEAF nodes, each ordered by minimum degree."""
    k = 20
    g = grid_graph(k)
    order = symbolic.nested_dissection(g)
    ij = [(v // k, v % k) for v in range(k * k)]
    A = np.array([v for v, (i, j) in enumerate(ij) if i + j < k - 1])
    B = np.array([v for v, (i, j) in enumerate(ij) if i + j > k - 1])
    sep = np.array([v for v, (i, j) in enumerate(ij) if i + j == k - 1])
    gA = g[A][:, A].tocsc(); gA.sort_indices()
    gB = g[B][:, B].tocsc(); gB.sort_indices()
    want = np.concatenate([A[symbolic.min_degree(gA)], B[symbolic.min_degree(gB)], sep])
    assert order.tolist() == want.tolist()


def test_nd_top_split_from_distances(monkeypatch):
    """Random connected graphs, top level re-derived from all-pairs distances (scipy's
    unweighted shortest paths) instead of level structures: the root is walked to a node of
    greater eccentricity as the rule says, the separator is the distance-m shell's nodes with a
    neighbour at distance m + 1, and the order is A's nodes, then B's, then the separator
    ascending; no edge joins A and B."""
    monkeypatch.setattr(symbolic, "ND_LEAF", 8)
    from scipy.sparse.csgraph import shortest_path
    for seed in range(8):
        rng = np.random.default_rng(300 + seed)
        N = 60 + 15 * seed
        U = random_sym_upper(N, 1.5 / N, 300 + seed).tolil()
        chain = rng.permutation(N)                      # a Hamiltonian path keeps it connected
        for a, b in zip(chain[:-1], chain[1:]):
            U[min(a, b), max(a, b)] = 1.0
        U = sp.csc_matrix(U)
        g = symbolic.sym_graph(U)
        D = shortest_path(g, unweighted=True)
        deg = np.diff(g.indptr)
        r = 0
        while True:
            far = np.flatnonzero(D[r] == D[r].max())
            v = int(far[np.lexsort((far, deg[far]))[0]])
            if D[v].max() > D[r].max():
                r = v
            else:
                break
        h = int(D[r].max()) + 1
        m = h // 2
        shell = np.flatnonzero(D[r] == m)
        sep = np.array([v for v in shell
                        if np.any(D[r][g.indices[g.indptr[v]:g.indptr[v + 1]]] == m + 1)])
        A = np.setdiff1d(np.flatnonzero(D[r] <= m), sep)
        B = np.flatnonzero(D[r] > m)
        order = symbolic.nested_dissection(g)
        assert sorted(order.tolist()) == list(range(N))
        assert sorted(order[:len(A)].tolist()) == A.tolist()
        assert sorted(order[len(A):len(A) + len(B)].tolist()) == B.tolist()
        assert order[len(A) + len(B):].tolist() == sep.tolist()
        Gd = g.toarray() != 0
        assert not Gd[np.ix_(A, B)].any()


def test_nd_reduces_tree_height_on_a_band():
    """A long band (windowed many-SOC pattern): nested dissection's elimination tree is far
    shallower than minimum degree's, which follows the band."""
    prob = problems.many_soc(n=6000, ncones=2000, q=4, nbounds=2000, seed=77)
    Ku = kkt.kkt_pattern(prob)
    pm = symbolic.analyze(Ku)
    pn = symbolic.analyze(Ku, "nd")
    hm = etree_height(symbolic.sym_graph(Ku), pm.perm)[0]
    hn = etree_height(symbolic.sym_graph(Ku), pn.perm)[0]
    assert hn * 2 < hm
