"""Pins of the oracle interior-point method and its gradients on problems with
closed-form answers (projections, box-constrained diagonal QP, SOCPs with a
known optimum, tiny LPs solved by vertex enumeration) and on the optimality
invariants; gradients against closed forms, a dense KKT solve, a dot-product
test and central finite differences.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import adjoint, ipm
from oracle.cones import Cones
from synth import problems
from synth.problems import Problem, _csc


def mkprob(P, c, A, b, G, h, l, q):
    n = len(c)
    return Problem(n=n, m=G.shape[0], p=A.shape[0], P=_csc(sp.triu(sp.csc_matrix(P))),
                   c=np.asarray(c, float), A=_csc(sp.csc_matrix(A)), b=np.asarray(b, float),
                   G=_csc(sp.csc_matrix(G)), h=np.asarray(h, float), l=l, q=list(q))


def soc_proj(v):
    v0, v1 = v[0], v[1:]
    nv = np.linalg.norm(v1)
    if nv <= v0:
        return v.copy()
    if nv <= -v0:
        return np.zeros_like(v)
    return 0.5 * (v0 + nv) * np.r_[1.0, v1 / nv]


def assert_optimal(prob, r):
    assert r.status == ipm.SOLVED
    cn = Cones(prob.l, prob.q)
    assert np.all(cn.lambda_min(r.s) > 0) and np.all(cn.lambda_min(r.z) > 0)
    assert r.pres <= 1e-7 and r.dres <= 1e-7


@pytest.mark.parametrize("case", ["inside", "polar", "between"])
def test_soc_projection(case):
    # min 1/2||x - v||^2  s.t. x in SOC   (P = I, c = -v, G = -I, h = 0)
    q = 5
    rng = np.random.default_rng(1)
    v = rng.standard_normal(q)
    v1n = np.linalg.norm(v[1:])
    v[0] = {"inside": 1.5 * v1n, "polar": -1.5 * v1n, "between": 0.3 * v1n}[case]
    prob = mkprob(np.eye(q), -v, np.zeros((0, q)), [], -np.eye(q), np.zeros(q), 0, [q])
    r = ipm.solve(prob)
    assert_optimal(prob, r)
    assert np.allclose(r.x, soc_proj(v), atol=1e-6)


def test_orthant_and_product_projection():
    rng = np.random.default_rng(2)
    v = rng.standard_normal(10)
    q = [4, 3]
    n = 3 + sum(q)
    prob = mkprob(np.eye(n), -v, np.zeros((0, n)), [], -np.eye(n), np.zeros(n), 3, q)
    r = ipm.solve(prob)
    assert_optimal(prob, r)
    want = np.r_[np.maximum(v[:3], 0), soc_proj(v[3:7]), soc_proj(v[7:])]
    assert np.allclose(r.x, want, atol=1e-6)


def box_qp(seed, n=12):
    rng = np.random.default_rng(seed)
    d = rng.uniform(0.5, 3.0, n)
    c = rng.standard_normal(n) * 2
    lo = -rng.uniform(0.2, 1.0, n)
    hi = rng.uniform(0.2, 1.0, n)
    G = np.vstack([np.eye(n), -np.eye(n)])
    h = np.r_[hi, -lo]
    return mkprob(np.diag(d), c, np.zeros((0, n)), [], G, h, 2 * n, []), d, c, lo, hi


@pytest.mark.parametrize("seed", range(3))
def test_box_constrained_diagonal_qp(seed):
    prob, d, c, lo, hi = box_qp(seed)
    r = ipm.solve(prob)
    assert_optimal(prob, r)
    assert np.allclose(r.x, np.clip(-c / d, lo, hi), atol=1e-6)


def test_socp_unit_ball():
    # min c'x s.t. ||x|| <= 1  ->  x* = -c/||c||;  rows: (1, x) in SOC => G = [0; -I], h = [1; 0]
    rng = np.random.default_rng(3)
    n = 6
    c = rng.standard_normal(n)
    G = np.vstack([np.zeros((1, n)), -np.eye(n)])
    h = np.r_[1.0, np.zeros(n)]
    prob = mkprob(np.zeros((n, n)), c, np.zeros((0, n)), [], G, h, 0, [n + 1])
    r = ipm.solve(prob)
    assert_optimal(prob, r)
    assert np.allclose(r.x, -c / np.linalg.norm(c), atol=1e-6)


def test_least_norm_residual_socp():
    # min t s.t. ||F x - g|| <= t  ->  x* = least-squares solution, t* = residual norm
    rng = np.random.default_rng(4)
    F = rng.standard_normal((9, 4))
    g = rng.standard_normal(9)
    n = 5                                   # (x, t)
    c = np.r_[np.zeros(4), 1.0]
    G = np.vstack([np.r_[np.zeros(4), -1.0], np.hstack([-F, np.zeros((9, 1))])])
    h = np.r_[0.0, -g]
    prob = mkprob(np.zeros((n, n)), c, np.zeros((0, n)), [], G, h, 0, [10])
    r = ipm.solve(prob)
    assert_optimal(prob, r)
    xls = np.linalg.lstsq(F, g, rcond=None)[0]
    assert np.allclose(r.x[:4], xls, atol=1e-6)
    assert np.isclose(r.x[4], np.linalg.norm(F @ xls - g), atol=1e-6)


def lp_vertices(c, A, b, G, h):
    """Brute force: every choice of n - p active inequality rows."""
    n, p = len(c), A.shape[0]
    best = []
    for rows in itertools.combinations(range(G.shape[0]), n - p):
        M = np.vstack([A, G[list(rows)]])
        rhs = np.r_[b, h[list(rows)]]
        if abs(np.linalg.det(M)) < 1e-9:
            continue
        x = np.linalg.solve(M, rhs)
        if np.all(G @ x <= h + 1e-9):
            best.append((c @ x, tuple(np.round(x, 12))))
    best.sort()
    return best


@pytest.mark.parametrize("seed", range(40))
def test_tiny_lps_vs_vertex_enumeration(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 5))
    p = int(rng.integers(0, 2))
    m = int(rng.integers(n + 2, 9))
    # bounded feasible region: box plus random cuts through an interior point
    x0 = rng.standard_normal(n)
    Gc = rng.standard_normal((m - 2 * n, n)) if m > 2 * n else np.zeros((0, n))
    G = np.vstack([np.eye(n), -np.eye(n), Gc])
    h = np.r_[x0 + rng.uniform(0.5, 2, n), -(x0 - rng.uniform(0.5, 2, n)),
              Gc @ x0 + rng.uniform(0.1, 1, Gc.shape[0])]
    A = rng.standard_normal((p, n))
    b = A @ x0
    c = rng.standard_normal(n)
    verts = lp_vertices(c, A, b, G, h)
    if len(verts) < 2 or verts[1][0] - verts[0][0] < 1e-6:
        pytest.skip("optimum not unique for this draw")
    prob = mkprob(np.zeros((n, n)), c, A, b, G, h, G.shape[0], [])
    r = ipm.solve(prob)
    assert_optimal(prob, r)
    assert np.allclose(r.x, np.array(verts[0][1]), atol=1e-6)
    assert abs(r.pobj - verts[0][0]) <= 1e-6 * max(1, abs(verts[0][0]))


def test_equality_only_qp_is_one_kkt_solve():
    rng = np.random.default_rng(5)
    n, p = 8, 3
    M = rng.standard_normal((n, n))
    P = M @ M.T + np.eye(n)
    A = rng.standard_normal((p, n))
    b = rng.standard_normal(p)
    c = rng.standard_normal(n)
    prob = mkprob(P, c, A, b, np.zeros((0, n)), np.zeros(0), 0, [])
    r = ipm.solve(prob)
    K = np.block([[P, A.T], [A, np.zeros((p, p))]])
    want = np.linalg.solve(K, np.r_[-c, b])
    assert r.status == ipm.SOLVED
    assert np.allclose(r.x, want[:n], atol=1e-8)


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "many_soc_s"])
def test_workload_invariants(name):
    prob = problems.workload(name)
    r = ipm.solve(prob)
    assert_optimal(prob, r)
    assert abs(r.pobj - r.dobj) <= 1e-6 * max(1.0, abs(r.pobj))
    assert all(0 < h["alpha"] <= 1 for h in r.history)


def test_lasso_optimality_structure():
    # y = F x - g exactly and t = |x| at the optimum
    prob = problems.workload("lasso_s")
    r = ipm.solve(prob)
    nx = prob.meta["x_true"].size
    ny = prob.p
    x, y, t = r.x[:nx], r.x[nx:nx + ny], r.x[nx + ny:]
    F = prob.A[:, :nx]
    assert np.allclose(y, F @ x - prob.b, atol=1e-7)
    assert np.allclose(t, np.abs(x), atol=1e-6)


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------
def tight():
    s = ipm.IPMSettings(eps_abs=1e-11, eps_rel=1e-11)
    return s


def test_box_qp_gradient_closed_form():
    prob, d, c, lo, hi = box_qp(7)
    r = ipm.solve(prob, tight())
    xs = r.x
    free = (xs > lo + 1e-6) & (xs < hi - 1e-6)
    n = prob.n
    for i in range(n):
        g = np.zeros(n); g[i] = 1.0            # L = x_i
        gr = adjoint.backward(prob, r, g)
        want_c = np.zeros(n)
        want_c[i] = -1.0 / d[i] if free[i] else 0.0
        assert np.allclose(gr["dc"], want_c, atol=1e-5)
        # active upper bound hi_i: dx_i/dhi_i = 1; active lower: dx_i/dlo_i = 1 (h holds -lo)
        want_h = np.zeros(2 * n)
        if xs[i] >= hi[i] - 1e-6:
            want_h[i] = 1.0
        if xs[i] <= lo[i] + 1e-6:
            want_h[n + i] = -1.0
        assert np.allclose(gr["dh"], want_h, atol=1e-5)


@pytest.mark.parametrize("seed,frac", [(8, 0.2), (9, -0.5), (21, 0.0)])
def test_soc_projection_jacobian_closed_form(seed, frac):
    """Jacobian of the SOC projection where ||v1|| > |v0| (a boundary point):
    1/2 [[1, vb'], [vb, (1 + v0/|v1|) I - (v0/|v1|) vb vb']],  vb = v1/|v1|.
    The derivative system is exact only in the limit of zero gap; the
    tolerance reflects the final iterate's distance from the boundary."""
    q = 4
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(q)
    v[0] = frac * np.linalg.norm(v[1:])
    prob = mkprob(np.eye(q), -v, np.zeros((0, q)), [], -np.eye(q), np.zeros(q), 0, [q])
    r = ipm.solve(prob, ipm.IPMSettings(eps_abs=1e-10, eps_rel=1e-10))
    v0, v1 = v[0], v[1:]
    nv = np.linalg.norm(v1)
    vb = v1 / nv
    Jac = 0.5 * np.block([[np.ones((1, 1)), vb[None, :]],
                          [vb[:, None], (1 + v0 / nv) * np.eye(q - 1) - (v0 / nv) * np.outer(vb, vb)]])
    for i in range(q):
        g = np.zeros(q); g[i] = 1.0
        gr = adjoint.backward(prob, r, g)
        # x*(v) with c = -v: dx_i/dv = -dx_i/dc
        assert np.allclose(-gr["dc"], Jac[i], atol=2e-3)


@pytest.mark.parametrize("name", ["small_qp", "lasso_diff_t"])
def test_adjoint_matches_dense_kkt_and_dot_product(name):
    prob = problems.small_qp(n=80, p=20, m=60, mrows=40) if name == "small_qp" else \
        problems.lasso(rows=120, cols=60, density=0.1, seed=9)
    r = ipm.solve(prob)
    rng = np.random.default_rng(10)
    g = rng.standard_normal(prob.n)
    a = adjoint.backward(prob, r, g)
    dn = adjoint.backward_dense(prob, r, g)
    for k in ("dc", "db", "dh", "dP", "dA", "dG"):
        assert np.allclose(a[k], dn[k], rtol=1e-8, atol=1e-8 * np.max(np.abs(dn[k]), initial=1.0))
    # dot-product test on the same factor: u'r = g'(K^-1 r)_x
    rr = rng.standard_normal(prob.n + prob.p + prob.m)
    w, _ = adjoint.final_factor(prob, r).solve(rr, ir_max=10)
    assert np.isclose(a["u"] @ rr, g @ w[:prob.n], rtol=1e-8)


def test_adjoint_vs_central_finite_differences():
    prob = problems.lasso(rows=80, cols=40, density=0.1, seed=12)
    st = tight()
    base = ipm.solve(prob, st)
    rng = np.random.default_rng(13)
    xref = rng.standard_normal(prob.n)
    g = base.x - xref                          # L = 1/2 ||x* - xref||^2
    gr = adjoint.backward(prob, base, g)
    hstep = 1e-6
    for vec, key, count in (("c", "dc", 6), ("h", "dh", 6), ("b", "db", 6)):
        data = getattr(prob, vec)
        for j in rng.choice(len(data), size=count, replace=False):
            vals = []
            for sgn in (+1, -1):
                pr = problems.Problem(**{**prob.__dict__})
                d2 = data.copy(); d2[j] += sgn * hstep
                setattr(pr, vec, d2)
                vals.append(ipm.solve(pr, st).x)
            xp, xm = vals
            fd = 0.5 * (xp - xm) @ (xp + xm - 2 * xref) / (2 * hstep)
            assert abs(gr[key][j] - fd) <= 1e-3 * max(abs(fd), 1e-3), (vec, j, gr[key][j], fd)
    # values of A and G on their patterns (the perturbation keeps the pattern): three seeded
    # entries and the three with the largest gradient (most entries of G sit on inactive bounds,
    # where the gradient vanishes)
    for mat, key in (("A", "dA"), ("G", "dG")):
        M = getattr(prob, mat)
        top = np.argsort(-np.abs(gr[key]))[:3]
        for t in np.unique(np.concatenate([rng.choice(M.nnz, size=3, replace=False), top])):
            vals = []
            for sgn in (+1, -1):
                pr = problems.Problem(**{**prob.__dict__})
                M2 = M.copy(); M2.data[t] += sgn * hstep
                setattr(pr, mat, M2)
                vals.append(ipm.solve(pr, st).x)
            xp, xm = vals
            fd = 0.5 * (xp - xm) @ (xp + xm - 2 * xref) / (2 * hstep)
            assert abs(gr[key][t] - fd) <= 1e-3 * max(abs(fd), 1e-3), (mat, t, gr[key][t], fd)


def test_adjoint_through_the_whole_solution_vs_central_finite_differences():
    """L = 1/2 |x* - xr|^2 + 1/2 |y* - yr|^2 + 1/2 |z* - zr|^2 + 1/2 |s* - sr|^2: the adjoint
    with g_y, g_z and g_s against central differences in c, b, h, A and G."""
    prob = problems.lasso(rows=80, cols=40, density=0.1, seed=12)
    st = tight()
    base = ipm.solve(prob, st)
    rng = np.random.default_rng(14)
    ref = {k: rng.standard_normal(len(getattr(base, k))) for k in ("x", "y", "z", "s")}
    gr = adjoint.backward(prob, base, base.x - ref["x"], gy=base.y - ref["y"], gz=base.z - ref["z"],
                          gs=base.s - ref["s"])

    def loss_diff(rp, rm):
        # L(+) - L(-) = sum over the blocks of 1/2 (v+ - v-)'(v+ + v- - 2 ref)
        return sum(0.5 * (getattr(rp, k) - getattr(rm, k)) @ (getattr(rp, k) + getattr(rm, k) - 2 * ref[k])
                   for k in ("x", "y", "z", "s"))

    hstep = 1e-6
    checks = []
    for vec, key in (("c", "dc"), ("h", "dh"), ("b", "db")):
        data = getattr(prob, vec)
        top = np.argsort(-np.abs(gr[key]))[:2]
        for j in np.unique(np.concatenate([rng.choice(len(data), size=2, replace=False), top])):
            res = []
            for sgn in (+1, -1):
                pr = problems.Problem(**{**prob.__dict__})
                d2 = data.copy(); d2[j] += sgn * hstep
                setattr(pr, vec, d2)
                res.append(ipm.solve(pr, st))
            checks.append((vec, j, gr[key][j], loss_diff(*res) / (2 * hstep)))
    for mat, key in (("A", "dA"), ("G", "dG")):
        M = getattr(prob, mat)
        top = np.argsort(-np.abs(gr[key]))[:2]
        for t in np.unique(np.concatenate([rng.choice(M.nnz, size=2, replace=False), top])):
            res = []
            for sgn in (+1, -1):
                pr = problems.Problem(**{**prob.__dict__})
                M2 = M.copy(); M2.data[t] += sgn * hstep
                setattr(pr, mat, M2)
                res.append(ipm.solve(pr, st))
            checks.append((mat, t, gr[key][t], loss_diff(*res) / (2 * hstep)))
    for what, j, adj, fd in checks:
        assert abs(adj - fd) <= 1e-3 * max(abs(fd), 1e-3), (what, j, adj, fd)


def test_box_qp_gradient_of_the_quadratic_closed_form():
    """dL/dP on the box QP (P = diag(d)): x*_i = -c_i/d_i on free coordinates, so
    dx*_i/dd_i = c_i/d_i^2 there, and 0 for clipped coordinates and for every other d_j."""
    prob, d, c, lo, hi = box_qp(7)
    r = ipm.solve(prob, tight())
    xs = r.x
    free = (xs > lo + 1e-6) & (xs < hi - 1e-6)
    assert free.sum() >= 3 and (~free).sum() >= 3
    Pu = prob.P.tocoo()
    assert np.array_equal(Pu.row, Pu.col)              # only the diagonal is stored
    for i in range(prob.n):
        g = np.zeros(prob.n); g[i] = 1.0                # L = x_i
        gr = adjoint.backward(prob, r, g)
        want = np.zeros(prob.n)
        want[i] = c[i] / d[i] ** 2 if free[i] else 0.0
        assert np.allclose(gr["dP"][np.argsort(Pu.row)], want, atol=1e-5), (i, gr["dP"], want)


def test_adjoint_of_the_quadratic_vs_central_finite_differences():
    """dL/dP on P's stored upper pattern against central differences of the stored values: a
    stored off-diagonal value P_ij enters the symmetric P twice (P_ij = P_ji), a diagonal value
    once.  Seeded diagonal and off-diagonal entries plus the largest-gradient ones."""
    prob = problems.small_qp(n=30, p=8, m=30, mrows=20, density=0.2, seed=31)
    st = tight()
    base = ipm.solve(prob, st)
    rng = np.random.default_rng(32)
    xref = rng.standard_normal(prob.n)
    gr = adjoint.backward(prob, base, base.x - xref)     # L = 1/2 |x* - xref|^2
    Pu = prob.P.tocoo()
    diag = np.flatnonzero(Pu.row == Pu.col)
    off = np.flatnonzero(Pu.row != Pu.col)
    assert len(off) > 10
    top_d = diag[np.argsort(-np.abs(gr["dP"][diag]))[:2]]
    top_o = off[np.argsort(-np.abs(gr["dP"][off]))[:3]]
    picks = np.unique(np.concatenate([rng.choice(diag, 3, replace=False), rng.choice(off, 4, replace=False),
                                      top_d, top_o]))
    hstep = 1e-6
    nchecked = {"diag": 0, "off": 0}
    for t in picks:
        xs = []
        for sgn in (+1, -1):
            pr = problems.Problem(**{**prob.__dict__})
            P2 = prob.P.copy(); P2.data[t] += sgn * hstep
            pr.P = P2
            xs.append(ipm.solve(pr, st).x)
        xp, xm = xs
        fd = 0.5 * (xp - xm) @ (xp + xm - 2 * xref) / (2 * hstep)
        assert abs(gr["dP"][t] - fd) <= 1e-3 * max(abs(fd), 1e-3), (t, Pu.row[t], Pu.col[t], gr["dP"][t], fd)
        nchecked["diag" if Pu.row[t] == Pu.col[t] else "off"] += 1
    assert nchecked["diag"] >= 3 and nchecked["off"] >= 4
