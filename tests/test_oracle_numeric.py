"""Pins of the oracle's LDL', refinement and cone algebra.

LDL' is compared with a textbook dense LDL' without pivoting written with
numpy (a different algorithm: right-looking, dense), with the reconstruction
P L D L' P' = K_reg, and with the inertia of a quasi-definite matrix.  The
cone algebra is compared with its defining identities (W'W z = s, lambda =
W z = W^-T s, the Jordan-product identities) and the max step with bisection
and with the smallest positive root of the boundary quadratic.
"""
import numpy as np
import pytest

from oracle import cones as C
from oracle import kkt, ldl, symbolic
from synth import problems


def dense_ldl(K):
    """Right-looking dense LDL' without pivoting (textbook)."""
    A = np.array(K, dtype=np.float64)
    N = A.shape[0]
    L = np.eye(N)
    D = np.zeros(N)
    for j in range(N):
        D[j] = A[j, j]
        L[j + 1:, j] = A[j + 1:, j] / D[j]
        A[j + 1:, j + 1:] -= D[j] * np.outer(L[j + 1:, j], L[j + 1:, j])
    return L, D


def interior_point_block(prob, seed):
    x, s, y, z = problems.random_point(prob, seed)
    cn = C.Cones(prob.l, prob.q)
    sc = C.nt_scaling(cn, s, z)
    return sc.block33()


SMALL = [
    lambda: problems.small_qp(n=60, p=10, m=50, mrows=30, density=0.15),
    lambda: problems.many_soc(n=80, ncones=12, q=4, nbounds=10, seed=3),
    lambda: problems.lasso(rows=60, cols=30, density=0.1, seed=5),
    lambda: problems.many_soc(n=60, ncones=5, q=7, nbounds=8, seed=11, windowed=False),
]


@pytest.mark.parametrize("delta", [1e-3, 1e-8])
@pytest.mark.parametrize("mk", range(len(SMALL)))
def test_ldl_matches_dense_textbook(mk, delta):
    """Entrywise agreement needs bounded growth: equality pivots equal to
    -delta (before their neighbours) amplify rounding by ~1/delta, so L and D
    are compared entrywise at delta = 1e-3 and by backward error at 1e-8."""
    prob = SMALL[mk]()
    orth, blocks = interior_point_block(prob, 1)
    F = ldl.KKTFactor(prob, reg=ldl.RegSettings(static_reg=delta))
    F.factor(orth, blocks)
    assert F.nreg == 0
    Kreg = kkt.kkt_upper(prob, orth, blocks, delta, delta).toarray()
    Kreg = Kreg + np.triu(Kreg, 1).T
    perm = F.pat.perm
    Kp = Kreg[np.ix_(perm, perm)]
    L = F.L_dense()
    # backward error of the sparse factorization
    R = L @ np.diag(F.D) @ L.T - Kp
    growth = np.max(np.abs(L)) ** 2 * np.max(np.abs(F.D))
    assert np.max(np.abs(R)) <= 1e-15 * len(Kp) * max(growth, np.max(np.abs(Kp))) * 10
    # inertia of the quasi-definite matrix: n positive, p + m negative
    assert np.sum(F.D > 0) == prob.n and np.sum(F.D < 0) == prob.p + prob.m
    if delta < 1e-4:
        return
    Ld, Dd = dense_ldl(Kp)
    scale = np.max(np.abs(Ld))
    assert np.max(np.abs(L - Ld)) <= 1e-11 * scale
    assert np.max(np.abs(F.D - Dd) / np.abs(Dd)) <= 1e-11
    # entries outside the symbolic pattern are (numerically) zero in the dense factor
    outside = (L == 0) & ~np.eye(len(L), dtype=bool)
    assert np.max(np.abs(Ld[outside]), initial=0.0) <= 1e-12 * scale


@pytest.mark.parametrize("mk", range(len(SMALL)))
def test_refined_solve_matches_dense_solve(mk):
    prob = SMALL[mk]()
    orth, blocks = interior_point_block(prob, 2)
    F = ldl.KKTFactor(prob)
    F.factor(orth, blocks)
    rhs = np.random.default_rng(3).standard_normal(F.N)
    x, steps = F.solve(rhs, ir_max=10)
    K = F.K_unreg.toarray()
    xd = np.linalg.solve(K, rhs)
    assert np.max(np.abs(x - xd)) <= 1e-9 * np.max(np.abs(xd))
    # refinement reduces the residual of the unregularized system monotonically
    x0 = F.solve_factor(rhs)
    r0 = np.max(np.abs(rhs - K @ x0))
    r1 = np.max(np.abs(rhs - K @ x))
    assert r1 <= r0


def test_dynamic_regularization_fires_on_wrong_sign_pivot():
    # decoupled x and z (G = 0): the z pivot is the (3,3) entry itself; a
    # positive value has the wrong sign for a dual pivot and is replaced by
    # -dyn_delta; the x pivot is the static regularization (right sign).
    prob = problems.Problem(n=1, m=1, p=0, P=problems._csc(np.zeros((1, 1))), c=np.zeros(1),
                            A=problems._csc(np.zeros((0, 1))), b=np.zeros(0),
                            G=problems._csc(np.zeros((1, 1))), h=np.zeros(1), l=1, q=[])
    reg = ldl.RegSettings(static_reg=1e-8, dyn_eps=1e-13, dyn_delta=1e-7)
    F = ldl.KKTFactor(prob, reg=reg)
    F.factor(np.array([1e-30]), [])
    d = dict(zip(F.pat.perm.tolist(), F.D.tolist()))
    assert d[0] == 1e-8 and d[1] == -1e-7 and F.nreg == 1
    F.factor(np.array([-1e-3]), [])
    d = dict(zip(F.pat.perm.tolist(), F.D.tolist()))
    assert d[1] == -1e-3 and F.nreg == 0


# ---------------------------------------------------------------------------
# cone algebra
# ---------------------------------------------------------------------------
def _soc_pair(q, seed):
    prob = problems.Problem(n=1, m=q, p=0, P=problems._csc(np.zeros((1, 1))), c=np.zeros(1),
                            A=problems._csc(np.zeros((0, 1))), b=np.zeros(0),
                            G=problems._csc(np.zeros((q, 1))), h=np.zeros(q), l=0, q=[q])
    _, s, _, z = problems.random_point(prob, seed)
    return C.Cones(0, [q]), s, z


def _mixed(seed, qs=(5, 3, 5, 2, 6, 9)):
    prob = problems.many_soc(n=40, ncones=6, q=5, nbounds=7, seed=seed)
    prob.q = list(qs)
    prob.m = prob.l + sum(prob.q)
    _, s, _, z = problems.random_point(prob, seed)
    return C.Cones(prob.l, prob.q), s, z


def _dense_W(sc, cn):
    m = cn.m
    return np.column_stack([sc.W(np.eye(m)[:, k]) for k in range(m)])


@pytest.mark.parametrize("seed,qs", [(k, (5, 3, 5, 2, 6, 9)) for k in range(6)] +
                         [(k, (33, 2, 130, 64)) for k in range(2)])
def test_nt_scaling_identities(seed, qs):
    cn, s, z = _mixed(seed, qs)
    sc = C.nt_scaling(cn, s, z)
    W = _dense_W(sc, cn)
    assert np.allclose(W, W.T, atol=1e-13)
    assert np.allclose(W @ W @ z, s, rtol=1e-13, atol=1e-13)              # W'W z = s
    assert np.allclose(sc.lam, W @ z, rtol=1e-13, atol=1e-13)             # lambda = W z
    assert np.allclose(sc.lam, sc.Winv(s), rtol=1e-12, atol=1e-13)        # lambda = W^-T s
    Winv = np.column_stack([sc.Winv(np.eye(cn.m)[:, k]) for k in range(cn.m)])
    assert np.allclose(W @ Winv, np.eye(cn.m), atol=1e-12)
    assert np.isclose(sc.lam @ sc.lam, s @ z, rtol=1e-13)
    orth, blocks = sc.block33()
    H = np.zeros((cn.m, cn.m))
    H[:cn.l, :cn.l] = np.diag(orth)
    for k, off in enumerate(cn.offsets):
        q = cn.q[k]
        H[off:off + q, off:off + q] = blocks[k]
    assert np.allclose(H, -(W.T @ W), atol=1e-12)
    # lambda'J lambda = s_n z_n per SOC
    for k, off in enumerate(cn.offsets):
        q = cn.q[k]
        J = np.diag(np.r_[1.0, -np.ones(q - 1)])
        lam = sc.lam[off:off + q]
        sn = np.sqrt(s[off:off + q] @ J @ s[off:off + q])
        zn = np.sqrt(z[off:off + q] @ J @ z[off:off + q])
        assert np.isclose(lam @ J @ lam, sn * zn, rtol=1e-12)


def test_nt_scaling_of_equal_points_is_identity():
    cn, s, _ = _mixed(3)
    sc = C.nt_scaling(cn, s, s)
    assert np.allclose(_dense_W(sc, cn), np.eye(cn.m), atol=1e-14)
    assert np.allclose(sc.lam, s, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_jordan_identities(seed):
    cn, u, v = _mixed(seed)
    e = cn.identity()
    assert np.allclose(cn.jordan(e, u), u, atol=0)
    assert np.allclose(cn.jordan(u, v), cn.jordan(v, u), atol=1e-15)
    x = cn.inv_jordan(u, v)
    assert np.allclose(cn.jordan(u, x), v, rtol=1e-12, atol=1e-12)
    # SOC product by hand for one cone
    off, q = cn.offsets[0], cn.q[0]
    a, b = u[off:off + q], v[off:off + q]
    want = np.r_[a @ b, a[0] * b[1:] + b[0] * a[1:]]
    assert np.allclose(cn.jordan(u, v)[off:off + q], want, rtol=1e-15)


def _in_cone(cn, u, tol=0.0):
    return np.all(cn.lambda_min(u) >= -tol)


@pytest.mark.parametrize("seed", range(8))
def test_max_step_vs_bisection_and_root(seed):
    cn, u, _ = _mixed(seed)
    du = np.random.default_rng(100 + seed).standard_normal(cn.m) * 3.0
    per = cn.max_step_per_cone(u, du)
    # orthant closed form
    ol = np.where(du[:cn.l] < 0, -u[:cn.l] / np.where(du[:cn.l] < 0, du[:cn.l], 1), np.inf)
    assert np.array_equal(per[:cn.l], ol)
    for k, off in enumerate(cn.offsets):
        q = cn.q[k]
        uk, dk = u[off:off + q], du[off:off + q]
        a = per[cn.l + k]
        inside = lambda t: (uk[0] + t * dk[0]) >= np.linalg.norm(uk[1:] + t * dk[1:])
        if np.isinf(a):
            assert inside(1e6)
            continue
        # bisection
        lo, hi = 0.0, 1.0
        while inside(hi):
            hi *= 2
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            lo, hi = (mid, hi) if inside(mid) else (lo, mid)
        assert abs(a - lo) <= 1e-12 * max(1.0, lo)
        # smallest positive root of (u + t du)'J(u + t du) = 0
        J = np.r_[1.0, -np.ones(q - 1)]
        qa, qb, qc = dk @ (J * dk), 2 * uk @ (J * dk), uk @ (J * uk)
        roots = np.roots([qa, qb, qc])
        roots = np.real(roots[np.isreal(roots)])
        roots = roots[roots > 0]
        assert np.isclose(a, roots.min(), rtol=1e-10)
    assert cn.max_step(u, du) == per.min()


def test_shift_interior():
    cn, u, _ = _mixed(1)
    assert np.array_equal(cn.shift_interior(u), u)          # already interior
    v = u.copy()
    v[0] = -3.0
    w = cn.shift_interior(v)
    assert np.all(cn.lambda_min(w) >= 1.0 - 1e-12)


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "many_soc_s"])
def test_row_work_and_leading_block_factor(name):
    """The bounded-prefix timing of the oracle's factorization rests on three facts, each checked
    against the full pattern and the full factorization: (1) or_row_work's row counts are the row
    counts of L's pattern and its per-row work is the sum over the row's entries of (position in
    the column + 1), plus one; in total sum_j c_j (c_j + 1) / 2 + N with c_j the column counts
    (closed form); (2) the pattern of the leading block is the full pattern restricted to rows
    and columns below the cut; (3) factoring only the rows below the cut on that pattern gives the
    same L rows and pivots as the full factorization."""
    import ctypes
    prob = problems.workload(name)
    F = ldl.KKTFactor(prob)
    _, s, _, z = problems.random_point(prob, 3)
    F.factor(*C.nt_scaling(C.Cones(prob.l, prob.q), s, z).block33())
    Kp = kkt.kkt_pattern(prob)
    Up = symbolic.permute_upper(Kp, F.pat.perm)
    parent = F.pat.parent
    N = F.N
    rowcnt, rowops = symbolic.row_work(Up, parent)
    Lp, Li = F.pat.Lp, F.pat.Li
    assert np.array_equal(rowcnt, np.bincount(Li, minlength=N))
    tpos = np.arange(len(Li)) - np.repeat(Lp[:-1], np.diff(Lp))
    assert np.allclose(rowops, np.bincount(Li, weights=tpos + 1.0, minlength=N) + 1.0, rtol=0, atol=0)
    c = np.diff(Lp).astype(np.float64)
    assert rowops.sum() == float(np.sum(c * (c + 1) / 2) + N)
    cut = N // 2 + 7
    Lp2, Li2 = symbolic.l_pattern_rows(Up, parent, cut)
    for j in range(cut):
        col = Li[Lp[j]:Lp[j + 1]]
        assert np.array_equal(Li2[Lp2[j]:Lp2[j + 1]], col[col < cut])
    ip, ii, pos = symbolic.permute_map(Kp, F.pat.perm)
    Kreg = F.asm.upper(*C.nt_scaling(C.Cones(prob.l, prob.q), s, z).block33(), F.reg.static_reg,
                       F.reg.static_reg)
    Ux = np.empty(len(ii)); Ux[pos] = Kreg.data
    Lx2 = np.zeros(len(Li2)); D2 = np.zeros(cut)
    nreg = ctypes.c_int64(0)
    from oracle._clib import lib
    rc = lib().or_ldl_numeric_rows(cut, cut, ip, ii, Ux, parent, Lp2, Li2, F.sign_perm, F.reg.dyn_eps,
                                   F.reg.dyn_delta, Lx2, D2, ctypes.byref(nreg))
    assert rc == 0
    assert np.array_equal(D2, F.D[:cut])
    for j in range(cut):
        col = Li[Lp[j]:Lp[j + 1]]
        assert np.array_equal(Lx2[Lp2[j]:Lp2[j + 1]], F.Lx[Lp[j]:Lp[j + 1]][col < cut])
