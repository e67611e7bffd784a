"""Full-size workloads on the device, checked through properties that hold at
any size and through sampled outputs the oracle computes itself.

- lasso (F 20000 x 10000, N_K = 80000), FP32+IR and FP64: KKT residuals and
  gap recomputed here from the returned (x, s, y, z) within the stopping rule,
  strict interiority, and the two precision modes agreeing to 1e-6 in x and
  objective; FP64 factor entries of the first rows of L (the oracle's
  up-looking factorization stops after a prefix of rows) to 1e-10.
- many_soc (n = 300000, 1e5 cones of dimension 4, N_K = 800000): residuals,
  gap, cone interiority, modes agreeing.
- big_cones (3000 cones of dimension 64, 300 of 256, 30 of 1024, 5000 bounds,
  n = 20000): as above; cones of 32 entries and more run one wavefront per
  cone.
- huber_m (the Huber generator at F 50000 x 20000, 40 entries per row,
  N_K = 320000; the full 500000 x 200000 instance would need a dense root
  front of about 2e5 columns, more than one GPU's memory): as above.
- lasso_diff (F 50000 x 20000, N_K = 180000): adjoint gradients of
  L = 1/2 |x* - x_ref|^2 against central finite differences (h = 1e-6) on
  seeded coordinates of c, b and h, 3 per gradient (18 re-solves) to keep the
  test within minutes.
"""
import hashlib
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import problems  # noqa: E402

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def solver(prob, **kw):
    import paper_2603_29197_amd as qg
    # FP32+IR solves use FP32 factors at every size here (the library's default keeps FP64 factors
    # below 1e10 matrix-core flops per factorization, where FP32 saves nothing)
    kw.setdefault("fp32_min_flops", 0.0)
    print(f"[gpu] setup {prob.name} n={prob.n} m={prob.m} p={prob.p}", flush=True)
    return qg.Solver(prob, **kw)


def check_optimal(prob, x, s, y, z, eps=1e-8, slack=1.05):
    """Stopping rule of the method (residuals and gap), recomputed in FP64 by
    the oracle's residual routine from the returned point."""
    from oracle import ipm as oipm
    r = oipm.residuals(prob, x, s, y, z)
    ok, pres, dres, gap = oipm.stop_test(prob, r, s, slack * eps, slack * eps)
    print(f"[gpu] {prob.name}: pres {pres:.2e} dres {dres:.2e} gap {gap:.2e} pobj {r['pobj']:.12g}", flush=True)
    assert ok
    return r["pobj"]


def check_interior(prob, s, z):
    l = prob.l
    assert np.all(s[:l] > 0) and np.all(z[:l] > 0)
    off = l
    for q in prob.q:
        for u in (s, z):
            assert u[off] > np.linalg.norm(u[off + 1:off + q])
        off += q


def solve_both(prob):
    import paper_2603_29197_amd as qg
    S = solver(prob, precision=qg.QG_FP32_IR)
    out = {}
    for name, prec in (("fp32", qg.QG_FP32_IR), ("fp64", qg.QG_FP64)):
        S.set_settings(precision=prec)
        x, s, y, z, info = S.solve()
        print(f"[gpu] {prob.name} {name}: {info['status_name']} iters {info['iters']} switch "
              f"{info['switch_iter']} ir {info['ir_steps']} step {info['ms_step_median']:.2f} ms (cone phase "
              f"{info['ms_cone']:.1f}, factor {info['ms_factor']:.1f}, solves {info['ms_trisolve']:.1f} ms "
              f"over the solve)", flush=True)
        assert info["status"] == 1
        out[name] = [host(t) for t in (x, s, y, z)]
    S.close()
    return out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name", ["lasso", "many_soc", "huber_m", "big_cones"])
def test_full_size_solution_properties(name):
    prob = problems.workload(name)
    out = solve_both(prob)
    objs = {}
    for mode, (x, s, y, z) in out.items():
        objs[mode] = check_optimal(prob, x, s, y, z)
        check_interior(prob, s, z)
    x32, x64 = out["fp32"][0], out["fp64"][0]
    assert np.max(np.abs(x32 - x64)) <= 1e-6 * max(1.0, np.max(np.abs(x64)))
    assert abs(objs["fp32"] - objs["fp64"]) <= 1e-6 * max(1.0, abs(objs["fp64"]))


@pytest.mark.timeout(600)
def test_lasso_full_factor_prefix_rows():
    """FP64 factor of the full lasso KKT (identity scaling, static
    regularization 1e-3) against the oracle's up-looking LDL' on the rows it
    finishes in a few seconds (every entry of L with row index below the
    prefix, and those pivots)."""
    import ctypes
    import paper_2603_29197_amd as qg
    from oracle import _clib, kkt, symbolic
    prob = problems.workload("lasso")
    gold = os.path.join(ROOT, "tests", "golden")
    perm = np.load(os.path.join(gold, "lasso_perm.npy"))
    want = json.load(open(os.path.join(gold, "patterns.json")))["lasso"]["perm"]
    assert hashlib.sha256(np.ascontiguousarray(perm, dtype=np.int32).tobytes()).hexdigest() == want
    delta = 1e-3
    S = solver(prob, precision=qg.QG_FP64, static_reg=delta)
    ones = np.ones(prob.m)
    S.step_scaling(dev(ones), dev(ones))
    S.step_factor(qg.QG_FP64)
    Kp = kkt.kkt_pattern(prob)
    Up = symbolic.permute_upper(Kp, perm)
    parent = symbolic.etree(Up)
    Lp, Li, _ = symbolic.l_pattern(Up, parent)
    Lx_g, D_g = S.step_get_factor(Lp, Li)
    S.close()
    N = len(perm)
    tpos = np.arange(len(Li), dtype=np.int64) - np.repeat(Lp[:-1], np.diff(Lp))
    ops = np.bincount(Li, weights=tpos.astype(np.float64), minlength=N) + np.bincount(Li, minlength=N) + 1.0
    k_end = int(np.searchsorted(np.cumsum(ops), 1.2e10))
    Kreg = kkt.kkt_upper(prob, -np.ones(prob.l), [], delta, delta)
    ip, ii, pos = symbolic.permute_map(Kp, perm)
    Ux = np.empty(len(ii))
    Ux[pos] = Kreg.data
    sign = kkt.pivot_signs(prob)[perm].astype(np.int8)
    Lx = np.zeros(len(Li))
    D = np.zeros(N)
    nreg = ctypes.c_int64(0)
    _clib.lib().or_ldl_numeric_rows(N, k_end, ip, ii, Ux, parent, Lp, Li, sign, 1e-13, 1e-7, Lx, D,
                                    ctypes.byref(nreg))
    sel = Li < k_end
    print(f"[gpu] lasso factor prefix: {k_end} of {N} rows, {int(sel.sum())} entries of L", flush=True)
    assert nreg.value == 0
    e_l = float(np.max(np.abs(Lx_g[sel] - Lx[sel])) / max(1.0, np.max(np.abs(Lx[sel]))))
    e_d = float(np.max(np.abs(D_g[:k_end] - D[:k_end]) / np.maximum(1.0, np.abs(D[:k_end]))))
    print(f"[gpu] lasso factor prefix: L rel err {e_l:.2e}, D rel err {e_d:.2e}", flush=True)
    assert e_l <= 1e-10 and e_d <= 1e-10


@pytest.mark.timeout(900)
def test_lasso_diff_full_gradient_fd():
    """Adjoint gradients against central finite differences on seeded
    coordinates (FP64, stopping rule tightened to 1e-10 for the +/- solves, so
    the difference quotient carries about 1e-4 of solver noise)."""
    import paper_2603_29197_amd as qg
    prob = problems.workload("lasso_diff")
    rng = np.random.default_rng(29197 + 5)
    x_ref = rng.standard_normal(prob.n)
    # the base solve uses the same tightened stopping rule as the +/- solves: near-degenerate
    # complementarity pairs make the derivative depend on how far the final iterate is from the
    # optimum
    S = solver(prob, precision=qg.QG_FP64, differentiable=1, eps_abs=1e-10, eps_rel=1e-10, max_iter=40)
    x, s, y, z, info = S.solve()
    assert info["status"] in (1, 2)
    xs = host(x)
    g = S.backward(dev(xs - x_ref))
    grads = {"c": host(g["dc"]), "b": host(g["db"]), "h": host(g["dh"])}
    S.set_settings(differentiable=0)
    base = {"c": prob.c.copy(), "b": prob.b.copy(), "h": prob.h.copy()}
    hstep = 1e-6
    worst = 0.0
    for key in ("c", "b", "h"):
        # two seeded coordinates and the one with the largest adjoint entry
        idx = np.unique(np.append(rng.choice(len(base[key]), 2, replace=False), np.argmax(np.abs(grads[key]))))
        adj = grads[key][idx]
        fds = []
        for j in idx:
            xs_pm = []
            for sgn in (1.0, -1.0):
                v = base[key].copy()
                v[j] += sgn * hstep
                S.update(**{key: v})
                xp, _, _, _, inf2 = S.solve()
                assert inf2["status"] in (1, 2)
                xs_pm.append(host(xp))
            S.update(**{key: base[key]})
            xp_, xm_ = xs_pm
            fds.append(0.5 * float((xp_ - xm_) @ (xp_ + xm_ - 2 * x_ref)) / (2 * hstep))
        fds = np.array(fds)
        # relative error with the floor 1e-3 * max_k |grad_k| over the whole gradient vector
        scale = 1e-3 * max(np.max(np.abs(grads[key])), np.max(np.abs(fds)), 1e-12)
        err = np.abs(adj - fds) / np.maximum(np.abs(fds), scale)
        print(f"[gpu] lasso_diff d/d{key}: adjoint {adj} fd {fds} rel err {err}", flush=True)
        worst = max(worst, float(np.max(err)))
    S.close()
    assert worst <= 1e-3
