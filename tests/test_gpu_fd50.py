"""The differentiation workload (lasso at F 50000 x 20000, density 0.002,
N_K = 180000; L = 1/2 |x* - x_ref|^2 with x_ref ~ N(0,1)): the adjoint
gradients dL/dc, dL/db and dL/dh from qg_backward on the stored final factor
against central finite differences (h = 1e-6) on 50 random coordinates of
each, one test per gradient (100 re-solves each).  The base solve and the
+/- solves use the stopping rule tightened to 1e-10, so the difference
quotient carries about 1e-4 of solver noise; the bound is 1e-3 relative with
the floor 1e-3 max_k |grad_k| (coordinates of a vanishing gradient).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from synth import problems  # noqa: E402

pytestmark = pytest.mark.gpu

NCOORD = 50
HSTEP = 1e-6


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("key", ["c", "b", "h"])
def test_lasso_diff_gradient_fd_50_coordinates(key):
    import paper_2603_29197_amd as qg
    prob = problems.workload("lasso_diff")
    rng = np.random.default_rng(29197 + 5)
    x_ref = rng.standard_normal(prob.n)
    print(f"[gpu] lasso_diff d/d{key}: setup", flush=True)
    S = qg.Solver(prob, precision=qg.QG_FP64, differentiable=1, eps_abs=1e-10, eps_rel=1e-10, max_iter=40)
    x, s, y, z, info = S.solve()
    assert info["status"] in (1, 2)
    xs = host(x)
    g = S.backward(dev(xs - x_ref))
    grad = host(g["d" + key])
    S.set_settings(differentiable=0)
    base = getattr(prob, key).copy()
    idx = np.sort(np.random.default_rng({"c": 51, "b": 52, "h": 53}[key]).choice(len(base), NCOORD, replace=False))
    fds = np.empty(NCOORD)
    for t, j in enumerate(idx):
        xs_pm = []
        for sgn in (1.0, -1.0):
            v = base.copy()
            v[j] += sgn * HSTEP
            S.update_vectors(**{key: dev(v)})
            xp, _, _, _, inf2 = S.solve()
            assert inf2["status"] in (1, 2)
            xs_pm.append(host(xp))
        xp_, xm_ = xs_pm
        fds[t] = 0.5 * float((xp_ - xm_) @ (xp_ + xm_ - 2 * x_ref)) / (2 * HSTEP)
    S.close()
    adj = grad[idx]
    scale = 1e-3 * max(np.max(np.abs(grad)), np.max(np.abs(fds)), 1e-12)
    err = np.abs(adj - fds) / np.maximum(np.abs(fds), scale)
    print(f"[gpu] lasso_diff d/d{key}: {NCOORD} coordinates, max rel err {np.max(err):.2e} "
          f"(max |grad| {np.max(np.abs(grad)):.3e}, max |fd| {np.max(np.abs(fds)):.3e})", flush=True)
    assert float(np.max(err)) <= 1e-3, (idx[np.argmax(err)], adj[np.argmax(err)], fds[np.argmax(err)])
