"""Batches of problems on one pattern (qg_setup_batch / qg_solve_batch): every
problem of the batch against the oracle's solve of that problem alone, and
against the library's own solve of it alone, in both precisions; the batch
covers small fronts (lasso_s: thousands of small fronts and a 1000-wide
root), a single large front per problem (small_qp: its copies factored and
solved by one launch sequence) and second-order cones (mixed_soc: the cone
rows come back problem by problem).  Each problem stops moving at the first
iterate that passes its own test, so it ends where its own solve ends; the
shared parts (the factorization's precision, the number of refinement
corrections) change its iterates by rounding only.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import ipm as oipm  # noqa: E402
from synth import problems  # noqa: E402

pytestmark = pytest.mark.gpu

BASES = {
    "small_qp": lambda: problems.workload("small_qp"),
    "lasso_s": lambda: problems.workload("lasso_s"),
    "mixed_soc": lambda: problems.many_soc(n=400, ncones=60, q=7, nbounds=50, seed=77, windowed=False),
}


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(1.0, np.max(np.abs(b))))


@pytest.mark.parametrize("name,k", [("small_qp", 4), ("lasso_s", 3), ("mixed_soc", 3)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_matches_single_oracle_solves(name, k, prec):
    import paper_2603_29197_amd as qg
    fam = problems.family(BASES[name](), k, seed=400 + k)
    refs = [oipm.solve(pr) for pr in fam]
    print(f"[gpu] batch {name} k={k} {prec}", flush=True)
    B = qg.BatchSolver(fam, precision=qg.QG_FP64 if prec == "fp64" else qg.QG_FP32_IR, fp32_min_flops=0.0)
    x, s, y, z, info = B.solve()
    assert info["status"] == 1, info["status_name"]
    x, s, y, z = (t.cpu().numpy() for t in (x, s, y, z))
    for i, (pr, ref) in enumerate(zip(fam, refs)):
        assert ref.status == oipm.SOLVED
        ex = relerr(x[i], ref.x)
        pobj = 0.5 * x[i] @ (pr.P @ x[i] + pr.P.T @ x[i] - pr.P.diagonal() * x[i]) + pr.c @ x[i]
        eo = abs(pobj - ref.pobj) / max(1.0, abs(ref.pobj))
        # the problem's own residuals at the returned point
        rz = pr.G @ x[i] + s[i] - pr.h
        ry = pr.A @ x[i] - pr.b
        print(f"[gpu]   problem {i}: x rel err {ex:.1e} obj rel err {eo:.1e} |ry| {np.max(np.abs(ry), initial=0):.1e} "
              f"|rz| {np.max(np.abs(rz), initial=0):.1e} s'z {s[i] @ z[i]:.1e}", flush=True)
        assert ex <= 1e-6 and eo <= 1e-6, (i, ex, eo)
        assert np.max(np.abs(rz), initial=0.0) <= 1e-6 * (1 + np.max(np.abs(pr.h), initial=0.0))
        assert np.max(np.abs(ry), initial=0.0) <= 1e-6 * (1 + np.max(np.abs(pr.b), initial=0.0))
        S = qg.Solver(pr, precision=qg.QG_FP64 if prec == "fp64" else qg.QG_FP32_IR, fp32_min_flops=0.0)
        xs, _, _, _, info1 = S.solve()
        S.close()
        assert info1["status"] == 1
        e1 = relerr(x[i], xs.cpu().numpy())
        print(f"[gpu]   problem {i}: against its own solve {e1:.1e} ({info1['iters']} iterations)", flush=True)
        assert e1 <= 1e-8, (i, e1)
    B.close()


def test_batch_of_one_equals_the_single_solver():
    """k = 1: the replicated analysis is the analysis itself, so the batch handle computes the
    same iterates as qg_setup's handle, bit for bit."""
    import paper_2603_29197_amd as qg
    prob = problems.workload("lasso_s")
    B = qg.BatchSolver([prob])
    xb, sb, yb, zb, ib = B.solve()
    S = qg.Solver(prob)
    x, s, y, z, i1 = S.solve()
    assert ib["iters"] == i1["iters"]
    assert torch.equal(xb[0], x) and torch.equal(zb[0], z) and torch.equal(yb[0], y) and torch.equal(sb[0], s)
    B.close()
    S.close()


def test_batch_handle_refuses_single_problem_calls():
    import ctypes
    import paper_2603_29197_amd as qg
    fam = problems.family(problems.workload("small_qp"), 2, seed=9)
    B = qg.BatchSolver(fam)
    L = qg.lib()
    assert L.qg_solve(B.handle, None, None, None, None, None) == -6
    assert L.qg_update_vectors(B.handle, None, None, None) == -6
    B.close()
