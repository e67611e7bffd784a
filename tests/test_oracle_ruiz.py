"""Pins of the oracle's Ruiz equilibration: convergence of the scaled data to unit column and row
maxima, one factor per second-order cone, and the scaled problem's solution mapping back to the
original problem's solution (through the oracle IPM)."""
import numpy as np
import pytest

from oracle import ipm as oipm
from oracle import ruiz
from synth import problems

PROBS = {
    "small_qp": lambda: problems.small_qp(n=40, p=10, m=40, mrows=40, seed=problems.BASE_SEED + 61),
    "soc": lambda: problems.many_soc(n=60, ncones=12, q=[3, 5, 4], nbounds=10, seed=62, windowed=False),
}


def _badly_scaled(prob, seed):
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    S = 10.0 ** rng.uniform(-3, 3, prob.n)
    RA = 10.0 ** rng.uniform(-3, 3, prob.p)
    RG = 10.0 ** rng.uniform(-3, 3, prob.m)
    q = problems.Problem(**{**prob.__dict__})
    q.P = sp.csc_matrix(sp.diags(S) @ prob.P @ sp.diags(S))
    q.c = S * prob.c
    q.A = sp.csc_matrix(sp.diags(RA) @ prob.A @ sp.diags(S))
    q.b = RA * prob.b
    q.G = sp.csc_matrix(sp.diags(RG) @ prob.G @ sp.diags(S))
    q.h = RG * prob.h
    return q


def _cone_slices(prob):
    off = prob.l
    for qk in prob.q:
        yield slice(off, off + qk)
        off += qk


@pytest.mark.parametrize("name", list(PROBS))
def test_no_pass_is_the_identity(name):
    prob = PROBS[name]()
    D, E, F, k = ruiz.equilibrate(prob, 0)
    assert np.all(D == 1) and np.all(E == 1) and np.all(F == 1)
    assert k == 1.0 / max(1.0, np.max(np.abs(prob.c)))


@pytest.mark.parametrize("name", list(PROBS))
def test_passes_converge_to_unit_maxima(name):
    """Many passes on data spread over six decades: every x column of the scaled matrix, every row
    of A, every orthant row of G and every second-order cone's block of rows has largest
    magnitude 1; the factors of one cone are equal."""
    prob = _badly_scaled(PROBS[name](), 5)
    D, E, F, k = ruiz.equilibrate(prob, 60)
    sp_ = ruiz.scaled_problem(prob, D, E, F, 1.0)
    Pu = sp_.P.toarray()
    Pf = np.abs(Pu + Pu.T - np.diag(np.diag(Pu)))
    A, G = np.abs(sp_.A.toarray()), np.abs(sp_.G.toarray())
    col = np.max(np.vstack([Pf, A, G]), axis=0)
    assert np.allclose(col, 1.0, rtol=1e-9)
    assert np.allclose(A.max(axis=1), 1.0, rtol=1e-9)
    assert np.allclose(G[:prob.l].max(axis=1), 1.0, rtol=1e-9)
    for sl in _cone_slices(prob):
        assert np.allclose(G[sl].max(), 1.0, rtol=1e-9)
        assert np.all(F[sl] == F[sl.start])
    assert 0 < k <= 1 and np.max(np.abs(D * prob.c)) * k <= 1.0 + 1e-15


@pytest.mark.parametrize("name", list(PROBS))
@pytest.mark.parametrize("passes", [1, 10])
def test_scaled_solution_maps_back(name, passes):
    """Solving the scaled problem and mapping its solution back gives the original problem's
    solution (both solved by the oracle IPM to 1e-10), so the scaled data and the mapping agree."""
    prob = _badly_scaled(PROBS[name](), 7)
    tight = oipm.IPMSettings(eps_abs=1e-10, eps_rel=1e-10)
    ref = oipm.solve(prob, tight)
    D, E, F, k = ruiz.equilibrate(prob, passes)
    r = oipm.solve(ruiz.scaled_problem(prob, D, E, F, k), tight)
    assert ref.status == 1 and r.status == 1
    x, s, y, z = ruiz.unscale(D, E, F, k, r.x, r.s, r.y, r.z)
    assert np.max(np.abs(x - ref.x)) <= 1e-6 * max(1.0, np.max(np.abs(ref.x)))
    res = oipm.residuals(prob, x, s, y, z)
    ok, pres, dres, gap = oipm.stop_test(prob, res, s, 1e-8, 1e-8)
    assert ok, (pres, dres, gap)
