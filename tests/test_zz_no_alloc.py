"""The entry point that allocates nothing (qg_max_step_noalloc), through the
C ABI: the same maximum step as the handle's qg_step_max_step on the same
(u, du), on two calls in a row, the second with a smaller input (the shared
device array keeps the first call's partial minima), and its size and
argument errors.
"""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cones as oc  # noqa: E402
from synth import problems  # noqa: E402

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def soc_offsets(prob):
    return torch.as_tensor(np.concatenate([[prob.l], prob.l + np.cumsum(prob.q)]).astype(np.int32),
                           device="cuda")


def noalloc_step(prob, u, du):
    import paper_2603_29197_amd as qg
    off = soc_offsets(prob) if prob.nsoc else None
    a = ctypes.c_double(-1.0)
    rc = qg.lib().qg_max_step_noalloc(prob.l, prob.nsoc, off.data_ptr() if off is not None else None,
                                      u.data_ptr(), du.data_ptr(), ctypes.byref(a), None)
    assert rc == 0, qg.lib().qg_strerror(rc)
    return a.value


def bigger():
    # 2309 cone units over ten workgroups: orthant entries, cones of 4 (one thread each) and cones
    # of 40, 64 and 300 entries (one wavefront each, several in one wavefront's 64 units)
    q = [4] * 600 + [64, 40, 300] + [4] * 900 + [64] * 4 + [40, 40, 4]
    return problems.many_soc(n=3000, q=q, nbounds=800, seed=91, windowed=False)


def smaller():
    return problems.many_soc(n=400, q=[3, 64, 31, 257, 32, 5, 100, 33, 700, 2, 65, 4, 129],
                             nbounds=100, seed=78, windowed=False)


def test_noalloc_max_step_matches_the_handle_on_two_calls():
    import paper_2603_29197_amd as qg
    for call, make in enumerate((bigger, smaller)):
        prob = make()
        units = prob.l + prob.nsoc
        print(f"[gpu] noalloc call {call}: l={prob.l} nsoc={prob.nsoc} units={units} m={prob.m}", flush=True)
        S = qg.Solver(prob)
        _, s, _, _ = problems.random_point(prob, 5 + call)
        rng = np.random.default_rng(6 + call)
        cn = oc.Cones(prob.l, prob.q)
        for scale in (0.1, 1.0, 10.0):
            du = scale * rng.standard_normal(prob.m)
            u_d, du_d = dev(s), dev(du)
            want = S.step_max_step(u_d, du_d)
            got = noalloc_step(prob, u_d, du_d)
            ref = cn.max_step(s, du)
            print(f"[gpu]   scale {scale}: noalloc {got!r} handle {want!r} oracle {ref!r}", flush=True)
            assert (np.isinf(got) and np.isinf(want)) or abs(got - want) <= 1e-14 * max(1.0, want)
            assert (np.isinf(got) and np.isinf(ref)) or abs(got - ref) <= 1e-12 * max(1.0, ref)
        # an unbounded direction (du inside the cone) gives +inf
        assert np.isinf(noalloc_step(prob, dev(s), dev(s)))
        S.close()


def test_noalloc_orthant_only_and_empty():
    import paper_2603_29197_amd as qg
    rng = np.random.default_rng(3)
    u = rng.uniform(0.5, 2.0, 1000)
    du = rng.standard_normal(1000)
    a = ctypes.c_double(0.0)
    ud, dud = dev(u), dev(du)
    assert qg.lib().qg_max_step_noalloc(1000, 0, None, ud.data_ptr(), dud.data_ptr(), ctypes.byref(a), None) == 0
    neg = du < 0
    assert a.value == np.min(-u[neg] / du[neg])
    assert qg.lib().qg_max_step_noalloc(0, 0, None, None, None, ctypes.byref(a), None) == 0
    assert np.isinf(a.value)


def test_noalloc_rejects_sizes_beyond_its_capacity():
    import paper_2603_29197_amd as qg
    from paper_2603_29197_amd._lib import QG_NOALLOC_MAX_UNITS
    a = ctypes.c_double(0.0)
    L = qg.lib()
    assert L.qg_max_step_noalloc(QG_NOALLOC_MAX_UNITS + 1, 0, None, None, None, ctypes.byref(a), None) == -8
    assert L.qg_max_step_noalloc(-1, 0, None, None, None, ctypes.byref(a), None) == -1
    assert L.qg_max_step_noalloc(4, 1, None, None, None, ctypes.byref(a), None) == -1
    assert L.qg_max_step_noalloc(4, 0, None, None, None, None, None) == -1
    assert L.qg_strerror(-8) == b"input exceeds a fixed capacity"
