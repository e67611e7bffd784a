"""Host-side checks of the device library (no GPU): the C ABI loads and
exports every entry point declared in include/qg.h, and its analysis
reproduces the oracle's integer pattern bit for bit."""
import hashlib
import json
import os
import re

import numpy as np
import pytest

from oracle import kkt, symbolic
from synth import problems

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KEYS = [("perm", np.int32), ("iperm", np.int32), ("parent", np.int32), ("colcount", np.int64),
        ("super_fund", np.int32), ("super_ptr", np.int32), ("rows_ptr", np.int64), ("rows", np.int32)]


def test_library_exports_every_declared_symbol():
    from paper_2603_29197_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "qg.h")).read()
    declared = set(re.findall(r"\b(qg_[a-z_0-9]+)\s*\(", hdr))
    L = _lib.lib()
    missing = [s for s in sorted(declared) if not hasattr(L, s)]
    assert not missing, missing
    assert declared <= set(_lib.EXPORTS) | {"qg_strerror"}


def test_strerror_and_defaults():
    import paper_2603_29197_amd as qg
    s = qg.default_settings()
    assert s.eps_abs == 1e-8 and s.eps_rel == 1e-8 and s.max_iter == 100 and s.step_frac == 0.99
    assert qg.lib().qg_strerror(-2) == b"invalid sparsity pattern"


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "many_soc_s", "lasso_diff_s"])
def test_analysis_matches_oracle_bit_exact(name):
    import paper_2603_29197_amd as qg
    prob = problems.workload(name)
    a = qg.analyze(prob)
    o = symbolic.analyze(kkt.kkt_pattern(prob))
    for k, _ in KEYS:
        assert np.array_equal(a[k], getattr(o, k)), k


@pytest.mark.parametrize("seed", range(8))
def test_analysis_matches_oracle_random_socp(seed):
    import paper_2603_29197_amd as qg
    prob = problems.many_soc(n=200 + 37 * seed, ncones=40 + 5 * seed, q=3 + seed % 4, nbounds=30,
                             seed=500 + seed, windowed=bool(seed % 2))
    a = qg.analyze(prob)
    o = symbolic.analyze(kkt.kkt_pattern(prob))
    for k, _ in KEYS:
        assert np.array_equal(a[k], getattr(o, k)), k


def _check_fronts(prob, a):
    """The device fronts: a renaming of the analysis' columns that keeps the
    elimination tree order, each front a head supernode plus merged children
    (at most 16 columns, rows > 128), rows covering every column's L."""
    N = a["N"]
    fperm = a["front_perm"]
    assert np.array_equal(np.sort(fperm), np.arange(N))
    finv = np.empty(N, np.int64); finv[fperm] = np.arange(N)
    dev = finv[a["perm"]]                       # analysis column -> front column
    par = a["parent"]
    has = par >= 0
    assert np.all(dev[par[has]] > dev[has])    # every column after its descendants
    fp, frp, fr = a["front_ptr"], a["front_rows_ptr"], a["front_rows"]
    nfr = len(fp) - 1
    col2f = np.repeat(np.arange(nfr), np.diff(fp))
    Up = symbolic.permute_upper(kkt.kkt_pattern(prob), a["perm"])
    Lp, Li, _ = symbolic.l_pattern(Up, symbolic.etree(Up))
    for f in range(nfr):
        rows = fr[frp[f]:frp[f + 1]]
        k = fp[f + 1] - fp[f]
        assert np.all(np.diff(rows) > 0)
        assert np.array_equal(rows[:k], np.arange(fp[f], fp[f + 1]))
    for j in range(N):
        c = dev[j]; f = col2f[c]
        rows = fr[frp[f]:frp[f + 1]]
        need = dev[Li[Lp[j]:Lp[j + 1]]]
        assert np.all(need > c)
        assert np.all(np.isin(need, rows)), j
    # fronts are unions of supernodes: one head, merged children small and tall
    sp, rp = a["super_ptr"], a["rows_ptr"]
    ns = len(sp) - 1
    sn_front = col2f[dev[sp[:-1]]]
    for s in range(ns):
        assert np.all(col2f[dev[np.arange(sp[s], sp[s + 1])]] == sn_front[s])
    for f in range(nfr):
        sns = np.where(sn_front == f)[0]
        head = sns.max()
        if len(sns) == 1:
            rows = fr[frp[f]:frp[f + 1]]
            assert np.array_equal(np.sort(dev[a["rows"][rp[head]:rp[head + 1]]]), rows)
        for s in sns[:-1]:
            assert sp[s + 1] - sp[s] <= 16 and rp[s + 1] - rp[s] > 128
    return nfr, ns


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "lasso_diff_s", "many_soc_s"])
def test_device_fronts_are_a_valid_grouping(name):
    import paper_2603_29197_amd as qg
    prob = problems.workload(name)
    nfr, ns = _check_fronts(prob, qg.analyze(prob))
    if name.startswith("lasso"):
        assert nfr < ns          # the tall one-column children of the dense root are merged


@pytest.mark.parametrize("seed", range(3))
def test_device_fronts_random(seed):
    import paper_2603_29197_amd as qg
    prob = problems.lasso(300 + 50 * seed, 150 + 20 * seed, 0.03, seed=900 + seed)
    _check_fronts(prob, qg.analyze(prob))


@pytest.mark.parametrize("name", ["huber_s", "many_soc", "lasso", "huber_l", "many_soc@nd"])
def test_analysis_matches_oracle_digest_full_size(name):
    """Digests written by tests/golden/make_golden.py from the oracle ("@nd": nested dissection)."""
    import paper_2603_29197_amd as qg
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "patterns.json")))[name]
    wl, _, ordering = name.partition("@")
    a = qg.analyze(problems.workload(wl), qg.QG_ORDER_ND if ordering == "nd" else qg.QG_ORDER_MD)
    assert a["N"] == gold["N"] and int(a["colcount"].sum()) == gold["nnz_L"]
    for k, dt in KEYS:
        if k == "iperm":
            continue
        assert hashlib.sha256(np.ascontiguousarray(a[k], dtype=dt).tobytes()).hexdigest() == gold[k], k


@pytest.mark.parametrize("threads", ["1", "3"])
def test_analysis_does_not_depend_on_the_thread_count(threads, monkeypatch):
    """The ordering's long pivot steps (huber_s ends in a ~4000-wide dense phase) run on a pool of
    host threads; with 1 or 3 threads the result is the oracle's digest, as with the default."""
    import paper_2603_29197_amd as qg
    monkeypatch.setenv("QG_ANALYSIS_THREADS", threads)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "patterns.json")))["huber_s"]
    a = qg.analyze(problems.workload("huber_s"))
    for k, dt in KEYS:
        if k == "iperm":
            continue
        assert hashlib.sha256(np.ascontiguousarray(a[k], dtype=dt).tobytes()).hexdigest() == gold[k], k


def test_invalid_inputs_are_rejected():
    import scipy.sparse as sp
    import paper_2603_29197_amd as qg
    from paper_2603_29197_amd._lib import QGError
    prob = problems.small_qp(n=20, p=4, m=10, mrows=10)
    bad = problems.Problem(**{**prob.__dict__})
    bad.P = sp.csc_matrix(prob.P.toarray() + np.tril(np.ones((20, 20)), -1))  # not upper
    with pytest.raises(QGError) as e:
        qg.analyze(bad)
    assert e.value.code == -2
    bad = problems.Problem(**{**prob.__dict__})
    bad.l = 9                                   # l + sum(q) != m
    with pytest.raises(QGError) as e:
        qg.analyze(bad)
    assert e.value.code == -1


def _raw_setup(prob, hooks=None, settings=None):
    """qg_setup through the C ABI with host data only; returns the code.  Every case below is
    rejected by validation, which runs before any device call."""
    import ctypes
    from paper_2603_29197_amd import _lib, api
    P, A, G, q = api._args(prob)
    c = np.ascontiguousarray(prob.c, dtype=np.float64)
    b = np.ascontiguousarray(prob.b, dtype=np.float64)
    hv = np.ascontiguousarray(prob.h, dtype=np.float64)
    h = ctypes.c_void_p()
    hooks = hooks or (_lib.ALLOC_FN(), _lib.FREE_FN(), None)
    rc = _lib.lib().qg_setup(ctypes.byref(h), prob.n, prob.m, prob.p, P.ptr(), c.ctypes.data_as(_lib.c_double_p),
                             A.ptr(), b.ctypes.data_as(_lib.c_double_p), G.ptr(),
                             hv.ctypes.data_as(_lib.c_double_p), prob.l, len(prob.q),
                             q.ctypes.data_as(_lib.c_int32_p),
                             ctypes.byref(settings) if settings is not None else None, None, *hooks)
    assert not h.value
    return rc


@pytest.mark.parametrize("where", ["c", "b", "h", "P", "A", "G"])
def test_nonfinite_data_is_rejected_before_the_device(where):
    """NaN or Inf anywhere in the data gives QG_ERR_NONFINITE from qg_setup."""
    prob = problems.small_qp(n=20, p=4, m=10, mrows=10)
    for bad_value in (np.nan, np.inf):
        bad = problems.Problem(**{**prob.__dict__})
        if where in ("c", "b", "h"):
            v = getattr(prob, where).copy(); v[3] = bad_value
            setattr(bad, where, v)
        else:
            M = getattr(prob, where).copy(); M.data[2] = bad_value
            setattr(bad, where, M)
        assert _raw_setup(bad) == -3, (where, bad_value)


@pytest.mark.parametrize("ruiz,diff", [(-1, 0), (101, 0), (5, 1)])
def test_ruiz_settings_are_validated(ruiz, diff):
    """Ruiz passes outside 0..QG_RUIZ_MAX, or with the differentiable mode, give QG_ERR_ARG."""
    import paper_2603_29197_amd as qg
    prob = problems.small_qp(n=20, p=4, m=10, mrows=10)
    s = qg.default_settings(ruiz_iters=ruiz, differentiable=diff)
    assert qg.default_settings().ruiz_iters == 0
    assert _raw_setup(prob, settings=s) == -1


def test_allocator_hooks_must_come_in_pairs():
    from paper_2603_29197_amd import _lib
    prob = problems.small_qp(n=20, p=4, m=10, mrows=10)
    only_alloc = (_lib.ALLOC_FN(lambda ctx, nbytes: None), _lib.FREE_FN(), None)
    assert _raw_setup(prob, only_alloc) == -1


@pytest.mark.parametrize("name", ["small_qp", "lasso_s", "many_soc_s", "lasso_diff_s"])
def test_nested_dissection_matches_oracle_bit_exact(name):
    import paper_2603_29197_amd as qg
    prob = problems.workload(name)
    a = qg.analyze(prob, qg.QG_ORDER_ND)
    o = symbolic.analyze(kkt.kkt_pattern(prob), "nd")
    for k, _ in KEYS:
        assert np.array_equal(a[k], getattr(o, k)), k


@pytest.mark.parametrize("seed", range(6))
def test_nested_dissection_matches_oracle_random_socp(seed):
    """Windowed and random-column SOCPs large enough to be dissected (more than 256 nodes)."""
    import paper_2603_29197_amd as qg
    prob = problems.many_soc(n=900 + 137 * seed, ncones=300 + 25 * seed, q=3 + seed % 4, nbounds=200,
                             seed=700 + seed, windowed=bool(seed % 2))
    a = qg.analyze(prob, qg.QG_ORDER_ND)
    o = symbolic.analyze(kkt.kkt_pattern(prob), "nd")
    for k, _ in KEYS:
        assert np.array_equal(a[k], getattr(o, k)), k


def test_analysis_rejects_an_unknown_ordering():
    import paper_2603_29197_amd as qg
    with pytest.raises(qg.QGError):
        qg.analyze(problems.workload("small_qp"), 2)
