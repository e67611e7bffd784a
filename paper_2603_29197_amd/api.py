"""Python front end of the C ABI: a solver object holding one handle, the
host-only analysis, and a torch.autograd.Function for gradients through the
solution.  Marshalling only: every numeric step runs in the HIP library.

Problem data follow the paper's setup call (Sec. 2.1, Listing 1):
``(n, m, p, P, c, A, b, G, h, l, nsoc, q)`` with P the upper triangle
(scipy CSC matrices, numpy vectors).
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import QG_FP32_IR, QG_FP64, check, lib, qg_csc, qg_info, qg_pattern, qg_settings


class _Csc:
    """Keeps the numpy buffers of one CSC matrix alive while C reads them."""

    def __init__(self, M, nrow, ncol):
        if M is None:
            self.s = None
            return
        M = M.tocsc()
        M.sort_indices()
        self.colptr = np.ascontiguousarray(M.indptr, dtype=np.int64)
        self.rowind = np.ascontiguousarray(M.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(M.data, dtype=np.float64)
        self.s = qg_csc(nrow, ncol, self.colptr.ctypes.data_as(_lib.c_int64_p),
                        self.rowind.ctypes.data_as(_lib.c_int32_p), self.val.ctypes.data_as(_lib.c_double_p))

    def ptr(self):
        return ctypes.byref(self.s) if self.s is not None else None


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(_lib.c_double_p)


def default_settings(**kw) -> qg_settings:
    s = qg_settings()
    lib().qg_default_settings(ctypes.byref(s))
    for k, v in kw.items():
        if not hasattr(s, k):
            raise KeyError(k)
        setattr(s, k, v)
    return s


def _pattern_dict(pt: qg_pattern) -> dict:
    N, ns, nf = pt.N, pt.nsuper, pt.nsuper_fund
    arr = lambda p, n, dt: np.ctypeslib.as_array(p, shape=(n,)).astype(dt).copy() if n > 0 else np.zeros(0, dt)
    rows_ptr = arr(pt.rows_ptr, ns + 1, np.int64)
    return dict(N=N, perm=arr(pt.perm, N, np.int32), iperm=arr(pt.iperm, N, np.int32),
                parent=arr(pt.parent, N, np.int32), colcount=arr(pt.colcount, N, np.int64),
                super_fund=arr(pt.super_fund, nf + 1, np.int32), super_ptr=arr(pt.super_ptr, ns + 1, np.int32),
                rows_ptr=rows_ptr, rows=arr(pt.rows, int(rows_ptr[-1]), np.int32),
                **_fronts_dict(pt, arr))


def _fronts_dict(pt: qg_pattern, arr) -> dict:
    nfr = pt.nfront
    frp = arr(pt.front_rows_ptr, nfr + 1, np.int64)
    return dict(front_perm=arr(pt.front_perm, pt.N, np.int32), front_ptr=arr(pt.front_ptr, nfr + 1, np.int32),
                front_rows_ptr=frp, front_rows=arr(pt.front_rows, int(frp[-1]), np.int32),
                nchain_front=int(pt.nchain_front))


def _args(prob):
    P = _Csc(prob.P if prob.P.nnz > 0 else prob.P, prob.n, prob.n)
    A = _Csc(prob.A, prob.p, prob.n) if prob.p > 0 else _Csc(None, 0, 0)
    G = _Csc(prob.G, prob.m, prob.n) if prob.m > 0 else _Csc(None, 0, 0)
    q = np.ascontiguousarray(np.asarray(prob.q, dtype=np.int32)) if len(prob.q) else np.zeros(1, np.int32)
    return P, A, G, q


def analyze(prob, ordering: int = 0) -> dict:
    """Host-only analysis (no device): the integer pattern of qg_pattern
    (ordering: QG_ORDER_MD or QG_ORDER_ND)."""
    P, A, G, q = _args(prob)
    h = ctypes.c_void_p()
    check(lib().qg_analyze(ctypes.byref(h), prob.n, prob.m, prob.p, P.ptr(), A.ptr(), G.ptr(), prob.l,
                           len(prob.q), q.ctypes.data_as(_lib.c_int32_p), int(ordering)), "qg_analyze")
    try:
        pt = qg_pattern()
        check(lib().qg_symbolic_pattern(h, ctypes.byref(pt)), "qg_symbolic_pattern")
        return _pattern_dict(pt)
    finally:
        lib().qg_symbolic_free(h)


class TorchDeviceMemory:
    """Device memory for a handle from PyTorch's caching allocator: every block
    the library asks for is a uint8 tensor kept alive here until the library
    gives it back, so torch's memory counters see the handle's footprint.
    ``source(nbytes)`` may replace the default tensor factory (it returns a
    tensor of at least ``nbytes`` bytes, or None to refuse)."""

    ALIGN = 256

    def __init__(self, torch, source=None):
        self.torch = torch
        self.source = source
        self.live = {}
        self.calls = 0
        self.c_alloc = _lib.ALLOC_FN(self._alloc)
        self.c_free = _lib.FREE_FN(self._free)

    def _alloc(self, ctx, nbytes):
        self.calls += 1
        try:
            t = self.source(int(nbytes)) if self.source is not None else \
                self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")
        except Exception:      # an allocator failure becomes QG_ERR_OOM in the library
            return None
        if t is None:
            return None
        ptr = int(t.data_ptr())
        if ptr % self.ALIGN:
            return None
        self.live[ptr] = t
        return ptr

    def _free(self, ctx, ptr):
        if ptr:
            self.live.pop(int(ptr), None)

    @property
    def nbytes(self) -> int:
        return sum(int(t.numel()) for t in self.live.values())


class Solver:
    """One device handle (qg_setup ... qg_cleanup) for a fixed sparsity pattern.

    ``memory``: "torch" (default) routes every device allocation of the handle
    through PyTorch's caching allocator; "hip" lets the library call hipMalloc;
    a callable ``f(nbytes) -> tensor | None`` supplies the blocks itself."""

    def __init__(self, prob, settings: Optional[qg_settings] = None, stream=None, memory="torch", **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        self.torch = torch
        self.prob = prob
        self.n, self.m, self.p = prob.n, prob.m, prob.p
        self.N = self.n + self.m + self.p
        self.settings = settings if settings is not None else default_settings(**kw)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.nsolve = 0          # solves run on this handle (checked by the autograd functions)
        P, A, G, q = _args(prob)
        self._keep = (P, A, G, q)
        self.handle = ctypes.c_void_p()
        if memory == "hip":
            self.memory = None
            hooks = (_lib.ALLOC_FN(), _lib.FREE_FN(), None)
        else:
            self.memory = TorchDeviceMemory(torch, None if memory == "torch" else memory)
            hooks = (self.memory.c_alloc, self.memory.c_free, None)
        c = np.ascontiguousarray(prob.c, dtype=np.float64)
        b = np.ascontiguousarray(prob.b, dtype=np.float64)
        hv = np.ascontiguousarray(prob.h, dtype=np.float64)
        check(lib().qg_setup(ctypes.byref(self.handle), prob.n, prob.m, prob.p, P.ptr(),
                             c.ctypes.data_as(_lib.c_double_p), A.ptr(),
                             b.ctypes.data_as(_lib.c_double_p) if prob.p else None, G.ptr(),
                             hv.ctypes.data_as(_lib.c_double_p) if prob.m else None, prob.l, len(prob.q),
                             q.ctypes.data_as(_lib.c_int32_p), ctypes.byref(self.settings),
                             ctypes.c_void_p(self.stream.cuda_stream), *hooks), "qg_setup")
        self.info = None

    # -- lifecycle ------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().qg_cleanup(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty(self, k):
        return self.torch.empty(max(k, 1), dtype=self.torch.float64, device="cuda")

    @staticmethod
    def _vp(t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    # -- main calls -----------------------------------------------------------
    def set_settings(self, **kw):
        for k, v in kw.items():
            if not hasattr(self.settings, k):
                raise KeyError(k)
            setattr(self.settings, k, v)
        check(lib().qg_set_settings(self.handle, ctypes.byref(self.settings)), "qg_set_settings")

    def update(self, Pval=None, c=None, Aval=None, b=None, Gval=None, h=None):
        keep = [None if v is None else np.ascontiguousarray(v, dtype=np.float64) for v in (Pval, c, Aval, b, Gval, h)]
        self._matrix_tokens = {}
        check(lib().qg_update(self.handle, *[_dptr(v) for v in keep]), "qg_update")

    def update_vectors(self, c=None, b=None, h=None):
        """c, b, h from device tensors (float64 on the handle's device), no host round trip."""
        t = self.torch
        keep = [None if v is None else v.detach().to(device="cuda", dtype=t.float64).contiguous()
                for v in (c, b, h)]
        for v, w in zip(keep, (self.n, self.p, self.m)):
            if v is not None and v.numel() != w:
                raise ValueError("vector length does not match the problem")
        check(lib().qg_update_vectors(self.handle, *[self._vp(v) for v in keep]), "qg_update_vectors")

    def solve(self):
        x, s, y, z = self._empty(self.n), self._empty(self.m), self._empty(self.p), self._empty(self.m)
        info = qg_info()
        self.nsolve += 1
        check(lib().qg_solve(self.handle, self._vp(x), self._vp(s), self._vp(y), self._vp(z),
                             ctypes.byref(info)), "qg_solve")
        self.info = info.as_dict()
        return x[:self.n], s[:self.m], y[:self.p], z[:self.m], self.info

    def backward(self, dl_dx, want_P: bool = True, want_A: bool = False, want_G: bool = False,
                 dl_dy=None, dl_dz=None, dl_ds=None):
        """Gradients of L(x*, y*, z*, s*) with dl_dx = dL/dx* (and optionally dL/dy*, dL/dz*,
        dL/ds*): dc, dh, db, and the values of P, A and G on their patterns (dP, dA, dG; None
        unless asked for and the matrix has entries)."""
        t = self.torch
        dl_dx = dl_dx.to(device="cuda", dtype=t.float64).contiguous()
        extra = [None if v is None else v.to(device="cuda", dtype=t.float64).contiguous()
                 for v in (dl_dy, dl_dz, dl_ds)]
        dc, dh, db = self._empty(self.n), self._empty(self.m), self._empty(self.p)
        nnz = {k: int(getattr(self.prob, k).nnz) for k in ("P", "A", "G")}
        want = {"P": want_P, "A": want_A, "G": want_G}
        out = {k: (self._empty(nnz[k]) if (want[k] and nnz[k] > 0) else None) for k in ("P", "A", "G")}
        check(lib().qg_backward_full(self.handle, self._vp(dl_dx), *[self._vp(v) for v in extra],
                                     self._vp(dc), self._vp(dh), self._vp(db), self._vp(out["P"]),
                                     self._vp(out["A"]), self._vp(out["G"])), "qg_backward_full")
        res = dict(dc=dc[:self.n], dh=dh[:self.m], db=db[:self.p])
        for k in ("P", "A", "G"):
            res["d" + k] = None if out[k] is None else out[k][:nnz[k]]
        return res

    def backward_batch(self, dl_dx, want_P: bool = True, want_A: bool = False, want_G: bool = False,
                       dl_dy=None, dl_dz=None, dl_ds=None):
        """k losses at once: dl_dx is (k, n), the optional dl_dy, dl_dz, dl_ds are (k, p), (k, m),
        (k, m); returns the gradients of backward() stacked along a leading axis of length k."""
        t = self.torch
        dl_dx = dl_dx.to(device="cuda", dtype=t.float64).contiguous()
        k = int(dl_dx.shape[0])
        assert dl_dx.shape == (k, self.n)
        extra = [None if v is None else v.to(device="cuda", dtype=t.float64).contiguous()
                 for v in (dl_dy, dl_dz, dl_ds)]
        for v, w in zip(extra, (self.p, self.m, self.m)):
            assert v is None or v.shape == (k, w)
        nnz = {key: int(getattr(self.prob, key).nnz) for key in ("P", "A", "G")}
        want = {"P": want_P, "A": want_A, "G": want_G}
        new = lambda w: t.empty((k, w), dtype=t.float64, device="cuda")
        dc, dh, db = new(self.n), new(self.m), new(self.p)
        out = {key: (new(nnz[key]) if (want[key] and nnz[key] > 0) else None) for key in ("P", "A", "G")}
        vp = lambda v: None if v is None or v.numel() == 0 else ctypes.c_void_p(v.data_ptr())
        check(lib().qg_backward_batch(self.handle, k, vp(dl_dx), *[vp(v) for v in extra], vp(dc), vp(dh),
                                      vp(db), vp(out["P"]), vp(out["A"]), vp(out["G"])), "qg_backward_batch")
        res = dict(dc=dc, dh=dh, db=db)
        for key in ("P", "A", "G"):
            res["d" + key] = out[key]
        return res

    def pattern(self) -> dict:
        pt = qg_pattern()
        check(lib().qg_get_pattern(self.handle, ctypes.byref(pt)), "qg_get_pattern")
        return _pattern_dict(pt)

    # -- step-level entry points ------------------------------------------------
    def step_scaling(self, s, z, want_lam=True, block=0):
        lam = self._empty(self.m) if want_lam else None
        check(lib().qg_step_scaling(self.handle, self._vp(s), self._vp(z), self._vp(lam), block), "qg_step_scaling")
        return None if lam is None else lam[:self.m]

    def step_get_kkt(self) -> np.ndarray:
        nnz = ctypes.c_int64(0)
        check(lib().qg_step_get_kkt(self.handle, None, ctypes.byref(nnz)), "qg_step_get_kkt")
        out = np.empty(nnz.value)
        check(lib().qg_step_get_kkt(self.handle, out.ctypes.data_as(_lib.c_double_p), None), "qg_step_get_kkt")
        return out

    def step_factor(self, precision=QG_FP64) -> int:
        nreg = ctypes.c_int(0)
        check(lib().qg_step_factor(self.handle, precision, ctypes.byref(nreg)), "qg_step_factor")
        return nreg.value

    def step_get_factor(self, Lp: np.ndarray, Li: np.ndarray):
        Lp = np.ascontiguousarray(Lp, dtype=np.int64)
        Li = np.ascontiguousarray(Li, dtype=np.int32)
        Lx = np.empty(len(Li))
        D = np.empty(len(Lp) - 1)
        check(lib().qg_step_get_factor(self.handle, Lp.ctypes.data_as(_lib.c_int64_p),
                                       Li.ctypes.data_as(_lib.c_int32_p), Lx.ctypes.data_as(_lib.c_double_p),
                                       D.ctypes.data_as(_lib.c_double_p)), "qg_step_get_factor")
        return Lx, D

    def step_solve(self, rhs, refine=0):
        x = self._empty(self.N)
        steps = ctypes.c_int(0)
        check(lib().qg_step_solve(self.handle, self._vp(rhs), self._vp(x), refine, ctypes.byref(steps)),
              "qg_step_solve")
        return x[:self.N], steps.value

    def step_max_step(self, u, du) -> float:
        a = ctypes.c_double(0.0)
        check(lib().qg_step_max_step(self.handle, self._vp(u), self._vp(du), ctypes.byref(a)), "qg_step_max_step")
        return a.value

    def step_cone_op(self, op: int, u, v=None):
        out = self._empty(self.m)
        check(lib().qg_step_cone_op(self.handle, op, self._vp(u), self._vp(v), self._vp(out)), "qg_step_cone_op")
        return out[:self.m]

    def step_corrector(self, ds_a, dz_a, sigma_mu: float):
        t = self._empty(self.m)
        check(lib().qg_step_corrector(self.handle, self._vp(ds_a), self._vp(dz_a), float(sigma_mu), self._vp(t)),
              "qg_step_corrector")
        return t[:self.m]


class BatchSolver:
    """k problems on one sparsity pattern solved together (qg_setup_batch / qg_solve_batch):
    the analysis of one problem is replicated, each iteration factors and solves all k at once.
    ``probs``: problems with identical n, m, p, cones and patterns of P, A, G."""

    def __init__(self, probs, settings: Optional[qg_settings] = None, stream=None, memory="torch", **kw):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("a HIP device is required")
        if not probs:
            raise ValueError("empty batch")
        p0 = probs[0]
        for q in probs[1:]:
            same = (q.n, q.m, q.p, q.l, list(q.q)) == (p0.n, p0.m, p0.p, p0.l, list(p0.q))
            for M0, M1 in ((p0.P, q.P), (p0.A, q.A), (p0.G, q.G)):
                same = same and np.array_equal(M0.indptr, M1.indptr) and np.array_equal(M0.indices, M1.indices)
            if not same:
                raise ValueError("the problems of a batch must share sizes, cones and sparsity patterns")
        self.torch = torch
        self.k, self.n, self.m, self.p = len(probs), p0.n, p0.m, p0.p
        self.settings = settings if settings is not None else default_settings(**kw)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        P, A, G, q = _args(p0)
        # value sets back to back on the shared pattern
        for csc, name in ((P, "P"), (A, "A"), (G, "G")):
            if csc.s is not None:
                csc.val = np.ascontiguousarray(np.concatenate([getattr(pr, name).tocsc().data for pr in probs]),
                                               dtype=np.float64)
                csc.s.val = csc.val.ctypes.data_as(_lib.c_double_p)
        c = np.ascontiguousarray(np.concatenate([pr.c for pr in probs]), dtype=np.float64)
        b = np.ascontiguousarray(np.concatenate([pr.b for pr in probs]), dtype=np.float64)
        hv = np.ascontiguousarray(np.concatenate([pr.h for pr in probs]), dtype=np.float64)
        self._keep = (P, A, G, q, c, b, hv)
        self.handle = ctypes.c_void_p()
        if memory == "hip":
            self.memory = None
            hooks = (_lib.ALLOC_FN(), _lib.FREE_FN(), None)
        else:
            self.memory = TorchDeviceMemory(torch, None if memory == "torch" else memory)
            hooks = (self.memory.c_alloc, self.memory.c_free, None)
        check(lib().qg_setup_batch(ctypes.byref(self.handle), self.k, p0.n, p0.m, p0.p, P.ptr(),
                                   c.ctypes.data_as(_lib.c_double_p), A.ptr(),
                                   b.ctypes.data_as(_lib.c_double_p) if p0.p else None, G.ptr(),
                                   hv.ctypes.data_as(_lib.c_double_p) if p0.m else None, p0.l, len(p0.q),
                                   q.ctypes.data_as(_lib.c_int32_p), ctypes.byref(self.settings),
                                   ctypes.c_void_p(self.stream.cuda_stream), *hooks), "qg_setup_batch")
        self.info = None

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            lib().qg_cleanup(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_settings(self, **kw):
        for key, v in kw.items():
            if not hasattr(self.settings, key):
                raise KeyError(key)
            setattr(self.settings, key, v)
        check(lib().qg_set_settings(self.handle, ctypes.byref(self.settings)), "qg_set_settings")

    def solve(self):
        """Returns x (k x n), s (k x m), y (k x p), z (k x m) as device tensors and the info dict."""
        t = self.torch
        mk = lambda w: t.empty(max(self.k * w, 1), dtype=t.float64, device="cuda")
        x, s, y, z = mk(self.n), mk(self.m), mk(self.p), mk(self.m)
        info = qg_info()
        vp = lambda a: ctypes.c_void_p(a.data_ptr())
        check(lib().qg_solve_batch(self.handle, vp(x), vp(s), vp(y), vp(z), ctypes.byref(info)), "qg_solve_batch")
        self.info = info.as_dict()
        shape = lambda a, w: a[:self.k * w].reshape(self.k, w)
        return shape(x, self.n), shape(s, self.m), shape(y, self.p), shape(z, self.m), self.info


def _autograd_function():
    import torch

    def _forward(ctx, c, h, b, Pval, solver, AG):
        Aval = AG[0] if len(AG) > 0 else None
        Gval = AG[1] if len(AG) > 1 else None
        ctx.n_extra = len(AG)
        # matrix values (fixed pattern) go through the host only when they differ from the values
        # the handle holds; the vectors are copied device to device
        token = lambda v: None if v is None else (v.data_ptr(), v._version, tuple(v.shape))
        mats = {"Pval": Pval, "Aval": Aval, "Gval": Gval}
        held = getattr(solver, "_matrix_tokens", {})
        changed = {k: v.detach().cpu().numpy() for k, v in mats.items() if v is not None and held.get(k) != token(v)}
        if changed:
            solver.update(**changed)
            solver._matrix_tokens = {**held, **{k: token(mats[k]) for k in changed}}
        solver.update_vectors(c=c, b=b, h=h)
        if not solver.settings.differentiable:
            solver.set_settings(differentiable=1)
        x, s, y, z, info = solver.solve()
        if info["status"] not in (1, 2):
            raise RuntimeError(f"QGSolve: the solve ended with status {info['status_name']}; there is no "
                               "solution to differentiate")
        solver.last = (x, s, y, z, info)
        ctx.solver = solver
        ctx.solve_id = solver.nsolve
        ctx.has = (Pval is not None, Aval is not None, Gval is not None)
        return x

    def _check_state(ctx):
        if ctx.solver.nsolve != ctx.solve_id:
            raise RuntimeError("QGSolve backward: the solver has run another solve since this forward, so its "
                               "stored factorization and iterate belong to that solve; use one Solver per "
                               "differentiated solve, or call backward before solving again")

    class QGSolve(torch.autograd.Function):
        """x* = QGSolve.apply(c, h, b, Pval, solver[, Aval, Gval]): forward
        updates the values (fixed pattern) and solves; backward returns
        dL/dc, dL/dh, dL/db and dL/d(P, A, G values) from one adjoint solve
        on the stored factor (None for value arrays passed as None)."""

        @staticmethod
        def forward(ctx, c, h, b, Pval, solver, *AG):
            return _forward(ctx, c, h, b, Pval, solver, AG).clone()

        @staticmethod
        def backward(ctx, gx):
            _check_state(ctx)
            hP, hA, hG = ctx.has
            g = ctx.solver.backward(gx, want_P=hP, want_A=hA, want_G=hG)
            clone = lambda v, has: v.clone() if (has and v is not None) else None
            extra = (clone(g["dA"], hA), clone(g["dG"], hG))[:ctx.n_extra]
            return (g["dc"].clone(), g["dh"].clone(), g["db"].clone(), clone(g["dP"], hP), None) + extra

    class QGSolveAll(torch.autograd.Function):
        """(x*, y*, z*, s*) = QGSolveAll.apply(c, h, b, Pval, solver[, Aval, Gval]): as QGSolve,
        for losses of the whole solution (one adjoint solve with the four output gradients)."""

        @staticmethod
        def forward(ctx, c, h, b, Pval, solver, *AG):
            x = _forward(ctx, c, h, b, Pval, solver, AG)
            _, s, y, z, _ = solver.last
            return x.clone(), y.clone(), z.clone(), s.clone()

        @staticmethod
        def backward(ctx, gx, gy, gz, gs):
            _check_state(ctx)
            hP, hA, hG = ctx.has
            g = ctx.solver.backward(gx, want_P=hP, want_A=hA, want_G=hG, dl_dy=gy, dl_dz=gz, dl_ds=gs)
            clone = lambda v, has: v.clone() if (has and v is not None) else None
            extra = (clone(g["dA"], hA), clone(g["dG"], hG))[:ctx.n_extra]
            return (g["dc"].clone(), g["dh"].clone(), g["db"].clone(), clone(g["dP"], hP), None) + extra

    return QGSolve, QGSolveAll


class _Lazy:
    def __init__(self, which: int):
        self.which = which
        self.f = None

    def apply(self, *args):
        if self.f is None:
            self.f = _autograd_function()[self.which]
        return self.f.apply(*args)


QGSolve = _Lazy(0)
QGSolveAll = _Lazy(1)
