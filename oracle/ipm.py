"""Oracle primal-dual interior-point method for problem (1) of the paper.

The paper runs QOCO's primal-dual interior-point method and only fixes that
each iteration factors the KKT matrix of eq. (2) once, solves with it twice
and performs per-cone operations (Sec. 2, Sec. 2.2); for the method itself
it defers to Vandenberghe's cone-QP paper.  This is our reading of that
method (Mehrotra predictor-corrector with Nesterov-Todd scaling, no
homogeneous embedding, no equilibration), with every choice spelled out:

  init: factor K with W = I, solve K [x; y; z] = [-c; b; h]; s = h - Gx,
        z = z; each of s and z is shifted into the interior (see
        ``Cones.shift_interior``).
  each iteration:
    1. r_x = Px + A'y + G'z + c, r_y = Ax - b, r_z = Gx + s - h,
       mu = s'z / nu (nu = l + nsoc);
    2. stop (absolute + relative tolerances on the unscaled data):
         max(|r_y|, |r_z|) <= ea + er max(|Ax|, |b|, |Gx|, |h|, |s|),
         |r_x| <= ea + er max(|Px|, |A'y|, |G'z|, |c|),
         |s'z| <= ea + er max(1, min(|pobj|, |dobj|))
       (all infinity norms; pobj = x'Px/2 + c'x, dobj = -x'Px/2 - b'y - h'z);
    3. NT scaling W, lambda = W z; (3,3) block of K <- -W'W; factor;
    4. affine: K d = [-r_x; -r_y; -r_z + s], ds_a = -s - W'W dz_a;
    5. alpha_a = min(1, step(s, ds_a), step(z, dz_a)); sigma = (1 - alpha_a)^3;
    6. combined: d_s = -lambda o lambda - (W^-T ds_a) o (W dz_a) + sigma mu e,
       t = W'(lambda \\ d_s), K d = [-r_x; -r_y; -r_z - t], ds = t - W'W dz;
    7. alpha = min(1, 0.99 min(step(s, ds), step(z, dz)));
    8. (x, s, y, z) += alpha (dx, ds, dy, dz).
  At max_iter the result is SOLVED_INACCURATE if the tests pass with 1e-5,
  else MAX_ITER.  Every solve uses refinement (``KKTFactor.solve``).

Test infrastructure only.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from .cones import Cones, nt_scaling
from .ldl import KKTFactor, RegSettings

SOLVED = 1
SOLVED_INACCURATE = 2
MAX_ITER = -1
NUMERICAL_ERROR = -2


@dataclass
class IPMSettings:
    eps_abs: float = 1e-8
    eps_rel: float = 1e-8
    max_iter: int = 100
    step_frac: float = 0.99
    inacc_eps: float = 1e-5
    reg: RegSettings = field(default_factory=RegSettings)


@dataclass
class IPMResult:
    x: np.ndarray
    s: np.ndarray
    y: np.ndarray
    z: np.ndarray
    status: int
    iters: int
    pobj: float
    dobj: float
    pres: float
    dres: float
    gap: float
    factor: KKTFactor
    history: list
    ms_per_iter: float = 0.0


def _inf(v):
    return float(np.max(np.abs(v), initial=0.0))


def residuals(prob, x, s, y, z):
    Px = prob.P @ x + prob.P.T @ x - prob.P.diagonal() * x   # P given as upper triangle
    ATy = prob.A.T @ y
    GTz = prob.G.T @ z
    Ax = prob.A @ x
    Gx = prob.G @ x
    rx = Px + ATy + GTz + prob.c
    ry = Ax - prob.b
    rz = Gx + s - prob.h
    xPx = float(x @ Px)
    pobj = 0.5 * xPx + float(prob.c @ x)
    dobj = -0.5 * xPx - float(prob.b @ y) - float(prob.h @ z)
    return dict(rx=rx, ry=ry, rz=rz, Px=Px, ATy=ATy, GTz=GTz, Ax=Ax, Gx=Gx, pobj=pobj, dobj=dobj,
                sz=float(s @ z))


def stop_test(prob, r, s, eps_abs, eps_rel):
    pres = max(_inf(r["ry"]), _inf(r["rz"]))
    dres = _inf(r["rx"])
    gap = abs(r["sz"])
    pscale = max(_inf(r["Ax"]), _inf(prob.b), _inf(r["Gx"]), _inf(prob.h), _inf(s))
    dscale = max(_inf(r["Px"]), _inf(r["ATy"]), _inf(r["GTz"]), _inf(prob.c))
    gscale = max(1.0, min(abs(r["pobj"]), abs(r["dobj"])))
    ok = (pres <= eps_abs + eps_rel * pscale and dres <= eps_abs + eps_rel * dscale
          and gap <= eps_abs + eps_rel * gscale)
    return ok, pres, dres, gap


def initial_point(prob, cones: Cones, F: KKTFactor):
    n, p = prob.n, prob.p
    F.factor(-np.ones(prob.l), [-np.eye(qk) for qk in prob.q])
    rhs = np.concatenate([-prob.c, prob.b, prob.h])
    sol, _ = F.solve(rhs)
    x, y, z = sol[:n], sol[n:n + p], sol[n + p:]
    s = prob.h - prob.G @ x
    return x, cones.shift_interior(s), y, cones.shift_interior(z)


def solve(prob, settings: IPMSettings | None = None, pattern=None, verbose: bool = False,
          max_iter: int | None = None) -> IPMResult:
    st = settings or IPMSettings()
    if max_iter is not None:
        st = IPMSettings(st.eps_abs, st.eps_rel, max_iter, st.step_frac, st.inacc_eps, st.reg)
    cones = Cones(prob.l, prob.q)
    n, p = prob.n, prob.p
    F = KKTFactor(prob, pattern=pattern, reg=st.reg)
    x, s, y, z = initial_point(prob, cones, F)
    e = cones.identity()
    hist = []
    status = MAX_ITER
    it = 0
    t_iter = []
    while True:
        r = residuals(prob, x, s, y, z)
        ok, pres, dres, gap = stop_test(prob, r, s, st.eps_abs, st.eps_rel)
        if verbose:
            print(f"it {it:3d} pobj {r['pobj']:+.8e} dobj {r['dobj']:+.8e} pres {pres:.2e} "
                  f"dres {dres:.2e} gap {gap:.2e}")
        if not np.all(np.isfinite([pres, dres, gap])):
            status = NUMERICAL_ERROR
            break
        if ok:
            status = SOLVED
            break
        if it >= st.max_iter:
            ok5, *_ = stop_test(prob, r, s, st.inacc_eps, st.inacc_eps)
            status = SOLVED_INACCURATE if ok5 else MAX_ITER
            break
        t0 = time.perf_counter()
        mu = r["sz"] / cones.nu if cones.nu > 0 else 0.0
        sc = nt_scaling(cones, s, z)
        orth, blocks = sc.block33()
        F.factor(orth, blocks)
        # affine (predictor) direction
        rhs = np.concatenate([-r["rx"], -r["ry"], -r["rz"] + s])
        d, ir1 = F.solve(rhs)
        dx_a, dy_a, dz_a = d[:n], d[n:n + p], d[n + p:]
        ds_a = -s - sc.WtW(dz_a)
        alpha_a = min(1.0, cones.max_step(s, ds_a), cones.max_step(z, dz_a))
        sigma = min(1.0, max(0.0, (1.0 - alpha_a) ** 3))
        # combined (corrector) direction
        lam = sc.lam
        dsv = -cones.jordan(lam, lam) - cones.jordan(sc.Winv(ds_a), sc.W(dz_a)) + sigma * mu * e
        t = sc.W(cones.inv_jordan(lam, dsv))
        rhs = np.concatenate([-r["rx"], -r["ry"], -r["rz"] - t])
        d, ir2 = F.solve(rhs)
        dx, dy, dz = d[:n], d[n:n + p], d[n + p:]
        ds = t - sc.WtW(dz)
        alpha = min(1.0, st.step_frac * min(cones.max_step(s, ds), cones.max_step(z, dz)))
        x = x + alpha * dx
        s = s + alpha * ds
        y = y + alpha * dy
        z = z + alpha * dz
        t_iter.append(time.perf_counter() - t0)
        hist.append(dict(it=it, mu=mu, alpha_a=alpha_a, sigma=sigma, alpha=alpha, ir=(ir1, ir2),
                         nreg=F.nreg, pres=pres, dres=dres, gap=gap))
        it += 1
    res = IPMResult(x=x, s=s, y=y, z=z, status=status, iters=it, pobj=r["pobj"], dobj=r["dobj"],
                    pres=pres, dres=dres, gap=gap, factor=F, history=hist,
                    ms_per_iter=1e3 * float(np.median(t_iter)) if t_iter else 0.0)
    return res
