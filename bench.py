"""Benchmark of the Newton step on one MI355X.

Workload: the Huber regression QP of the large-QP configuration -- variables
(x, u, v, w), Ax = F x - u - v = g, -w <= v <= w, objective 1/2 |u|^2 + 1'w,
F with 40 N(0,1) entries per row, g = F x_true + N(0,1) with 5% outliers --
at F 100000 x 40000 (n = 340000, p = 100000, m = 200000, KKT dimension
640000, a dense root front of about 40000 columns), seeded and synthetic.
The configuration's own size (F 500000 x 200000) ends in a ~2e5-wide root:
2.7e15 flops per factorization, about 17 s at the FP32 matrix-core peak,
and its host analysis alone takes hours; this instance is the largest of
the same generator whose benchmark fits in minutes.

One step = one Newton step of the interior-point method (residuals, NT
scaling and the (3,3) block, one factorization, the affine and combined
refined solves, the cone kernels, the update), with the problem resident on
the device.  The timed region is exactly K Newton steps in FP32+IR mode
(consecutive solves from the initial point, the last one cut at the step
count); ``value`` is the median Newton-step time (HIP events) over those K
steps.  The plain-FP64 mode is timed the same way (same W and K) and
reported beside it, and one full solve to the 1e-8 stopping test is run in
each mode for the solve time.  The roofline entry covers the dominant
kernel, the MFMA trailing update of the large fronts, timed per launch with
HIP events in a separate, short profiled solve.  The CPU baseline is the
FP64 oracle's up-looking factorization of the same KKT matrix, run on a
bounded prefix of its rows and scaled by exact per-row operation counts.
The other configurations (small QP, lasso, many-SOC, and the
differentiation workload with its adjoint) are reported under "configs".

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extra]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton-step ms (factor+solve) & solve s to 1e-8 gap: FP32+IR vs FP64, 1 MI355X"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
PEAK_GBS = 8000.0
# HBM bytes per launch of trail_update on the benchmark workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs, each scaled by what the counter reads for a plain device copy of known size.
# Counters describe one build of the kernel and one workload: None until they are taken for both.
# HBM bytes per launch of the FP32 128x128 kernel on the default workload: FETCH_SIZE + WRITE_SIZE, each scaled
# by its reading for a 256 MiB device copy (rocprofv3 counter runs of this bench; null once the kernel or the
# workload changes)
TRAFFIC_BYTES_PER_LAUNCH = {"fp32": 2.367e9, "fp64": None}
WORKLOAD = "huber_l"
WORKLOAD_TEXT = ("Huber QP (large-QP configuration's generator) F 100000x40000, 40 nnz per row, 5% outliers "
                 "(n=340000, p=100000, m=200000, N_K=640000); the configuration's F 500000x200000 needs "
                 "~2.7e15 flops per factorization and hours of host analysis")
GOLD = os.path.join(ROOT, "tests", "golden")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def med(xs):
    return float(statistics.median(xs)) if xs else 0.0


def cpu_baseline(prob, name: str, seconds: float):
    """Oracle LDL' (plain FP64, single thread) on a prefix of its rows, with the oracle's own
    ordering of this workload (stored by tests/golden/make_golden.py, checked against its digest).
    The per-row work of the whole factorization comes from the row counts alone; the pattern and
    the values are formed for the timed rows only."""
    import ctypes
    import numpy as np
    from oracle import _clib, kkt, ldl, symbolic
    perm = np.load(os.path.join(GOLD, f"{name}_perm.npy"))
    want = json.load(open(os.path.join(GOLD, "patterns.json")))[name]["perm"]
    if hashlib.sha256(np.ascontiguousarray(perm, dtype=np.int32).tobytes()).hexdigest() != want:
        raise RuntimeError("stored oracle ordering does not match its digest")
    Kp = kkt.kkt_pattern(prob)
    Up = symbolic.permute_upper(Kp, perm)
    parent = symbolic.etree(Up)
    N = len(perm)
    rowcnt, rowops = symbolic.row_work(Up, parent)
    cum = np.cumsum(rowops)
    nnz_cum = np.cumsum(rowcnt)
    total = float(cum[-1])
    reg = ldl.RegSettings()
    Kreg = kkt.kkt_upper(prob, -np.ones(prob.l), [], reg.static_reg, reg.static_reg)
    ip, ii, pos = symbolic.permute_map(Kp, perm)
    Ux = np.empty(len(ii)); Ux[pos] = Kreg.data
    sign = kkt.pivot_signs(prob)[perm].astype(np.int8)
    L = _clib.lib()

    def rows(k_end, k_mark=-1):
        Lp, Li = symbolic.l_pattern_rows(Up, parent, k_end)
        Lx = np.zeros(len(Li)); D = np.zeros(k_end)
        nreg = ctypes.c_int64(0)
        t_mark = ctypes.c_double(0.0)
        t0 = time.perf_counter()
        L.or_ldl_numeric_rows_marked(k_end, k_end, k_mark, ip, ii, Ux, parent, Lp, Li, sign, reg.dyn_eps,
                                     reg.dyn_delta, Lx, D, ctypes.byref(nreg), ctypes.byref(t_mark))
        return time.perf_counter() - t0, t_mark.value

    # The rows come in elimination order: the sparse part of the tree first, then the dense root front
    # (the trailing chain of columns with parent j + 1), whose rows cost far more per row but run faster
    # per multiply-add.  The sample is the whole sparse part and the first rows of the root; the root's
    # rate, timed inside the same run from its first row on, extrapolates the rest.
    k_root = N - 1
    while k_root > 0 and parent[k_root - 1] == k_root:
        k_root -= 1
    k_cal = int(min(N, np.searchsorted(cum, 2e8) + 1))
    rate = cum[k_cal - 1] / max(1e-6, rows(k_cal)[0])
    budget_ops = rate * seconds
    if cum[k_root - 1] < 0.8 * budget_ops and k_root < N:
        # the sparse part fits the budget: add root rows until the budget is spent (the calibration rate
        # of the sparse rows underestimates the root's), then time the last quarter of the sampled root
        # rows, whose longer rows run closest to the rate of the rest of the root
        k_end = int(min(N, np.searchsorted(cum, cum[k_root - 1] + 1.5 * budget_ops) + 1,
                        np.searchsorted(nnz_cum, 2e8) + 1))
        k_end = max(k_end, min(N, k_root + 64))
        # time per root row = a + b (multiply-adds of the row), fitted on the two halves of the sampled root
        # rows (the sparse part before them takes a negligible share of the first half), then applied to
        # the rest of the root
        k_mark = k_root + (k_end - k_root) // 2
        dt, t_mark = rows(k_end, k_mark)
        done = float(cum[k_end - 1])
        n1, o1, t1 = k_mark - k_root, float(cum[k_mark - 1] - cum[k_root - 1]), t_mark
        n2, o2, t2 = k_end - k_mark, float(cum[k_end - 1] - cum[k_mark - 1]), dt - t_mark
        det = n1 * o2 - n2 * o1
        a = (t1 * o2 - t2 * o1) / det if det != 0 else -1.0
        b = (n1 * t2 - n2 * t1) / det if det != 0 else -1.0
        if not (a >= 0.0 and b > 0.0):
            a, b = 0.0, t2 / max(1.0, o2)
        est_ms = 1e3 * (dt + a * (N - k_end) + b * (total - done))
        how = (f"rows 0..{k_end - 1} of {N} in {dt:.1f} s: the sparse part of the tree (rows 0..{k_root - 1}) and "
               f"the first {k_end - k_root} rows of the {N - k_root}-column root front, {100 * done / total:.3f}% of "
               f"{total:.3e} multiply-adds; the rest extrapolated with time per root row = {a * 1e6:.2f} us + "
               f"{b * 1e9:.3f} ns per multiply-add, fitted on the two halves of the sampled root rows")
    else:
        k_end = int(min(N, np.searchsorted(cum, budget_ops) + 1, np.searchsorted(nnz_cum, 2e8) + 1))
        dt, _ = rows(k_end)
        done = float(cum[k_end - 1])
        est_ms = 1e3 * dt * total / done
        how = (f"rows 0..{k_end - 1} of {N} = {100 * done / total:.3f}% of {total:.3e} multiply-adds in {dt:.1f} s, "
               f"scaled by the exact per-row operation count")
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(est_ms, 1), "unit": "ms per Newton step (factorization only, extrapolated)",
            "cores": 1, "kind": "oracle", "host_cpu": cpu,
            "sample": f"oracle up-looking LDL' of the {name} KKT (initial point), {how}; solves and cone work "
                      f"not included"}


def newton_steps(S, precision, k):
    """Exactly k Newton steps: consecutive solves from the initial point, the last one cut at the
    remaining count.  Returns the per-step event times, their precisions and the solve infos."""
    times, is32, infos = [], [], []
    while len(times) < k:
        S.set_settings(precision=precision, max_iter=k - len(times), profile=0)
        _, _, _, _, info = S.solve()
        infos.append(info)
        if info["nstep_ms"] == 0:
            break
        times += info["step_ms"]
        is32 += info["step_fp32"]
    S.set_settings(max_iter=100)
    return times, is32, infos


def rel_diff(a, b):
    import numpy as np
    return float(np.max(np.abs(a - b)) / max(1.0, float(np.max(np.abs(b)))))


def oracle_errors(qg, name, precisions):
    """Error of device solves against the oracle's stored solution of a workload (written by
    tests/golden/make_solutions.py, which calls only the oracle)."""
    import numpy as np
    from synth import problems
    ref = np.load(os.path.join(GOLD, f"{name}_oracle.npz"))
    prob = problems.workload(name)
    S = qg.Solver(prob)
    out = {}
    for tag, prec in precisions:
        S.set_settings(precision=prec)
        x, _, _, _, info = S.solve()
        xs = x.cpu().numpy()
        out[tag] = {"x_rel_err": rel_diff(xs, ref["x"]),
                    "obj_rel_err": abs(info["pobj"] - float(ref["pobj"])) / max(1.0, abs(float(ref["pobj"]))),
                    "status": info["status_name"], "iters": info["iters"]}
    S.close()
    return out


def run_config(qg, torch, name, warmup, steps, backward=False, ordering=0, prob=None):
    """Another configuration: FP32+IR and FP64 full solves (same warmup and count), median
    Newton-step ms, solve seconds, and the agreement of the two modes."""
    from synth import problems
    prob = prob if prob is not None else problems.workload(name)
    t0 = time.perf_counter()
    S = qg.Solver(prob, differentiable=1 if backward else 0, ordering=ordering)
    res = {"setup_s": round(time.perf_counter() - t0, 2), "N_K": prob.n + prob.m + prob.p,
           "ordering": "nested dissection" if ordering == qg.QG_ORDER_ND else "minimum degree",
           "analysis_s": None}
    xs = {}
    for tag, prec in (("fp32_ir", qg.QG_FP32_IR), ("fp64", qg.QG_FP64)):
        S.set_settings(precision=prec)
        for _ in range(warmup):
            S.solve()
        infos = []
        for _ in range(steps):
            x, _, _, _, info = S.solve()
            infos.append(info)
        last = infos[-1]
        res["analysis_s"] = round(last["ms_analyze"] / 1e3, 2)
        xs[tag] = (x.cpu().numpy(), last["pobj"])
        res[tag] = {"newton_step_ms": round(med([i["ms_step_median"] for i in infos]), 3),
                    "solve_s": round(med([i["ms_solve"] for i in infos]) / 1e3, 4), "iters": last["iters"],
                    "switch_iter": last["switch_iter"], "ir_steps": last["ir_steps"],
                    "factor_ms_total": round(last["ms_factor"], 2), "nfactor": last["nfactor"],
                    "factor_flops": last["factor_flops"], "nnz_L": last["nnz_L"],
                    "ntrisolve": list(last["ntrisolve"]), "nresidual": last["nresidual"],
                    "trisolve_ir_ms_total": round(last["ms_trisolve"], 2),
                    "cone_ms_total": round(last["ms_cone"], 2), "status": last["status_name"],
                    "pres": last["pres"], "dres": last["dres"], "gap": last["gap"]}
        log(f"[bench] {name} {tag}: step {res[tag]['newton_step_ms']} ms solve {res[tag]['solve_s']} s "
            f"iters {last['iters']}")
    res["fp32_ir_vs_fp64"] = {"x_rel_diff": rel_diff(xs["fp32_ir"][0], xs["fp64"][0]),
                              "obj_rel_diff": abs(xs["fp32_ir"][1] - xs["fp64"][1]) / max(1.0, abs(xs["fp64"][1]))}
    res["speedup_fp32ir_vs_fp64_step"] = round(res["fp64"]["newton_step_ms"] / max(1e-9, res["fp32_ir"]["newton_step_ms"]), 3)
    if backward:
        import numpy as np
        g = torch.tensor(np.random.default_rng(5).standard_normal(prob.n), device="cuda")
        S.set_settings(precision=qg.QG_FP64)
        S.solve()
        S.backward(g)
        torch.cuda.synchronize()
        t = time.perf_counter()
        S.backward(g)
        torch.cuda.synchronize()
        res["backward_ms"] = round(1e3 * (time.perf_counter() - t), 2)
    S.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the other configurations")
    ap.add_argument("--workload", default=WORKLOAD, help=argparse.SUPPRESS)
    ap.add_argument("--ordering", default="md", choices=("md", "nd"), help=argparse.SUPPRESS)
    ap.add_argument("--cone-lanes", type=int, default=1, choices=(0, 1), help=argparse.SUPPRESS)
    ap.add_argument("--fp32-steps-only", action="store_true",
                    help="setup and the timed FP32+IR Newton steps only, for runs under a profiler; prints no JSON line")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 256 MiB three times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); multi-GPU is not part of this build",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: 3 copies of {src.numel() * 4} bytes (read {src.numel() * 4}, write {src.numel() * 4} each)")
        return
    import numpy as np
    import paper_2603_29197_amd as qg
    from synth import problems

    name = args.workload
    prob = problems.workload(name)
    log(f"[bench] setup {name}")
    t0 = time.perf_counter()
    S = qg.Solver(prob, precision=qg.QG_FP32_IR, cone_lanes=args.cone_lanes,
                  ordering=qg.QG_ORDER_ND if args.ordering == "nd" else qg.QG_ORDER_MD)
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.1f} s")

    def timed(precision, tag):
        w_times, _, _ = newton_steps(S, precision, args.warmup)
        log(f"[bench] {tag} warmup: {len(w_times)} steps")
        torch.cuda.synchronize()
        t = time.perf_counter()
        times, is32, infos = newton_steps(S, precision, args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        log(f"[bench] {tag}: {len(times)} steps in {wall:.2f} s over {len(infos)} solve(s), median "
            f"{med(times):.2f} ms")
        return times, is32, infos, wall

    t32, f32, i32, wall32 = timed(qg.QG_FP32_IR, "fp32+ir")
    if args.fp32_steps_only:
        S.close()
        return
    t64, _, i64, wall64 = timed(qg.QG_FP64, "fp64")
    step32, step64 = med(t32), med(t64)

    # one full solve to the 1e-8 stopping test in each mode
    full = {}
    for tag, prec in (("fp32_ir", qg.QG_FP32_IR), ("fp64", qg.QG_FP64)):
        S.set_settings(precision=prec, max_iter=100)
        x, _, _, _, info = S.solve()
        full[tag] = (x.cpu().numpy(), info)
        log(f"[bench] full {tag}: {info['status_name']} iters {info['iters']} switch {info['switch_iter']} "
            f"solve {info['ms_solve'] / 1e3:.2f} s")

    roof = None
    if not args.no_profile:
        # trailing-update launches of a short solve (initial factorization + 2 Newton steps), each
        # bracketed by HIP events on the stream it runs on
        S.set_settings(precision=qg.QG_FP32_IR, profile=1, max_iter=2)
        _, _, _, _, p32 = S.solve()
        S.set_settings(precision=qg.QG_FP64, profile=1, max_iter=1)
        _, _, _, _, p64 = S.solve()
        S.set_settings(profile=0, max_iter=100)
        def kern(info, slot):
            l, ms, fl = info["kern_launches"][slot], info["kern_ms"][slot], info["kern_flops"][slot]
            return (int(l), ms, fl, fl / (ms * 1e-3) / 1e12 if ms > 0 else 0.0)
        # slot 3 = FP32 on 128 x 128 tiles (trail_update_big), the kernel with the most flops;
        # slot 1 = FP32 on 64 x 64 tiles (trail_update<float>: the rank-64 updates inside a super-panel);
        # slot 0 = FP64 (trail_update<double>, 64 x 64 tiles: the FP64 mode has no 128 x 128 kernel)
        lb, msb, flb, ab = kern(p32, 3)
        ls, mss, fls, as_ = kern(p32, 1)
        l64, ms64, fl64, a64 = kern(p64, 0)
        if lb > 0 and msb > 0:
            roof = {"kernel": "trail_update_big (FP32, MFMA f32 16x16x4, 128x128 tiles: the rank-256 trailing "
                              "updates of large fronts)",
                    "bound": "mfma", "achieved": round(ab, 2), "peak": PEAK_TFLOPS["fp32"],
                    "unit": "TFLOP/s", "frac": round(ab / PEAK_TFLOPS["fp32"], 4),
                    "traffic": TRAFFIC_BYTES_PER_LAUNCH["fp32"],
                    "launches": lb, "avg_launch_us": round(1e3 * msb / lb, 2), "flops_per_launch_avg": flb / lb,
                    "measured_over": "initial factorization + 2 Newton steps, FP32+IR, HIP events per launch",
                    "small_tile_kernel": {"kernel": "trail_update<float>", "launches": ls,
                                          "achieved": round(as_, 2),
                                          "avg_launch_us": round(1e3 * mss / max(1, ls), 2)},
                    # the whole FP32 factorizations of the profiled solve (initial + 2 steps): the factor
                    # flops over their wall time between events on the caller's stream (every stream joined)
                    "whole_factorizations_fp32": {
                        "achieved": round(p32["factor_flops"] * p32["nfactor"] / (p32["ms_factor"] * 1e-3) / 1e12, 2),
                        "frac": round(p32["factor_flops"] * p32["nfactor"] / (p32["ms_factor"] * 1e-3) / 1e12
                                      / PEAK_TFLOPS["fp32"], 4),
                        "ms_per_factorization": round(p32["ms_factor"] / max(1, p32["nfactor"]), 2)},
                    "all_trailing_updates_fp32": {"achieved": round((flb + fls) / ((msb + mss) * 1e-3) / 1e12, 2),
                                                  "frac": round((flb + fls) / ((msb + mss) * 1e-3) / 1e12
                                                                / PEAK_TFLOPS["fp32"], 4)}}
            if l64 > 0 and ms64 > 0:
                roof["fp64_kernel"] = {"kernel": "trail_update<double> (all FP64 trailing updates)",
                                       "achieved": round(a64, 2), "peak": PEAK_TFLOPS["fp64"],
                                       "frac": round(a64 / PEAK_TFLOPS["fp64"], 4),
                                       "traffic": TRAFFIC_BYTES_PER_LAUNCH["fp64"],
                                       "launches": l64, "avg_launch_us": round(1e3 * ms64 / l64, 2)}
    # the solve phase of the full FP32+IR solve against HBM: per triangular solve 2 nnz(L) s_L + 4 N 8
    # bytes (s_L = 4 with an FP32 factor, 8 with FP64), per residual nnz(K upper) (8 + 4) + 3 N 8 bytes
    last = full["fp32_ir"][1]
    N = prob.n + prob.p + prob.m
    nnzK = len(S.step_get_kkt())
    tri64, tri32 = last["ntrisolve"]
    b_solve = tri32 * (2 * last["nnz_L"] * 4 + 4 * N * 8) + tri64 * (2 * last["nnz_L"] * 8 + 4 * N * 8) \
        + last["nresidual"] * (nnzK * 12 + 3 * N * 8)
    gbs = b_solve / (last["ms_trisolve"] * 1e-3) / 1e9 if last["ms_trisolve"] > 0 else 0.0
    solve_roof = {"rows": "triangular solves + refinement residuals", "bound": "hbm", "achieved": round(gbs, 1),
                  "peak": PEAK_GBS, "unit": "GB/s", "frac": round(gbs / PEAK_GBS, 4), "bytes_algorithmic": b_solve,
                  "ms": round(last["ms_trisolve"], 2), "triangular_solves": [tri64, tri32],
                  "residuals": last["nresidual"]}
    # cone kernels of the full solve: ~200 B per cone row per iteration (scaling 32, right-hand sides 48,
    # ds 32, two line searches 64, the update 24 (n + 2m + p) / m) plus 8 B per (3,3)-block entry
    m = prob.m
    cone_bytes = last["iters"] * (200.0 * m + 24.0 * (prob.n + 2 * m + prob.p) + 8.0 * (prob.l + sum(q * (q + 1) // 2 for q in prob.q)))
    cgbs = cone_bytes / (last["ms_cone"] * 1e-3) / 1e9 if last["ms_cone"] > 0 else 0.0
    cone_roof = {"rows": "NT scaling, (3,3) block, right-hand sides, ds, line searches, update", "bound": "hbm",
                 "achieved": round(cgbs, 1), "peak": PEAK_GBS, "unit": "GB/s", "frac": round(cgbs / PEAK_GBS, 4),
                 "bytes_algorithmic": cone_bytes, "ms": round(last["ms_cone"], 2)}

    # error of the FP32+IR solution against FP64 at this size, and against the oracle on the same
    # generator at the size the oracle solves (F 10000 x 4000)
    x32, inf32 = full["fp32_ir"]
    x64, inf64 = full["fp64"]
    errs = {"fp32_ir_vs_fp64_full_size": {"x_rel_diff": rel_diff(x32, x64),
                                           "obj_rel_diff": abs(inf32["pobj"] - inf64["pobj"]) / max(1.0, abs(inf64["pobj"]))}}
    try:
        errs["vs_oracle_huber_s"] = oracle_errors(qg, "huber_s", (("fp32_ir", qg.QG_FP32_IR), ("fp64", qg.QG_FP64)))
    except FileNotFoundError:
        errs["vs_oracle_huber_s"] = None

    configs = None
    if not args.no_extra and name == WORKLOAD:
        configs = {}
        msoc = problems.workload("many_soc")
        # many_soc runs with nested dissection (its windowed cones make a long band, whose
        # minimum-degree elimination tree is 918 fronts deep) and, for comparison, minimum degree
        for key, cname, w, k, bw, ordr, pr in (("small_qp", "small_qp", 1, 3, False, qg.QG_ORDER_MD, None),
                                               ("lasso", "lasso", 1, 3, False, qg.QG_ORDER_MD, None),
                                               ("many_soc", "many_soc", 1, 2, False, qg.QG_ORDER_ND, msoc),
                                               ("many_soc_md", "many_soc", 1, 2, False, qg.QG_ORDER_MD, msoc),
                                               ("lasso_diff", "lasso_diff", 0, 1, True, qg.QG_ORDER_MD, None)):
            log(f"[bench] config {key}")
            configs[key] = run_config(qg, torch, cname, w, k, backward=bw, ordering=ordr, prob=pr)
        for cname in ("small_qp", "lasso"):
            try:
                configs[cname]["vs_oracle"] = oracle_errors(qg, cname, (("fp32_ir", qg.QG_FP32_IR),
                                                                        ("fp64", qg.QG_FP64)))
            except FileNotFoundError:
                pass

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(prob, name, args.cpu_seconds)
        log(f"[bench] cpu baseline {cpu['value']} ms/step")
    out = {
        "metric": METRIC, "value": round(step32, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall32 / max(1, args.steps), 2),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT if name == WORKLOAD else name,
                   "mode": "FP32 factors + FP64 refinement, FP64 after gap < 1e-6",
                   "step": "one Newton step; K steps timed over consecutive solves from the initial point; "
                           "value = median Newton-step ms"},
        "fp32_ir": {"newton_step_ms": round(step32, 3), "step_ms_p90": round(float(np.percentile(t32, 90)), 3),
                    "steps_with_fp32_factor": int(sum(f32)), "timed_solves": len(i32),
                    "solve_s": round(inf32["ms_solve"] / 1e3, 3), "iters": inf32["iters"],
                    "switch_iter": inf32["switch_iter"], "ir_steps": inf32["ir_steps"],
                    "step_ms_fp32_iters": round(inf32["ms_step_median_fp32"], 3), "status": inf32["status_name"],
                    "factor_ms_total": round(inf32["ms_factor"], 2), "nfactor": inf32["nfactor"],
                    "pres": inf32["pres"], "dres": inf32["dres"],
                    "gap": inf32["gap"], "pobj": inf32["pobj"]},
        "fp64": {"newton_step_ms": round(step64, 3), "step_ms_p90": round(float(np.percentile(t64, 90)), 3),
                 "ms_per_step": round(1e3 * wall64 / max(1, args.steps), 2), "timed_solves": len(i64),
                 "solve_s": round(inf64["ms_solve"] / 1e3, 3), "iters": inf64["iters"], "status": inf64["status_name"],
                 "factor_ms_total": round(inf64["ms_factor"], 2), "nfactor": inf64["nfactor"],
                 "pres": inf64["pres"], "dres": inf64["dres"],
                 "gap": inf64["gap"], "pobj": inf64["pobj"]},
        "speedup_fp32ir_vs_fp64_step": round(step64 / step32, 3) if step32 > 0 else None,
        "speedup_fp32ir_vs_fp64_solve": round(inf64["ms_solve"] / inf32["ms_solve"], 3) if inf32["ms_solve"] > 0 else None,
        "errors": errs,
        "setup_s": round(setup_s, 2), "analysis_s": round(inf32["ms_analyze"] / 1e3, 2), "nnz_L": inf32["nnz_L"], "factor_flops": inf32["factor_flops"],
        "step_split_ms": {"factor": round(inf32["ms_factor"], 2), "trisolve_ir": round(inf32["ms_trisolve"], 2),
                          "cone": round(inf32["ms_cone"], 2),
                          "other": round(inf32["ms_solve"] - inf32["ms_factor"] - inf32["ms_trisolve"]
                                         - inf32["ms_cone"], 2),
                          "per": "whole FP32+IR solve (device event times; other = wall time minus the rest)"},
        "roofline": roof, "solve_roofline": solve_roof, "cone_roofline": cone_roof, "cpu_baseline": cpu,
        "configs": configs,
    }
    print(json.dumps(out), flush=True)
    S.close()


if __name__ == "__main__":
    main()
