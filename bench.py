"""Benchmark of the Newton step on one MI355X.

Workload: the lasso QP (variables x, y, t; y = F x - g; -t <= x <= t;
objective 1/2 |y|^2 + lam 1't) with F 20000 x 10000 at density 0.005, seeded
and synthetic (KKT dimension 80000, about 1.1e6 upper KKT entries).

One timed step = one full interior-point solve (initial point through the
1e-8 stopping test) in FP32+IR mode, with the problem resident on the
device; ``value`` is the median Newton-step time (residuals, scaling,
factorization, both refined solves, cone kernels, update) over the
iterations of the timed solves.  The plain-FP64 mode is timed the same way
afterwards and reported beside it.  The roofline entry covers the dominant
kernel, the MFMA trailing update of the large fronts, timed per launch with
HIP events in a separate profiled solve.  The CPU baseline is the FP64
oracle's up-looking factorization of the same KKT matrix, run on a bounded
prefix of its rows and scaled by exact per-row operation counts.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Newton-step ms (factor+solve) & solve s to 1e-8 gap: FP32+IR vs FP64, 1 MI355X"
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
# HBM bytes per launch of trail_update on this workload, from rocprofv3 FETCH_SIZE and WRITE_SIZE
# runs (profiles/trail_update_lasso.md), each scaled by what the counter reads for a plain device
# copy of known size (FETCH_SIZE x 1.9998, WRITE_SIZE x 1.0). Counters describe one build of the
# kernel: reset to None when trail_update changes until they are taken again.
TRAFFIC_BYTES_PER_LAUNCH = {"fp32": 4.851e7, "fp64": 1.010e8}
WORKLOAD = "lasso F 20000x10000 density 0.005 (n=40000, p=20000, m=20000, N_K=80000)"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(prob, seconds: float):
    """Oracle LDL' (plain FP64, single thread) on a prefix of its rows."""
    import hashlib
    import numpy as np
    from oracle import _clib, kkt, ldl, symbolic
    gold = os.path.join(ROOT, "tests", "golden")
    perm = np.load(os.path.join(gold, "lasso_perm.npy"))
    want = json.load(open(os.path.join(gold, "patterns.json")))["lasso"]["perm"]
    if hashlib.sha256(np.ascontiguousarray(perm, dtype=np.int32).tobytes()).hexdigest() != want:
        raise RuntimeError("stored oracle ordering does not match its digest")
    Kp = kkt.kkt_pattern(prob)
    Up = symbolic.permute_upper(Kp, perm)
    parent = symbolic.etree(Up)
    Lp, Li, colcount = symbolic.l_pattern(Up, parent)
    N = len(perm)
    # inner-loop operations of the up-looking factorization per row: the t-th
    # entry (t = 0, 1, ..) of column j costs t multiply-adds when its row is done
    tpos = np.arange(len(Li), dtype=np.int64) - np.repeat(Lp[:-1], np.diff(Lp))
    ops = np.bincount(Li, weights=tpos.astype(np.float64), minlength=N) + np.bincount(Li, minlength=N) + 1.0
    cum = np.cumsum(ops)
    total = float(cum[-1])
    reg = ldl.RegSettings()
    Kreg = kkt.kkt_upper(prob, -np.ones(prob.l), [], reg.static_reg, reg.static_reg)
    ip, ii, pos = symbolic.permute_map(Kp, perm)
    Ux = np.empty(len(ii)); Ux[pos] = Kreg.data
    sign = kkt.pivot_signs(prob)[perm].astype(np.int8)
    Lx = np.zeros(len(Li)); D = np.zeros(N)
    import ctypes
    nreg = ctypes.c_int64(0)
    L = _clib.lib()
    # calibrate on a small prefix, then size the sample to ~`seconds`
    k_cal = int(np.searchsorted(cum, 2e8))
    t0 = time.perf_counter()
    L.or_ldl_numeric_rows(N, k_cal, ip, ii, Ux, parent, Lp, Li, sign, reg.dyn_eps, reg.dyn_delta, Lx, D,
                          ctypes.byref(nreg))
    rate = cum[k_cal - 1] / max(1e-6, time.perf_counter() - t0)
    k_end = int(min(N, np.searchsorted(cum, rate * seconds)))
    t0 = time.perf_counter()
    L.or_ldl_numeric_rows(N, k_end, ip, ii, Ux, parent, Lp, Li, sign, reg.dyn_eps, reg.dyn_delta, Lx, D,
                          ctypes.byref(nreg))
    dt = time.perf_counter() - t0
    done = float(cum[k_end - 1])
    est_ms = 1e3 * dt * total / done
    return {"value": round(est_ms, 1), "unit": "ms per Newton step (factorization only, extrapolated)",
            "cores": 1, "kind": "oracle",
            "sample": f"oracle up-looking LDL' of the lasso KKT (initial point), rows 0..{k_end - 1} of {N} "
                      f"= {100 * done / total:.2f}% of {total:.3e} multiply-adds in {dt:.1f} s, scaled by the "
                      f"exact per-row operation count; solves and cone work (<1% of the step) not included"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-profile", action="store_true")
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
    import paper_2603_29197_amd as qg
    from synth import problems

    prob = problems.workload("lasso")
    log(f"[bench] setup {WORKLOAD}")
    t0 = time.perf_counter()
    S = qg.Solver(prob, precision=qg.QG_FP32_IR)
    setup_s = time.perf_counter() - t0
    log(f"[bench] setup {setup_s:.1f} s")

    def run(precision, steps, warmup, tag):
        S.set_settings(precision=precision, profile=0)
        for w in range(warmup):
            _, _, _, _, info = S.solve()
            log(f"[bench] {tag} warmup {w}: {info['status_name']} iters {info['iters']} "
                f"{info['ms_solve']:.1f} ms")
        infos = []
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k in range(steps):
            _, _, _, _, info = S.solve()
            infos.append(info)
            log(f"[bench] {tag} step {k}: {info['status_name']} iters {info['iters']} switch "
                f"{info['switch_iter']} solve {info['ms_solve']:.1f} ms step {info['ms_step_median']:.2f} ms")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t
        return infos, wall

    infos32, wall32 = run(qg.QG_FP32_IR, args.steps, args.warmup, "fp32+ir")
    infos64, wall64 = run(qg.QG_FP64, max(1, args.steps), 0, "fp64")
    med = lambda xs: float(statistics.median(xs))
    step32 = med([i["ms_step_median"] for i in infos32])
    step64 = med([i["ms_step_median"] for i in infos64])

    roof = None
    if not args.no_profile:
        S.set_settings(precision=qg.QG_FP32_IR, profile=1)
        _, _, _, _, pinfo = S.solve()
        S.set_settings(profile=0)
        launches, ms, flops = pinfo["kern_launches"][1], pinfo["kern_ms"][1], pinfo["kern_flops"][1]
        if launches > 0 and ms > 0:
            achieved = flops / (ms * 1e-3) / 1e12
            roof = {"kernel": "trail_update<float> (MFMA f32 16x16x4 trailing update of large fronts)",
                    "bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK_TFLOPS["fp32"],
                    "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["fp32"], 4),
                    "traffic": TRAFFIC_BYTES_PER_LAUNCH["fp32"],
                    "launches": int(launches), "avg_launch_us": round(1e3 * ms / launches, 2),
                    "flops_per_launch_avg": flops / launches}
            l64, ms64, fl64 = pinfo["kern_launches"][0], pinfo["kern_ms"][0], pinfo["kern_flops"][0]
            if l64 > 0 and ms64 > 0:
                a64 = fl64 / (ms64 * 1e-3) / 1e12
                roof["fp64_kernel"] = {"kernel": "trail_update<double>", "achieved": round(a64, 2),
                                       "peak": PEAK_TFLOPS["fp64"], "frac": round(a64 / PEAK_TFLOPS["fp64"], 4),
                                       "traffic": TRAFFIC_BYTES_PER_LAUNCH["fp64"],
                                       "launches": int(l64), "avg_launch_us": round(1e3 * ms64 / l64, 2)}
    # the solve phase (triangular solves and refinement residuals of the timed FP32+IR solve) against
    # HBM: per triangular solve 2 nnz(L) s_L + 4 N 8 bytes (s_L = 4 with an FP32 factor, 8 with FP64),
    # per residual nnz(K upper) (8 + 4) + 3 N 8 bytes
    last = infos32[-1]
    N = prob.n + prob.p + prob.m
    nnzK = len(S.step_get_kkt())
    tri64, tri32 = last["ntrisolve"]
    b_solve = tri32 * (2 * last["nnz_L"] * 4 + 4 * N * 8) + tri64 * (2 * last["nnz_L"] * 8 + 4 * N * 8) \
        + last["nresidual"] * (nnzK * 12 + 3 * N * 8)
    gbs = b_solve / (last["ms_trisolve"] * 1e-3) / 1e9 if last["ms_trisolve"] > 0 else 0.0
    solve_roof = {"rows": "triangular solves + refinement residuals", "bound": "hbm", "achieved": round(gbs, 1),
                  "peak": 8000.0, "unit": "GB/s", "frac": round(gbs / 8000.0, 4), "bytes_algorithmic": b_solve,
                  "ms": round(last["ms_trisolve"], 2), "triangular_solves": [tri64, tri32],
                  "residuals": last["nresidual"],
                  "note": "the FP32 factor (~0.2 GB) largely fits the 256 MB last-level cache: effective rate"}
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        cpu = cpu_baseline(prob, args.cpu_seconds)
        log(f"[bench] cpu baseline {cpu['value']} ms/step")
    last32, last64 = infos32[-1], infos64[-1]
    out = {
        "metric": METRIC, "value": round(step32, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * wall32 / max(1, args.steps), 2),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "mode": "FP32 factors + FP64 refinement, FP64 after gap < 1e-6",
                   "step": "one full solve to the 1e-8 stopping test; value = median Newton-step ms"},
        "fp32_ir": {"newton_step_ms": round(step32, 3), "solve_s": round(last32["ms_solve"] / 1e3, 4),
                    "iters": last32["iters"], "switch_iter": last32["switch_iter"],
                    "ir_steps": last32["ir_steps"], "step_ms_fp32_iters": round(last32["ms_step_median_fp32"], 3),
                    "factor_ms_total": round(last32["ms_factor"], 2), "pres": last32["pres"],
                    "dres": last32["dres"], "gap": last32["gap"], "pobj": last32["pobj"]},
        "fp64": {"newton_step_ms": round(step64, 3), "solve_s": round(last64["ms_solve"] / 1e3, 4),
                 "iters": last64["iters"], "factor_ms_total": round(last64["ms_factor"], 2),
                 "pres": last64["pres"], "dres": last64["dres"], "gap": last64["gap"], "pobj": last64["pobj"]},
        "speedup_fp32ir_vs_fp64_step": round(step64 / step32, 3) if step32 > 0 else None,
        "setup_s": round(setup_s, 2), "nnz_L": last32["nnz_L"], "factor_flops": last32["factor_flops"],
        "step_split_ms": {"factor": round(last["ms_factor"], 2), "trisolve_ir": round(last["ms_trisolve"], 2),
                          "cone": round(last["ms_cone"], 2),
                          "other": round(last["ms_solve"] - last["ms_factor"] - last["ms_trisolve"]
                                         - last["ms_cone"], 2),
                          "per": "whole FP32+IR solve (device event times; other = wall time minus the rest)"},
        "step_ms_p90": {"fp32_ir": round(last["ms_step_p90"], 3), "fp64": round(infos64[-1]["ms_step_p90"], 3)},
        "roofline": roof, "solve_roofline": solve_roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    S.close()


if __name__ == "__main__":
    main()
