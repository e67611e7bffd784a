// Primal-dual interior-point loop for problem (1), all numeric work on the
// device (paper Sec. 2.3); the host keeps only the scalars it needs to
// decide (stopping test, precision switch, refinement test).
//
// Method (our reading of the cone-QP method the paper's solver implements:
// Mehrotra predictor-corrector with Nesterov-Todd scaling):
//   init: factor K with W = I, solve K [x; y; z] = [-c; b; h], s = h - Gx,
//         shift s and z into the interior;
//   iterate: residuals and stopping test; NT scaling and the (3,3) block;
//   one factorization; affine solve K d = [-r_x; -r_y; -r_z + s],
//   ds_a = -s - W'W dz_a; alpha_a, sigma = (1 - alpha_a)^3; corrector
//   t = W'(lam \ (-lam o lam - (W^-T ds_a) o (W dz_a) + sigma mu e)),
//   K d = [-r_x; -r_y; -r_z - t], ds = t - W'W dz; alpha =
//   min(1, 0.99 max step); update.
// Precision (FP32_IR): FP32 factors with FP64 refinement while the scaled
// gap |s'z| / max(1, min(|pobj|, |dobj|)) >= switch_gap; FP64 factors from
// then on, and for the rest of the iteration whenever refinement with an
// FP32 factor fails its test.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "vec.hpp"

namespace qg {

namespace {

struct Events {
    // 0-7: phases; 8-13: the Newton steps' start, cone-phase start and end, two sets used in turn
    // (a step's times are read after the next step's first wait); 14-15: the scaling kernel
    hipEvent_t e[16] = {};
    bool ok = false;
    void create() {
        ok = true;
        for (auto &x : e) if (hipEventCreate(&x) != hipSuccess) ok = false;
    }
    void destroy() {
        for (auto &x : e) if (x) (void)hipEventDestroy(x);
    }
};

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

double median(std::vector<double> v) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const size_t n = v.size();
    return n % 2 ? v[n / 2] : 0.5 * (v[n / 2 - 1] + v[n / 2]);
}

// Percentile q in [0, 1] by linear interpolation between order statistics.
double percentile(std::vector<double> v, double q) {
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)pos, hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

struct Scalars {
    double pres, dres, gap, pobj, dobj, sz;
    bool ok;
};

Scalars stop_test(qg_handle *h, const double *sc, double ea, double er) {
    Scalars r;
    r.pres = std::max(sc[S_RY], sc[S_RZ]);
    r.dres = sc[S_RX];
    r.sz = sc[S_SZ];
    // equilibrated data: the inner products carry the objective scaling k (the max-norm terms were
    // taken back to the caller's units by the residual kernel)
    const double ik = h->ruiz > 0 ? 1.0 / h->ruiz_k : 1.0;
    r.gap = std::fabs(sc[S_SZ]) * ik;
    r.pobj = (0.5 * sc[S_XPX] + sc[S_CX]) * ik;
    r.dobj = (-0.5 * sc[S_XPX] - sc[S_BY] - sc[S_HZ]) * ik;
    const double pscale = std::max({sc[S_AX], sc[S_B], sc[S_GX], sc[S_H], sc[S_S]});
    const double dscale = std::max({sc[S_PX], sc[S_ATY], sc[S_GTZ], sc[S_C]});
    const double gscale = std::max(1.0, std::min(std::fabs(r.pobj), std::fabs(r.dobj)));
    r.ok = r.pres <= ea + er * pscale && r.dres <= ea + er * dscale && r.gap <= ea + er * gscale;
    return r;
}

}  // namespace

// One refined solve; in FP32 mode a failed refinement test is reported.
// Counts of the solve phase's work (for its roofline): triangular solves by
// factor precision ([0] FP64, [1] FP32) and refinement residuals K x.
struct SolveWork {
    int64_t tri[2] = {0, 0};
    int64_t residuals = 0;
};

static int solve_with(qg_handle *h, const double *rhs, double *x, int prec, int *ir_total, bool *failed,
                      Events &ev, double *ms, SolveWork &work) {
    int steps = 0;
    bool ok = true;
    const int ir_max = prec == QG_FP32_IR ? h->st.ir_max32 : h->st.ir_max;
    (void)hipEventRecord(ev.e[4], h->stream);
    int rc = refined_solve(h, rhs, x, prec, ir_max, &steps, prec == QG_FP32_IR ? &ok : nullptr);
    if (rc) return rc;
    (void)hipEventRecord(ev.e[5], h->stream);
    // the refinement test has drained the stream up to here: the event completes at once (polled)
    while (hipEventQuery(ev.e[5]) == hipErrorNotReady) {
    }
    work.tri[prec == QG_FP32_IR ? 1 : 0] += 1 + steps;     // the solve and one per correction
    work.residuals += steps + 1;                           // one per correction and the last test
    *ir_total += steps;
    *failed = !ok;
    *ms += elapsed(ev.e[4], ev.e[5]);
    return QG_OK;
}

int ipm_solve(qg_handle *h, double *xo, double *so, double *yo, double *zo, qg_info *info) {
    const auto t_start = std::chrono::steady_clock::now();
    const qg_settings &st = h->st;
    Device &d = h->d;
    const int32_t n = h->n, p = h->p, m = h->m, N = h->N;
    const int nu = h->pp.l + h->pp.nsoc;
    Events ev;
    ev.create();
    int rc = QG_OK;
    int ir_total = 0, nreg_total = 0, nfactor = 0, nsolve = 0, switch_iter = -1;
    if (st.precision == QG_FP32_IR && h->plan.large_flops < st.fp32_min_flops) switch_iter = 0;
    double ms_factor = 0, ms_solve = 0, ms_cone = 0;
    SolveWork work;
    std::vector<double> step_ms, step32, step64;
    std::vector<int32_t> step_is32;
    // FP32 factors only where the matrix-core work of the factorization is large enough to pay for
    // the extra refinement corrections (settings.fp32_min_flops)
    bool fp64_only = st.precision != QG_FP32_IR || h->plan.large_flops < st.fp32_min_flops;
    // residual scalars of each problem of a batch (one problem: kb = 1) and of the whole stack
    const int32_t kb = h->ncopy;
    std::vector<double> scal_all((size_t)kb * NSCAL), mu_host(2 * (size_t)kb, 1.0);
    double scal[NSCAL];
    auto combine = [&]() {
        for (int q = 0; q < NSCAL; ++q) {
            double v = scal_all[(size_t)q];
            for (int32_t i = 1; i < kb; ++i) {
                const double w = scal_all[(size_t)i * NSCAL + q];
                v = ((SCAL_MAXMASK >> q) & 1u) ? nan_max(v, w) : v + w;
            }
            scal[q] = v;
        }
    };
    // every problem of the batch meets the test (its own residuals, scales and gap); a problem that
    // meets it stops moving (its gate, mu_host[kb + i], drops to 0), so each problem ends at the
    // first iterate that passes its own test, as when it is solved alone
    auto all_pass = [&](double ea, double er) {
        bool all = true;
        for (int32_t i = 0; i < kb; ++i) {
            if (mu_host[(size_t)kb + i] == 0.0) continue;
            if (stop_test(h, scal_all.data() + (size_t)i * NSCAL, ea, er).ok) mu_host[(size_t)kb + i] = 0.0;
            else all = false;
        }
        return all;
    };
    Scalars sr{};
    int status = QG_MAX_ITER, it = 0;
    h->solved = false;
    h->final_factor = false;
    auto fail = [&](int code) { ev.destroy(); return code; };

    // ---- initial point: W = I ----
    int prec = fp64_only ? QG_FP64 : QG_FP32_IR;
    if ((rc = launch_identity_vec(h, d.t.p))) return fail(rc);
    if ((rc = launch_scaling(h, d.t.p, d.t.p, nullptr, 0))) return fail(rc);
    (void)hipEventRecord(ev.e[2], h->stream);
    if ((rc = launch_factor(h, prec))) return fail(rc);
    (void)hipEventRecord(ev.e[3], h->stream);
    ++nfactor;
    {
        // rhs = [-c; b; h]
        if ((rc = launch_scale_copy(h, n, -1.0, d.c.p, d.rhs.p))) return fail(rc);
        QG_HIP(h, hipMemcpyAsync(d.rhs.p + n, d.b.p, sizeof(double) * p, hipMemcpyDeviceToDevice, h->stream));
        QG_HIP(h, hipMemcpyAsync(d.rhs.p + n + p, d.h.p, sizeof(double) * m, hipMemcpyDeviceToDevice, h->stream));
        bool failed = false;
        if ((rc = solve_with(h, d.rhs.p, d.sol.p, prec, &ir_total, &failed, ev, &ms_solve, work))) return fail(rc);
        ms_factor += elapsed(ev.e[2], ev.e[3]);
        if (failed && prec == QG_FP32_IR) {
            prec = QG_FP64;
            if ((rc = launch_factor(h, prec))) return fail(rc);
            ++nfactor;
            if ((rc = solve_with(h, d.rhs.p, d.sol.p, prec, &ir_total, &failed, ev, &ms_solve, work))) return fail(rc);
        }
        ++nsolve;
        QG_HIP(h, hipMemcpyAsync(d.x.p, d.sol.p, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
        QG_HIP(h, hipMemcpyAsync(d.y.p, d.sol.p + n, sizeof(double) * p, hipMemcpyDeviceToDevice, h->stream));
        QG_HIP(h, hipMemcpyAsync(d.z.p, d.sol.p + n + p, sizeof(double) * m, hipMemcpyDeviceToDevice, h->stream));
        // s = h - G x: residual with s = 0 gives rz = Gx - h
        if ((rc = launch_fill(h, m, 0.0, d.s.p))) return fail(rc);
        if ((rc = launch_residual(h, d.x.p, d.y.p, d.z.p, d.s.p, scal_all.data()))) return fail(rc);
        if ((rc = launch_scale_copy(h, m, -1.0, d.rz.p, d.s.p))) return fail(rc);
        if ((rc = launch_shift_interior(h, d.s.p))) return fail(rc);
        if ((rc = launch_shift_interior(h, d.z.p))) return fail(rc);
    }
    double *dvec = d.sol.p;               // Newton direction (N)
    const double *dz_of = dvec + n + p;
    int pending = -1, pending_is32 = 0;   // event set of the last Newton step, its times not read yet
    auto consume_step = [&]() {
        if (pending < 0) return;
        hipEvent_t *T = ev.e + 8 + 3 * pending;
        ms_cone += elapsed(T[1], T[2]);
        const double sm = elapsed(T[0], T[2]);
        step_ms.push_back(sm);
        step_is32.push_back(pending_is32);
        (pending_is32 ? step32 : step64).push_back(sm);
        pending = -1;
    };
    while (true) {
        const int par = it & 1;
        hipEvent_t *T = ev.e + 8 + 3 * par;
        (void)hipEventRecord(T[0], h->stream);
        if ((rc = launch_residual(h, d.x.p, d.y.p, d.z.p, d.s.p, scal_all.data()))) return fail(rc);
        consume_step();                    // the wait in launch_residual has passed the last step's end
        combine();
        sr = stop_test(h, scal, st.eps_abs, st.eps_rel);
        if (kb > 1) sr.ok = all_pass(st.eps_abs, st.eps_rel);
        if (st.verbose)
            fprintf(stderr, "it %3d pobj %+.8e dobj %+.8e pres %.2e dres %.2e gap %.2e %s\n", it, sr.pobj,
                    sr.dobj, sr.pres, sr.dres, sr.gap, prec == QG_FP32_IR ? "fp32" : "fp64");
        if (!std::isfinite(sr.pres) || !std::isfinite(sr.dres) || !std::isfinite(sr.gap)) {
            status = QG_NUMERICAL_ERROR;
            break;
        }
        if (sr.ok) { status = QG_SOLVED; break; }
        if (it >= st.max_iter) {
            const bool ok5 = kb > 1 ? all_pass(st.eps_inacc, st.eps_inacc)
                                    : stop_test(h, scal, st.eps_inacc, st.eps_inacc).ok;
            status = ok5 ? QG_SOLVED_INACCURATE : QG_MAX_ITER;
            break;
        }
        const double mu = nu > 0 ? sr.sz / nu : 0.0;
        // each problem's own complementarity measure for its centering (a batch: nu / kb cone units each)
        for (int32_t i = 0; i < kb; ++i) mu_host[(size_t)i] = nu > 0 ? scal_all[(size_t)i * NSCAL + S_SZ] / (nu / kb) : 0.0;
        QG_HIP(h, hipMemcpyAsync(d.mu.p, mu_host.data(), sizeof(double) * 2 * kb, hipMemcpyHostToDevice, h->stream));
        const double gscaled = sr.gap / std::max(1.0, std::min(std::fabs(sr.pobj), std::fabs(sr.dobj)));
        if (!fp64_only && gscaled < st.switch_gap) fp64_only = true;
        prec = fp64_only ? QG_FP64 : QG_FP32_IR;
        if (prec == QG_FP64 && switch_iter < 0 && st.precision == QG_FP32_IR) switch_iter = it;
        // scaling + (3,3) block, once per iteration (its time is read after the affine solve's wait)
        (void)hipEventRecord(ev.e[14], h->stream);
        if ((rc = launch_scaling(h, d.s.p, d.z.p, d.lam.p, 0))) return fail(rc);
        (void)hipEventRecord(ev.e[15], h->stream);
        bool scaling_timed = false;
        // Newton step; an FP32 factor whose refinement fails its test makes
        // the whole step run again with an FP64 factor (and FP64 from then on)
        for (int attempt = 0; attempt < 2; ++attempt) {
            (void)hipEventRecord(ev.e[2], h->stream);
            if ((rc = launch_factor(h, prec))) return fail(rc);
            (void)hipEventRecord(ev.e[3], h->stream);
            if ((rc = nreg_async(h))) return fail(rc);
            ++nfactor;
            // affine direction
            if ((rc = launch_build_rhs(h, d.s.p, 1.0, d.rhs.p))) return fail(rc);
            bool failed = false, failed2 = false;
            if ((rc = solve_with(h, d.rhs.p, dvec, prec, &ir_total, &failed, ev, &ms_solve, work))) return fail(rc);
            ++nsolve;
            ms_factor += elapsed(ev.e[2], ev.e[3]);
            if (!scaling_timed) {
                ms_cone += elapsed(ev.e[14], ev.e[15]);
                scaling_timed = true;
            }
            nreg_total += nreg_pinned(h);   // copied before the solve, which has been waited for
            if (!failed) {
                (void)hipEventRecord(ev.e[6], h->stream);
                if ((rc = launch_ds_from_dz(h, d.s.p, -1.0, dz_of, d.dsa.p))) return fail(rc);
                if ((rc = launch_reset_steps(h))) return fail(rc);
                if ((rc = launch_step_min(h, d.s.p, d.dsa.p, 0))) return fail(rc);
                if ((rc = launch_step_min(h, d.z.p, dz_of, 1))) return fail(rc);
                // corrector (sigma from the affine step length on the device)
                if ((rc = launch_corrector(h, d.dsa.p, dz_of, -1.0, d.mu.p, d.t.p))) return fail(rc);
                if ((rc = launch_build_rhs(h, d.t.p, -1.0, d.rhs.p))) return fail(rc);
                (void)hipEventRecord(ev.e[7], h->stream);
                if ((rc = solve_with(h, d.rhs.p, dvec, prec, &ir_total, &failed2, ev, &ms_solve, work))) return fail(rc);
                ++nsolve;
                ms_cone += elapsed(ev.e[6], ev.e[7]);
            }
            if ((failed || failed2) && prec == QG_FP32_IR) {
                fp64_only = true;
                prec = QG_FP64;
                if (switch_iter < 0) switch_iter = it;
                continue;
            }
            break;
        }
        (void)hipEventRecord(T[1], h->stream);
        if ((rc = launch_ds_from_dz(h, d.t.p, 1.0, dz_of, d.ds.p))) return fail(rc);
        if ((rc = launch_step_min(h, d.s.p, d.ds.p, 2))) return fail(rc);
        if ((rc = launch_step_min(h, d.z.p, dz_of, 3))) return fail(rc);
        if ((rc = launch_update(h, dvec, d.ds.p, st.step_frac, d.alpha.p + 1))) return fail(rc);
        (void)hipEventRecord(T[2], h->stream);
        pending = par;                     // no wait here: the next residual's wait covers it
        pending_is32 = prec == QG_FP32_IR ? 1 : 0;
        ++it;
    }
    // outputs (equilibrated data: back to the caller's units)
    if (h->ruiz > 0) {
        if ((rc = launch_unscale_outputs(h, xo, so, yo, zo))) return fail(rc);
    } else {
        if (xo) QG_HIP(h, hipMemcpyAsync(xo, d.x.p, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
        if (so) QG_HIP(h, hipMemcpyAsync(so, d.s.p, sizeof(double) * m, hipMemcpyDeviceToDevice, h->stream));
        if (yo) QG_HIP(h, hipMemcpyAsync(yo, d.y.p, sizeof(double) * p, hipMemcpyDeviceToDevice, h->stream));
        if (zo) QG_HIP(h, hipMemcpyAsync(zo, d.z.p, sizeof(double) * m, hipMemcpyDeviceToDevice, h->stream));
    }
    h->solved = (status == QG_SOLVED || status == QG_SOLVED_INACCURATE);
    h->last_status = status;
    // derivative system at the final iterate (FP64), kept for qg_backward
    if (h->solved && st.differentiable) {
        if ((rc = launch_scaling(h, d.s.p, d.z.p, nullptr, 1))) return fail(rc);
        if ((rc = launch_factor(h, QG_FP64))) return fail(rc);
        ++nfactor;
        h->final_factor = true;
    }
    QG_HIP(h, hipStreamSynchronize(h->stream));
    ev.destroy();
    if (info) {
        info->status = status;
        info->iters = it;
        info->switch_iter = switch_iter;
        info->ir_steps = ir_total;
        info->nreg = nreg_total;
        info->nfactor = nfactor;
        info->nsolve = nsolve;
        info->pobj = sr.pobj; info->dobj = sr.dobj;
        info->pres = sr.pres; info->dres = sr.dres; info->gap = sr.gap;
        info->ms_setup = h->ms_setup;
        info->ms_analyze = h->ms_analyze;
        info->ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
        info->ms_factor = ms_factor;
        info->ms_trisolve = ms_solve;
        info->ms_cone = ms_cone;
        info->ms_step_median = median(step_ms);
        info->ms_step_median_fp32 = median(step32);
        info->ms_step_median_fp64 = median(step64);
        info->ms_step_p90 = percentile(step_ms, 0.9);
        info->ntrisolve[0] = work.tri[0];
        info->ntrisolve[1] = work.tri[1];
        info->nresidual = work.residuals;
        info->nstep_ms = (int32_t)std::min<size_t>(step_ms.size(), QG_STEP_MS_MAX);
        for (int32_t k = 0; k < info->nstep_ms; ++k) {
            info->step_ms[k] = step_ms[(size_t)k];
            info->step_fp32[k] = step_is32[(size_t)k];
        }
        info->nnz_L = h->sym.nnz_L;
        info->factor_flops = h->sym.flops;
        prof_collect(h, info->kern_launches, info->kern_ms, info->kern_flops);
    } else {
        int64_t a[4]; double b_[4], c_[4];
        prof_collect(h, a, b_, c_);
    }
    return QG_OK;
}

}  // namespace qg
