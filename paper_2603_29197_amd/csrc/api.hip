// C ABI (qg.h): setup / update / solve / backward, the host-only analysis,
// and the step-level entry points.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "batch.hpp"
#include "vec.hpp"

struct qg_symbolic {
    qg::ProblemPattern pp;
    qg::KktPattern kp;
    qg::Symbolic sym;
    qg::Symbolic fronts;
};

namespace qg {

// ----------------------------------------------------------------------------
// adjoint: K_fin u = [g; 0; 0] on the stored derivative factor (FP64 + IR)
// ----------------------------------------------------------------------------
__global__ void dP_kernel(int32_t n, const int64_t *__restrict__ Pp, const int32_t *__restrict__ Pi,
                          const double *__restrict__ u, const double *__restrict__ x, double *__restrict__ dP) {
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    for (int64_t t = Pp[j]; t < Pp[j + 1]; ++t) {
        const int32_t i = Pi[t];
        dP[t] = (i == j) ? -u[i] * x[i] : -(u[i] * x[j] + u[j] * x[i]);
    }
}

// On the pattern of a constraint matrix M (columns = primal variables, rows
// = the constraint's dual variables v): dL/dM_ij = -(v_i u_x,j + u_v,i x_j),
// one thread per column.
__global__ void dM_kernel(int32_t n, const int64_t *__restrict__ Mp, const int32_t *__restrict__ Mi,
                          const double *__restrict__ v, const double *__restrict__ uv,
                          const double *__restrict__ ux, const double *__restrict__ x, double *__restrict__ dM) {
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    for (int64_t t = Mp[j]; t < Mp[j + 1]; ++t) {
        const int32_t i = Mi[t];
        dM[t] = -(v[i] * ux[j] + uv[i] * x[j]);
    }
}

// rhs_x[j] = g[j] - sum_i G_ij gs[i] (G' g_s, G's values read from the K values), one thread per column
__global__ void gx_minus_gtgs_kernel(int32_t n, const int64_t *__restrict__ Gp, const int32_t *__restrict__ Gi,
                                     const int64_t *__restrict__ posG, const double *__restrict__ kval,
                                     const double *__restrict__ g, const double *__restrict__ gs,
                                     double *__restrict__ out) {
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    double acc = 0.0;
    for (int64_t t = Gp[j]; t < Gp[j + 1]; ++t) acc += kval[posG[t]] * gs[Gi[t]];
    out[j] = g[j] - acc;
}

int adjoint_backward(qg_handle *h, const double *g, const double *gy, const double *gz, const double *gs,
                     double *dc, double *dh, double *db, double *dP, double *dA, double *dG) {
    Device &d = h->d;
    const int32_t n = h->n, p = h->p, m = h->m;
    int rc;
    // rhs = [g - G' g_s; g_y; g_z]  (ds = dh - G dx - dG x carries g_s)
    if (gs && m > 0 && !h->pp.G.rowind.empty()) {
        gx_minus_gtgs_kernel<<<(n + 255) / 256, 256, 0, h->stream>>>(n, d.Gp.p, d.Gi.p, d.posG.p, d.kval.p, g, gs,
                                                                      d.rhs.p);
        QG_HIP(h, hipGetLastError());
    } else {
        QG_HIP(h, hipMemcpyAsync(d.rhs.p, g, sizeof(double) * n, hipMemcpyDeviceToDevice, h->stream));
    }
    if (p > 0) {
        if (gy) QG_HIP(h, hipMemcpyAsync(d.rhs.p + n, gy, sizeof(double) * p, hipMemcpyDeviceToDevice, h->stream));
        else if ((rc = launch_fill(h, p, 0.0, d.rhs.p + n))) return rc;
    }
    if (m > 0) {
        if (gz) QG_HIP(h, hipMemcpyAsync(d.rhs.p + n + p, gz, sizeof(double) * m, hipMemcpyDeviceToDevice, h->stream));
        else if ((rc = launch_fill(h, m, 0.0, d.rhs.p + n + p))) return rc;
    }
    if ((rc = refined_solve(h, d.rhs.p, d.sol.p, QG_FP64, 10, nullptr))) return rc;
    const double *u = d.sol.p;
    // u_z + g_s: the z-side factor of dL/dh and dL/dG (d.res is free after the refined solve)
    const double *uz = u + n + p;
    if (gs && m > 0) {
        QG_HIP(h, hipMemcpyAsync(d.res.p, uz, sizeof(double) * m, hipMemcpyDeviceToDevice, h->stream));
        if ((rc = launch_axpy(h, m, 1.0, gs, d.res.p))) return rc;
        uz = d.res.p;
    }
    if (dc && (rc = launch_scale_copy(h, n, -1.0, u, dc))) return rc;
    if (db && p > 0) QG_HIP(h, hipMemcpyAsync(db, u + n, sizeof(double) * p, hipMemcpyDeviceToDevice, h->stream));
    if (dh && m > 0) QG_HIP(h, hipMemcpyAsync(dh, uz, sizeof(double) * m, hipMemcpyDeviceToDevice, h->stream));
    if (dP && !h->pp.P.rowind.empty()) {
        dP_kernel<<<(n + 255) / 256, 256, 0, h->stream>>>(n, d.Pp.p, d.Pi.p, u, d.x.p, dP);
        QG_HIP(h, hipGetLastError());
    }
    if (dA && !h->pp.A.rowind.empty()) {
        dM_kernel<<<(n + 255) / 256, 256, 0, h->stream>>>(n, d.Ap.p, d.Ai.p, d.y.p, u + n, u, d.x.p, dA);
        QG_HIP(h, hipGetLastError());
    }
    if (dG && !h->pp.G.rowind.empty()) {
        dM_kernel<<<(n + 255) / 256, 256, 0, h->stream>>>(n, d.Gp.p, d.Gi.p, d.z.p, uz, u, d.x.p, dG);
        QG_HIP(h, hipGetLastError());
    }
    QG_HIP(h, hipStreamSynchronize(h->stream));
    return QG_OK;
}

static bool finite_all(const double *v, int64_t len) {
    for (int64_t i = 0; i < len; ++i) if (!std::isfinite(v[i])) return false;
    return true;
}

// Number of non-finite entries over up to three device vectors (NULL skipped), into *bad.
__global__ void count_nonfinite_kernel(const double *__restrict__ a, int32_t na, const double *__restrict__ b,
                                       int32_t nb, const double *__restrict__ c, int32_t nc, int32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    int f = 0;
    if (a && i < na && !isfinite(a[i])) f = 1;
    if (b && i < nb && !isfinite(b[i])) f = 1;
    if (c && i < nc && !isfinite(c[i])) f = 1;
    if (f) atomicAdd(bad, 1);
}

static int count_nonfinite(qg_handle *h, const double *a, int32_t na, const double *b, int32_t nb,
                           const double *c, int32_t nc, int *bad) {
    const int32_t len = std::max({a ? na : 0, b ? nb : 0, c ? nc : 0});
    *bad = 0;
    if (len <= 0) return QG_OK;
    int32_t *cnt = h->d.flag.p;
    QG_HIP(h, hipMemsetAsync(cnt, 0, sizeof(int32_t), h->stream));
    count_nonfinite_kernel<<<(len + 255) / 256, 256, 0, h->stream>>>(a, na, b, nb, c, nc, cnt);
    QG_HIP(h, hipGetLastError());
    int32_t v = 0;
    QG_HIP(h, hipMemcpyAsync(&v, cnt, sizeof(v), hipMemcpyDeviceToHost, h->stream));
    QG_HIP(h, hipStreamSynchronize(h->stream));
    *bad = v;
    return QG_OK;
}

static int allocate_device(qg_handle *h) {
    Device &d = h->d;
    const Plan &pl = h->plan;
    const KktPattern &kp = h->kp;
    int rc;
#define UP(buf, vec) if ((rc = dupload(h, d.buf, vec))) return rc
    std::vector<int32_t> perm(h->fronts.perm), iperm(h->fronts.iperm);
    UP(perm, perm);
    UP(iperm, iperm);
    UP(blk33, kp.blk33);
    UP(blk_off, kp.blk33_off);
    UP(soc_off, h->pp.soc_off);
    {
        std::vector<int32_t> big;
        for (int32_t k = 0; k < h->pp.nsoc; ++k)
            if (h->pp.soc_off[k + 1] - h->pp.soc_off[k] >= QBIG) big.push_back(k);
        h->nbig = (int32_t)big.size();
        // every cone of one problem with the same 2 <= q <= 16 entries: lane-group cone kernels
        h->grp_q = 0;
        if (h->ncopy == 1 && h->pp.nsoc > 0) {
            const int32_t q0 = h->pp.soc_off[1] - h->pp.soc_off[0];
            bool uni = q0 >= 2 && q0 <= 16;
            for (int32_t k = 1; k < h->pp.nsoc && uni; ++k) uni = h->pp.soc_off[k + 1] - h->pp.soc_off[k] == q0;
            if (uni) h->grp_q = q0;
        }
        UP(big_cones, big);
        std::vector<int32_t> ccone;
        std::vector<int64_t> cstart;
        for (int32_t j = 0; j < h->nbig; ++j) {
            const int64_t q = h->pp.soc_off[big[j] + 1] - h->pp.soc_off[big[j]];
            for (int64_t t = 0; t < q * (q + 1) / 2; t += BIG_CHUNK) { ccone.push_back(j); cstart.push_back(t); }
        }
        if (ccone.size() > 0x7fffffffu) return QG_ERR_ARG;
        h->nbigchunk = (int64_t)ccone.size();
        UP(big_chunk_cone, ccone);
        UP(big_chunk_start, cstart);
        if ((rc = dalloc(h, d.bigsc, 2 * (size_t)h->nbig))) return rc;
    }
    UP(sn_first, pl.sn_first);
    UP(sn_rows, pl.sn_rows);
    UP(task_sn, pl.task_sn);
    UP(task_col, pl.task_col);
    UP(ctb_src, pl.ctb_src);
    UP(ch_ptr, pl.ch_ptr);
    UP(ch_list, pl.ch_list);
    UP(lvl_small_sn, pl.lvl_small_sn);
    UP(sn_rptr, pl.sn_rptr);
    UP(fr_off, pl.fr_off);
    UP(task_ptr, pl.task_ptr);
    UP(ctb_ptr, pl.ctb_ptr);
    UP(uv_off, pl.uv_off);
    UP(ent_dst, pl.ent_dst);
    UP(ent_sptr, pl.ent_sptr);
    UP(ent_reg, pl.ent_reg);
    UP(ent_src, pl.ent_src);
    UP(zseg_off, pl.zseg_off);
    UP(zseg_len, pl.zseg_len);
    UP(task0, pl.task0);
    UP(reg_sign, pl.reg_sign);
    UP(chain_comp_ptr, pl.chain_comp_ptr);
    UP(chain_grp_ptr, pl.chain_grp_ptr);
    UP(chain_sn, pl.chain_sn);
    UP(ent_front, pl.ent_front);
    std::vector<int32_t> zc((size_t)h->m, -1);
    for (int32_t k = 0; k < h->pp.nsoc; ++k)
        for (int32_t r = h->pp.soc_off[k]; r < h->pp.soc_off[k + 1]; ++r) zc[r] = k;
    UP(zcone, zc);
    UP(Pp, h->pp.P.colptr);
    UP(Pi, h->pp.P.rowind);
    UP(Ap, h->pp.A.colptr);
    UP(Ai, h->pp.A.rowind);
    UP(Gp, h->pp.G.colptr);
    UP(Gi, h->pp.G.rowind);
    UP(posG, kp.posG);
#undef UP
    const size_t N = (size_t)h->N, m = (size_t)h->m;
    // One factor exists at a time (FP32 while the FP32+IR mode is on, FP64 from the switch on),
    // so the FP32 fronts, inverses and W blocks are views into the FP64 buffers: 8 bytes per
    // stored entry instead of 12.
    if ((rc = dalloc(h, d.front64, (size_t)pl.front_total))) return rc;
    if ((rc = dalloc(h, d.uvec, (size_t)pl.uv_total))) return rc;
    if ((rc = dalloc(h, d.vwork, (size_t)pl.task_sn.size()))) return rc;
    if ((rc = dalloc(h, d.dinv64, (size_t)pl.dinv_total))) return rc;
    if ((rc = dalloc(h, d.sinv64, (size_t)pl.sinv_total))) return rc;
    if ((rc = dalloc(h, d.w64, (size_t)pl.w_total))) return rc;
    auto view32 = [](DBuf<float> &v, const DBuf<double> &b) { v.p = reinterpret_cast<float *>(b.p); v.n = b.n; };
    view32(d.front32, d.front64);
    view32(d.dinv32, d.dinv64);
    view32(d.sinv32, d.sinv64);
    view32(d.w32, d.w64);
    if ((rc = dalloc(h, d.ubuf, (size_t)pl.max_r * pl.ncopy))) return rc;
    if ((rc = dalloc(h, d.vbuf, (size_t)pl.max_r * pl.ncopy))) return rc;
    if ((rc = dalloc(h, d.nreg, 1))) return rc;
    if ((rc = dalloc(h, d.x, (size_t)h->n))) return rc;
    if ((rc = dalloc(h, d.y, (size_t)h->p))) return rc;
    if ((rc = dalloc(h, d.s, m))) return rc;
    if ((rc = dalloc(h, d.z, m))) return rc;
    if ((rc = dalloc(h, d.rx, (size_t)h->n))) return rc;
    if ((rc = dalloc(h, d.ry, (size_t)h->p))) return rc;
    if ((rc = dalloc(h, d.rz, m))) return rc;
    if ((rc = dalloc(h, d.rhs, N))) return rc;
    if ((rc = dalloc(h, d.sol, N))) return rc;
    if ((rc = dalloc(h, d.res, N))) return rc;
    if ((rc = dalloc(h, d.corr, N))) return rc;
    if ((rc = dalloc(h, d.xp, N))) return rc;
    if ((rc = dalloc(h, d.dsa, m))) return rc;
    if ((rc = dalloc(h, d.ds, m))) return rc;
    if ((rc = dalloc(h, d.t, m))) return rc;
    if ((rc = dalloc(h, d.lam, m))) return rc;
    if ((rc = dalloc(h, d.w, (size_t)h->pp.l))) return rc;
    if ((rc = dalloc(h, d.wbar, m))) return rc;
    if ((rc = dalloc(h, d.beta, (size_t)h->pp.nsoc))) return rc;
    if ((rc = dalloc(h, d.scal, 64))) return rc;
    if ((rc = dalloc(h, d.scal_inst, (size_t)h->ncopy * NSCAL))) return rc;
    if ((rc = dalloc(h, d.alpha, 4))) return rc;
    if ((rc = dalloc(h, d.amin, 4 * (size_t)h->ncopy))) return rc;
    if ((rc = dalloc(h, d.mu, 2 * (size_t)h->ncopy))) return rc;
    if ((rc = dalloc(h, d.flag, 1))) return rc;
    // per-block partials: the sparse residual kernels use 256 / RL rows per block
    size_t nblk = (N + 256 / RL - 1) / (256 / RL) + (size_t)((h->pp.l + h->pp.nsoc + 255) / 256) +
                  (size_t)((h->nbig + 3) / 4) + 1 + (size_t)h->ncopy;
    // the residual reductions: at most RED_BLOCKS blocks per problem of a batch
    const int64_t rows1 = N / h->ncopy;
    nblk = std::max<size_t>(nblk, (size_t)h->ncopy * (size_t)std::min<int64_t>(RED_BLOCKS, rows1 / 64 + 1));
    if ((rc = dalloc(h, d.partials, nblk * NSCAL))) return rc;
    return QG_OK;
}

static int check_device(qg_handle *h) {
    int dev = 0, count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return QG_ERR_DEVICE;
    QG_HIP(h, hipGetDevice(&dev));
    hipDeviceProp_t prop;
    QG_HIP(h, hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return QG_ERR_DEVICE;
    h->device = dev;
    return QG_OK;
}

}  // namespace qg

using namespace qg;

extern "C" {

int qg_default_settings(qg_settings *s) {
    if (!s) return QG_ERR_ARG;
    s->eps_abs = 1e-8;
    s->eps_rel = 1e-8;
    s->eps_inacc = 1e-5;
    s->max_iter = 100;
    s->precision = QG_FP64;
    s->switch_gap = 1e-6;
    s->static_reg = 1e-8;
    s->dyn_eps = 1e-13;
    s->dyn_delta = 1e-7;
    s->static_reg32 = 1e-4;
    s->dyn_eps32 = 1e-8;
    s->dyn_delta32 = 1e-4;
    s->ir_max = 3;
    s->ir_max32 = 10;
    s->ir_tol = 1e-12;
    s->step_frac = 0.99;
    s->differentiable = 0;
    s->verbose = 0;
    s->profile = 0;
    s->chains = 1;
    s->fp32_min_flops = 1e10;
    s->ordering = QG_ORDER_MD;
    s->cone_lanes = 1;
    s->tiny_groups = 1;
    s->graphs = 1;
    s->ruiz_iters = 0;
    return QG_OK;
}

const char *qg_strerror(int code) {
    switch (code) {
        case QG_OK: return "ok";
        case QG_ERR_ARG: return "invalid argument";
        case QG_ERR_PATTERN: return "invalid sparsity pattern";
        case QG_ERR_NONFINITE: return "non-finite value in the data";
        case QG_ERR_OOM: return "out of memory";
        case QG_ERR_HIP: return "HIP runtime error";
        case QG_ERR_STATE: return "call out of order";
        case QG_ERR_DEVICE: return "no gfx950 device";
        case QG_ERR_SIZE: return "input exceeds a fixed capacity";
        default: return "unknown error";
    }
}

int qg_analyze(qg_symbolic **out, qg_int n, qg_int m, qg_int p, const qg_csc *P, const qg_csc *A,
               const qg_csc *G, qg_int l, qg_int nsoc, const qg_int *q, int ordering) {
    if (!out || (ordering != QG_ORDER_MD && ordering != QG_ORDER_ND)) return QG_ERR_ARG;
    *out = nullptr;
    qg_symbolic *s = new (std::nothrow) qg_symbolic();
    if (!s) return QG_ERR_OOM;
    try {
        int rc = build_problem_pattern(s->pp, n, m, p, P, A, G, l, nsoc, q, false);
        if (rc) { delete s; return rc; }
        build_kkt_pattern(s->pp, s->kp);
        analyze_pattern(s->kp, s->sym, ordering);
        if ((rc = group_fronts(s->sym, s->fronts))) { delete s; return rc; }
    } catch (const std::bad_alloc &) {
        delete s;
        return QG_ERR_OOM;
    } catch (...) {
        delete s;
        return QG_ERR_PATTERN;
    }
    *out = s;
    return QG_OK;
}

static void fill_pattern(const Symbolic &sym, const Symbolic &fr, qg_pattern *o) {
    o->N = sym.N;
    o->nsuper_fund = (qg_int)sym.super_fund.size() - 1;
    o->nsuper = (qg_int)sym.super_ptr.size() - 1;
    o->perm = sym.perm.data();
    o->iperm = sym.iperm.data();
    o->parent = sym.parent.data();
    o->colcount = sym.colcount.data();
    o->super_fund = sym.super_fund.data();
    o->super_ptr = sym.super_ptr.data();
    o->rows_ptr = sym.rows_ptr.data();
    o->rows = sym.rows.data();
    o->nfront = (qg_int)fr.super_ptr.size() - 1;
    o->front_perm = fr.perm.data();
    o->front_ptr = fr.super_ptr.data();
    o->front_rows_ptr = fr.rows_ptr.data();
    o->front_rows = fr.rows.data();
    o->nchain_front = 0;
}

int qg_symbolic_pattern(const qg_symbolic *sym, qg_pattern *out) {
    if (!sym || !out) return QG_ERR_ARG;
    fill_pattern(sym->sym, sym->fronts, out);
    return QG_OK;
}

void qg_symbolic_free(qg_symbolic *sym) { delete sym; }

void qg_cleanup(qg_handle *h) {
    if (!h) return;
    drop_graphs(h);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->bulk) (void)hipStreamSynchronize(h->bulk);
    if (h->prep) (void)hipStreamSynchronize(h->prep);
    dfree_all(h);
    for (hipEvent_t e : {h->ev_panel, h->ev_bulk, h->ev_prep})
        if (e) (void)hipEventDestroy(e);
    if (h->bulk) (void)hipStreamDestroy(h->bulk);
    if (h->prep) (void)hipStreamDestroy(h->prep);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->ev_sync) (void)hipEventDestroy(h->ev_sync);
    if (h->pin) (void)hipHostFree(h->pin);
    delete h;
}

// Side streams and ordering events of the factorization.
static int create_streams(qg_handle *h) {
    QG_HIP(h, hipStreamCreateWithFlags(&h->bulk, hipStreamNonBlocking));
    QG_HIP(h, hipStreamCreateWithFlags(&h->prep, hipStreamNonBlocking));
    QG_HIP(h, hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    QG_HIP(h, hipEventCreateWithFlags(&h->ev_sync, hipEventDisableTiming));
    QG_HIP(h, hipHostMalloc((void **)&h->pin, PIN_DOUBLES * sizeof(double), hipHostMallocDefault));
    QG_HIP(h, hipEventCreateWithFlags(&h->ev_panel, hipEventDisableTiming));
    QG_HIP(h, hipEventCreateWithFlags(&h->ev_bulk, hipEventDisableTiming));
    QG_HIP(h, hipEventCreateWithFlags(&h->ev_prep, hipEventDisableTiming));
    return QG_OK;
}

int qg_setup(qg_handle **out, qg_int n, qg_int m, qg_int p, const qg_csc *P, const double *c,
             const qg_csc *A, const double *b, const qg_csc *G, const double *hv, qg_int l, qg_int nsoc,
             const qg_int *q, const qg_settings *s, void *hip_stream, qg_alloc_fn alloc, qg_free_fn free_fn,
             void *alloc_ctx) {
    if (!out) return QG_ERR_ARG;
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return QG_ERR_ARG;
    if (s && s->ordering != QG_ORDER_MD && s->ordering != QG_ORDER_ND) return QG_ERR_ARG;
    if (s && (s->ruiz_iters < 0 || s->ruiz_iters > QG_RUIZ_MAX || (s->ruiz_iters > 0 && s->differentiable)))
        return QG_ERR_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    qg_handle *h = new (std::nothrow) qg_handle();
    if (!h) return QG_ERR_OOM;
    if (s) h->st = *s; else qg_default_settings(&h->st);
    h->ruiz = h->st.ruiz_iters;
    h->stream = (hipStream_t)hip_stream;
    h->alloc = alloc;
    h->free_fn = free_fn;
    h->alloc_ctx = alloc_ctx;
    int rc = QG_OK;
    try {
        rc = build_problem_pattern(h->pp, n, m, p, P, A, G, l, nsoc, q, true);
        if (!rc && (!c || (p > 0 && !b) || (m > 0 && !hv))) rc = QG_ERR_ARG;
        if (!rc && (!finite_all(c, n) || (p > 0 && !finite_all(b, p)) || (m > 0 && !finite_all(hv, m))))
            rc = QG_ERR_NONFINITE;
        if (rc) { delete h; return rc; }
        h->n = n; h->m = m; h->p = p; h->N = n + m + p;
        h->hc.assign(c, c + n);
        h->hb.assign(b ? b : c, b ? b + p : c);
        h->hh.assign(hv ? hv : c, hv ? hv + m : c);
        if ((rc = check_device(h))) { delete h; return rc; }
        build_kkt_pattern(h->pp, h->kp);
        h->nnzK = (int64_t)h->kp.Ki.size();
        const auto ta = std::chrono::steady_clock::now();
        analyze_pattern(h->kp, h->sym, h->st.ordering);
        h->ms_analyze = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
        if ((rc = build_plan(h))) { qg_cleanup(h); return rc; }
        if ((rc = create_streams(h))) { qg_cleanup(h); return rc; }
        if ((rc = allocate_device(h))) { qg_cleanup(h); return rc; }
        if ((rc = factor_init_attributes(h))) { qg_cleanup(h); return rc; }
        if ((rc = upload_static_values(h, true))) { qg_cleanup(h); return rc; }
        if (hipStreamSynchronize(h->stream) != hipSuccess) { qg_cleanup(h); return QG_ERR_HIP; }
    } catch (const std::bad_alloc &) {
        qg_cleanup(h);
        return QG_ERR_OOM;
    } catch (...) {
        qg_cleanup(h);
        return QG_ERR_PATTERN;
    }
    h->ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return QG_OK;
}

// Cone-ordered rows of the stack -> problem-major rows: out[i m + w] = in[zrow(i, w)].
__global__ void unstack_cone_rows(const double *__restrict__ in, double *__restrict__ out, int32_t k, int32_t m,
                                  int32_t l) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (int64_t)k * m) return;
    const int32_t i = (int32_t)(t / m), w = (int32_t)(t % m);
    const int64_t src = w < l ? (int64_t)i * l + w : (int64_t)k * l + (int64_t)i * (m - l) + (w - l);
    out[t] = in[src];
}

int qg_setup_batch(qg_handle **out, qg_int k, qg_int n, qg_int m, qg_int p, const qg_csc *P, const double *c,
                   const qg_csc *A, const double *b, const qg_csc *G, const double *hv, qg_int l, qg_int nsoc,
                   const qg_int *q, const qg_settings *s, void *hip_stream, qg_alloc_fn alloc, qg_free_fn free_fn,
                   void *alloc_ctx) {
    if (!out) return QG_ERR_ARG;
    *out = nullptr;
    if (k < 1 || n < 0 || m < 0 || p < 0 || l < 0 || nsoc < 0) return QG_ERR_ARG;
    if ((alloc == nullptr) != (free_fn == nullptr)) return QG_ERR_ARG;
    if (s && s->ordering != QG_ORDER_MD && s->ordering != QG_ORDER_ND) return QG_ERR_ARG;
    if (s && s->ruiz_iters != 0) return QG_ERR_ARG;
    if ((int64_t)k * (n + m + p) > INT32_MAX) return QG_ERR_ARG;
    const auto t0 = std::chrono::steady_clock::now();
    qg_handle *h = new (std::nothrow) qg_handle();
    if (!h) return QG_ERR_OOM;
    if (s) h->st = *s; else qg_default_settings(&h->st);
    h->st.differentiable = 0;
    h->stream = (hipStream_t)hip_stream;
    h->alloc = alloc;
    h->free_fn = free_fn;
    h->alloc_ctx = alloc_ctx;
    int rc = QG_OK;
    try {
        // one problem's pattern: validated, analysed once
        ProblemPattern pp1;
        rc = build_problem_pattern(pp1, n, m, p, P, A, G, l, nsoc, q, false);
        if (!rc && (!c || (p > 0 && !b) || (m > 0 && !hv))) rc = QG_ERR_ARG;
        if (!rc && ((P && !P->val) || (A && !A->val) || (G && !G->val))) rc = QG_ERR_ARG;
        if (rc) { delete h; return rc; }
        auto nnz = [](const qg_csc *M) { return M ? (int64_t)M->colptr[M->ncol] : 0; };
        if ((P && !finite_all(P->val, k * nnz(P))) || (A && !finite_all(A->val, k * nnz(A))) ||
            (G && !finite_all(G->val, k * nnz(G))) || !finite_all(c, (int64_t)k * n) ||
            (p > 0 && !finite_all(b, (int64_t)k * p)) || (m > 0 && !finite_all(hv, (int64_t)k * m))) {
            delete h;
            return QG_ERR_NONFINITE;
        }
        StackMap mp;
        mp.k = k; mp.n = n; mp.p = p; mp.m = m; mp.l = l;
        StackedCsc Ps, As, Gs;
        stack_problem(mp, P, A, G, Ps, As, Gs);
        std::vector<int32_t> qs;
        for (int32_t i = 0; i < k; ++i) qs.insert(qs.end(), q, q + nsoc);
        rc = build_problem_pattern(h->pp, k * n, k * m, k * p, P ? &Ps.csc : nullptr, A ? &As.csc : nullptr,
                                   G ? &Gs.csc : nullptr, k * l, k * nsoc, qs.data(), true);
        if (rc) { delete h; return rc; }
        h->ncopy = k;
        h->n1 = n; h->m1 = m; h->p1 = p; h->l1 = l;
        h->n = k * n; h->m = k * m; h->p = k * p; h->N = h->n + h->m + h->p;
        h->hc.assign(c, c + (size_t)k * n);
        h->hb.assign(b ? b : c, b ? b + (size_t)k * p : c);
        h->hh.assign((size_t)k * m, 0.0);
        for (int32_t i = 0; i < k; ++i)
            for (int32_t w = 0; w < m; ++w) h->hh[(size_t)mp.zrow(i, w)] = hv[(size_t)i * m + w];
        if ((rc = check_device(h))) { delete h; return rc; }
        build_kkt_pattern(h->pp, h->kp);
        h->nnzK = (int64_t)h->kp.Ki.size();
        const auto ta = std::chrono::steady_clock::now();
        KktPattern kp1;
        build_kkt_pattern(pp1, kp1);
        Symbolic sym1, fronts1;
        analyze_pattern(kp1, sym1, h->st.ordering);
        if ((rc = group_fronts(sym1, fronts1))) { qg_cleanup(h); return rc; }
        replicate_symbolic(sym1, mp, h->sym);
        replicate_symbolic(fronts1, mp, h->fronts);
        h->ms_analyze = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ta).count();
        if ((rc = build_plan(h))) { qg_cleanup(h); return rc; }
        if ((rc = create_streams(h))) { qg_cleanup(h); return rc; }
        if ((rc = allocate_device(h))) { qg_cleanup(h); return rc; }
        if ((rc = factor_init_attributes(h))) { qg_cleanup(h); return rc; }
        if ((rc = upload_static_values(h, true))) { qg_cleanup(h); return rc; }
        if (hipStreamSynchronize(h->stream) != hipSuccess) { qg_cleanup(h); return QG_ERR_HIP; }
    } catch (const std::bad_alloc &) {
        qg_cleanup(h);
        return QG_ERR_OOM;
    } catch (...) {
        qg_cleanup(h);
        return QG_ERR_PATTERN;
    }
    h->ms_setup = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = h;
    return QG_OK;
}

int qg_solve_batch(qg_handle *h, double *x, double *s, double *y, double *z, qg_info *info) {
    if (!h) return QG_ERR_ARG;
    int rc = ipm_solve(h, x, nullptr, y, nullptr, info);
    if (rc) return rc;
    const int64_t tot = (int64_t)h->ncopy * h->m1;
    if (tot > 0) {
        const unsigned g = (unsigned)((tot + 255) / 256);
        if (s) unstack_cone_rows<<<g, 256, 0, h->stream>>>(h->d.s.p, s, h->ncopy, h->m1, h->l1);
        if (z) unstack_cone_rows<<<g, 256, 0, h->stream>>>(h->d.z.p, z, h->ncopy, h->m1, h->l1);
        QG_HIP(h, hipGetLastError());
        QG_HIP(h, hipStreamSynchronize(h->stream));
    }
    return QG_OK;
}

int qg_update(qg_handle *h, const double *Pval, const double *c, const double *Aval, const double *b,
              const double *Gval, const double *hv) {
    if (!h) return QG_ERR_ARG;
    if (h->ncopy > 1) return QG_ERR_STATE;
    auto chk = [](const double *v, size_t len) { return v == nullptr || finite_all(v, (int64_t)len); };
    if (!chk(Pval, h->pp.P.val.size()) || !chk(c, h->n) || !chk(Aval, h->pp.A.val.size()) ||
        !chk(b, h->p) || !chk(Gval, h->pp.G.val.size()) || !chk(hv, h->m))
        return QG_ERR_NONFINITE;
    if (Pval) h->pp.P.val.assign(Pval, Pval + h->pp.P.val.size());
    if (Aval) h->pp.A.val.assign(Aval, Aval + h->pp.A.val.size());
    if (Gval) h->pp.G.val.assign(Gval, Gval + h->pp.G.val.size());
    h->solved = false;
    h->final_factor = false;
    // vectors go straight into the device copies (the host copies only serve setup); with Ruiz
    // equilibration into the caller's-units copies, and the scalings are formed again after them
    const bool rz = h->ruiz > 0;
    if (c && h->n > 0) QG_HIP(h, hipMemcpyAsync((rz ? h->d.craw : h->d.c).p, c, sizeof(double) * h->n, hipMemcpyHostToDevice, h->stream));
    if (b && h->p > 0) QG_HIP(h, hipMemcpyAsync((rz ? h->d.braw : h->d.b).p, b, sizeof(double) * h->p, hipMemcpyHostToDevice, h->stream));
    if (hv && h->m > 0) QG_HIP(h, hipMemcpyAsync((rz ? h->d.hraw : h->d.h).p, hv, sizeof(double) * h->m, hipMemcpyHostToDevice, h->stream));
    if (Pval || Aval || Gval) {
        const int rc = upload_static_values(h, false);
        if (rc) return rc;
    } else if (rz && (c || b || hv)) {
        const int rc = launch_scale_vectors(h);
        if (rc) return rc;
    }
    QG_HIP(h, hipStreamSynchronize(h->stream));
    return QG_OK;
}

int qg_update_vectors(qg_handle *h, const double *c, const double *b, const double *hv) {
    if (!h) return QG_ERR_ARG;
    if (h->ncopy > 1) return QG_ERR_STATE;
    int bad = 0;
    int rc = count_nonfinite(h, c, h->n, b, h->p, hv, h->m, &bad);
    if (rc) return rc;
    if (bad) return QG_ERR_NONFINITE;
    h->solved = false;
    h->final_factor = false;
    const bool rz = h->ruiz > 0;   // equilibrated data: the objective scaling k of the setup is kept
    if (c && h->n > 0) QG_HIP(h, hipMemcpyAsync((rz ? h->d.craw : h->d.c).p, c, sizeof(double) * h->n, hipMemcpyDeviceToDevice, h->stream));
    if (b && h->p > 0) QG_HIP(h, hipMemcpyAsync((rz ? h->d.braw : h->d.b).p, b, sizeof(double) * h->p, hipMemcpyDeviceToDevice, h->stream));
    if (hv && h->m > 0) QG_HIP(h, hipMemcpyAsync((rz ? h->d.hraw : h->d.h).p, hv, sizeof(double) * h->m, hipMemcpyDeviceToDevice, h->stream));
    if (rz && (c || b || hv)) {
        if ((rc = launch_scale_vectors(h))) return rc;
    }
    QG_HIP(h, hipStreamSynchronize(h->stream));
    return QG_OK;
}

int qg_set_settings(qg_handle *h, const qg_settings *s) {
    if (!h || !s) return QG_ERR_ARG;
    if (h->ruiz > 0 && s->differentiable) return QG_ERR_ARG;   // the equilibration is fixed at setup
    h->st = *s;
    drop_graphs(h);   // the captured launches hold the regularization parameters as arguments
    return QG_OK;
}

int qg_solve(qg_handle *h, double *x, double *s, double *y, double *z, qg_info *info) {
    if (!h) return QG_ERR_ARG;
    if (h->ncopy > 1) return QG_ERR_STATE;
    return ipm_solve(h, x, s, y, z, info);
}

int qg_backward(qg_handle *h, const double *dl_dx, double *dl_dc, double *dl_dh, double *dl_db,
                double *dl_dPval, double *dl_dAval, double *dl_dGval) {
    return qg_backward_full(h, dl_dx, nullptr, nullptr, nullptr, dl_dc, dl_dh, dl_db, dl_dPval, dl_dAval,
                            dl_dGval);
}

int qg_backward_full(qg_handle *h, const double *dl_dx, const double *dl_dy, const double *dl_dz,
                     const double *dl_ds, double *dl_dc, double *dl_dh, double *dl_db, double *dl_dPval,
                     double *dl_dAval, double *dl_dGval) {
    if (!h || !dl_dx) return QG_ERR_ARG;
    if (!h->solved || !h->final_factor) return QG_ERR_STATE;
    return adjoint_backward(h, dl_dx, dl_dy, dl_dz, dl_ds, dl_dc, dl_dh, dl_db, dl_dPval, dl_dAval, dl_dGval);
}

int qg_backward_batch(qg_handle *h, int32_t k, const double *dl_dx, const double *dl_dy, const double *dl_dz,
                      const double *dl_ds, double *dl_dc, double *dl_dh, double *dl_db, double *dl_dPval,
                      double *dl_dAval, double *dl_dGval) {
    if (!h || k < 0 || (k > 0 && !dl_dx)) return QG_ERR_ARG;
    if (!h->solved || !h->final_factor) return QG_ERR_STATE;
    const size_t n = (size_t)h->n, p = (size_t)h->p, m = (size_t)h->m;
    const size_t nP = (size_t)h->pp.P.rowind.size(), nA = (size_t)h->pp.A.rowind.size(),
                 nG = (size_t)h->pp.G.rowind.size();
    auto at = [](auto *base, size_t len, int32_t j) { return base ? base + len * (size_t)j : base; };
    for (int32_t j = 0; j < k; ++j) {
        const int rc = adjoint_backward(h, at(dl_dx, n, j), at(dl_dy, p, j), at(dl_dz, m, j), at(dl_ds, m, j),
                                        at(dl_dc, n, j), at(dl_dh, m, j), at(dl_db, p, j), at(dl_dPval, nP, j),
                                        at(dl_dAval, nA, j), at(dl_dGval, nG, j));
        if (rc) return rc;
    }
    return QG_OK;
}

int qg_get_pattern(const qg_handle *h, qg_pattern *out) {
    if (!h || !out) return QG_ERR_ARG;
    fill_pattern(h->sym, h->fronts, out);
    out->nchain_front = (qg_int)h->plan.chain_sn.size();
    return QG_OK;
}

int qg_last_hip_error(const qg_handle *h) { return h ? h->last_hip : 0; }

// ---------------------------- step-level ----------------------------------
int qg_step_scaling(qg_handle *h, const double *s, const double *z, double *lam, int block) {
    if (!h || !s || !z) return QG_ERR_ARG;
    h->final_factor = false;
    int rc = launch_scaling(h, s, z, h->d.lam.p, block);
    if (rc) return rc;
    if (lam && h->m > 0)
        QG_HIP(h, hipMemcpyAsync(lam, h->d.lam.p, sizeof(double) * h->m, hipMemcpyDeviceToDevice, h->stream));
    QG_HIP(h, hipStreamSynchronize(h->stream));
    return QG_OK;
}

int qg_step_get_kkt(const qg_handle *h, double *kval, int64_t *nnz) {
    if (!h) return QG_ERR_ARG;
    if (nnz) *nnz = h->nnzK;
    if (!kval) return QG_OK;
    qg_handle *hh = const_cast<qg_handle *>(h);
    QG_HIP(hh, hipMemcpyAsync(kval, h->d.kval.p, sizeof(double) * h->nnzK, hipMemcpyDeviceToHost, h->stream));
    QG_HIP(hh, hipStreamSynchronize(h->stream));
    return QG_OK;
}

int qg_step_factor(qg_handle *h, int precision, int *nreg) {
    if (!h || (precision != QG_FP64 && precision != QG_FP32_IR)) return QG_ERR_ARG;
    h->final_factor = false;
    int rc = launch_factor(h, precision);
    if (rc) return rc;
    return read_nreg(h, nreg);
}

int qg_step_get_factor(const qg_handle *h, const int64_t *Lp, const int32_t *Li, double *Lx, double *D) {
    if (!h || !Lp || !Li || !Lx || !D || h->last_precision < 0) return QG_ERR_ARG;
    qg_handle *hh = const_cast<qg_handle *>(h);
    const Plan &pl = h->plan;
    const size_t tot = (size_t)pl.front_total;
    std::vector<double> fr(tot);
    if (h->last_precision == QG_FP32_IR) {
        std::vector<float> f32(tot);
        QG_HIP(hh, hipMemcpyAsync(f32.data(), h->d.front32.p, sizeof(float) * tot, hipMemcpyDeviceToHost, h->stream));
        QG_HIP(hh, hipStreamSynchronize(h->stream));
        for (size_t i = 0; i < tot; ++i) fr[i] = f32[i];
    } else {
        QG_HIP(hh, hipMemcpyAsync(fr.data(), h->d.front64.p, sizeof(double) * tot, hipMemcpyDeviceToHost, h->stream));
        QG_HIP(hh, hipStreamSynchronize(h->stream));
    }
    // L and D in the analysis' numbering: column j of the analysis is column
    // fronts.iperm[sym.perm[j]] of the device fronts
    const int32_t N = h->N;
    std::vector<int32_t> dev(N), grp(N);
    for (int32_t j = 0; j < N; ++j) dev[j] = h->fronts.iperm[h->sym.perm[j]];
    for (int32_t s = 0; s < pl.ns; ++s)
        for (int32_t c = pl.sn_first[s]; c < pl.sn_first[s + 1]; ++c) grp[c] = s;
    for (int32_t col = 0; col < N; ++col) {
        const int32_t dc = dev[col], s = grp[dc];
        const int32_t jc = dc - pl.sn_first[s];
        const int64_t r = pl.sn_rptr[s + 1] - pl.sn_rptr[s];
        const int32_t *rows = pl.sn_rows.data() + pl.sn_rptr[s];
        const double *F = fr.data() + pl.fr_off[s];
        D[col] = F[(int64_t)jc * r + jc];
        for (int64_t t = Lp[col]; t < Lp[col + 1]; ++t) {
            if (Li[t] <= col || Li[t] >= N) return QG_ERR_PATTERN;
            const int32_t di = dev[Li[t]];
            const int32_t *it = std::lower_bound(rows, rows + r, di);
            if (it == rows + r || *it != di || it - rows <= jc) return QG_ERR_PATTERN;
            Lx[t] = F[(int64_t)jc * r + (it - rows)];
        }
    }
    return QG_OK;
}

int qg_step_solve(qg_handle *h, const double *rhs, double *x, int refine, int *steps) {
    if (!h || !rhs || !x || refine < 0 || h->last_precision < 0) return QG_ERR_ARG;
    int rc = refined_solve(h, rhs, x, h->last_precision, refine, steps);
    if (rc) return rc;
    QG_HIP(h, hipStreamSynchronize(h->stream));
    return QG_OK;
}

int qg_step_max_step(qg_handle *h, const double *u, const double *du, double *alpha) {
    if (!h || !u || !du || !alpha) return QG_ERR_ARG;
    int rc = launch_reset_steps(h);
    if (rc) return rc;
    if ((rc = launch_step_min(h, u, du, 0))) return rc;
    unsigned long long bits = 0;
    QG_HIP(h, hipMemcpyAsync(&bits, h->d.amin.p, sizeof(bits), hipMemcpyDeviceToHost, h->stream));
    QG_HIP(h, hipStreamSynchronize(h->stream));
    std::memcpy(alpha, &bits, sizeof(double));
    return QG_OK;
}

int qg_step_cone_op(qg_handle *h, int op, const double *u, const double *v, double *out) {
    if (!h || !u || !out || op < 0 || op > 4 || ((op == 3 || op == 4) && !v)) return QG_ERR_ARG;
    int rc = launch_cone_op(h, op, u, v, out);
    if (rc) return rc;
    QG_HIP(h, hipStreamSynchronize(h->stream));
    return QG_OK;
}

int qg_step_corrector(qg_handle *h, const double *ds_a, const double *dz_a, double sigma_mu, double *t) {
    if (!h || !ds_a || !dz_a || !t || !(sigma_mu >= 0.0)) return QG_ERR_ARG;
    int rc = launch_corrector(h, ds_a, dz_a, sigma_mu, h->d.mu.p, t);
    if (rc) return rc;
    QG_HIP(h, hipStreamSynchronize(h->stream));
    return QG_OK;
}

}  // extern "C"
