// Device solver state behind the C ABI (qg.h): problem data, the
// supernodal plan derived from the analysis, and every device buffer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "analysis.hpp"
#include "kernels.hpp"
#include "qg.h"

namespace qg {

// A device allocation owned by the handle.
template <typename T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
};

// Supernodal multifrontal plan (host copies + device copies).
//  * every supernode s owns a dense front of r_s x r_s (column-major,
//    leading dimension r_s) at fr_off[s]; its first k_s columns hold L (unit
//    diagonal implied, D on the diagonal) after the factorization and its
//    trailing (r_s-k_s)^2 block the update passed to the parent;
//  * fronts are assembled column by column: task (s, j) zeroes column j,
//    scatters the K entries of that column and adds, in child order, every
//    child column that maps onto it (relative indices);
//  * small fronts (r_s <= SMALL_R) are factored one workgroup per front in
//    LDS, level by level; large fronts by a blocked right-looking sequence.
struct Plan {
    int32_t ns = 0, nlevels = 0;
    std::vector<int32_t> sn_first;        // ns + 1
    std::vector<int64_t> sn_rptr;         // ns + 1 (row lists)
    std::vector<int32_t> sn_rows;
    std::vector<int64_t> fr_off;          // ns + 1 (front offsets, elements)
    std::vector<int32_t> lvl_ptr, lvl_sn; // supernodes by level
    std::vector<int32_t> lvl_small_ptr, lvl_small_sn;   // small ones by level
    std::vector<int32_t> lvl_small_maxr;                // largest small front per level
    std::vector<int64_t> lvl_small_rsum;                // rows of the small fronts per level, summed
    std::vector<int32_t> lvl_tiny_cnt;                  // leading small fronts of <= TINY_R rows run on lane
                                                        // groups (0: the level has fewer than TINY_MIN)
    std::vector<int32_t> lvl_tiny8_cnt;                 // leading ones among those of <= TINY_R8 rows
    std::vector<int32_t> lvl_large_ptr, lvl_large_sn;   // large ones by level
    std::vector<int64_t> task_ptr;        // per level: column tasks (s, j)
    std::vector<int32_t> task_sn, task_col;
    std::vector<int64_t> task0;           // per supernode: task index of its column 0
    std::vector<int64_t> asm_ptr;         // per (s, j) task: K entries of that column
    std::vector<int64_t> asm_src;         // index into kval
    std::vector<int32_t> asm_row;         // local row in the front
    std::vector<int64_t> ctb_ptr;         // per task: child contributions
    std::vector<int32_t> ctb_child, ctb_col;
    std::vector<int64_t> ctb_src;         // position of each contribution in the solve work vector
    std::vector<int64_t> rel_ptr;         // per supernode: relative map of its update rows
    std::vector<int32_t> rel;
    // numeric assembly, level by level: every front entry that receives a value, with its
    // sources in summation order (the K entry first, then the children's update entries in
    // child order), and the segments of front storage cleared before the gather
    std::vector<int64_t> ent_lvl_ptr;     // nlevels + 1
    std::vector<int64_t> ent_dst;         // destination (offset in the front buffer)
    std::vector<int64_t> ent_sptr;        // sources of each entry (nent + 1)
    std::vector<int8_t> ent_reg;          // pivot kind for the static regularization of a pivot diagonal, else -1
    std::vector<int64_t> ent_src;         // >= 0: offset in the front buffer (a child's update entry);
                                          // < 0: -(index into the K values) - 1
    std::vector<int64_t> zseg_lvl_ptr;    // nlevels + 1
    std::vector<int64_t> zseg_off;        // cleared segments: offset and length
    std::vector<int32_t> zseg_len;
    std::vector<int64_t> uv_off;          // per supernode: offset of its update vector (solves)
    std::vector<int64_t> dinv_off;        // per supernode: offset of its inverse diagonal blocks
    int64_t dinv_total = 0;
    std::vector<int64_t> sinv_off;        // per supernode: inverses (X, X') of its SB x SB diagonal blocks
    int64_t sinv_total = 0;
    std::vector<int64_t> w_off;           // per supernode: the blocks W_J = L(below J, J) X_J, super-block
                                          // by super-block, each column-major with ld = r - J1
    int64_t w_total = 0;
    std::vector<int32_t> ch_ptr, ch_list; // children supernodes
    std::vector<int8_t> reg_sign;         // per permuted column: +1 x, -1 y, 0 z
    int64_t front_total = 0, uv_total = 0;
    int32_t max_r = 0;
    double large_flops = 0.0;             // dense flops of the large fronts per factorization
    // batch of ncopy identical problems (qg_setup_batch): fronts [z ns1, (z + 1) ns1) are copy z of
    // fronts [0, ns1); a large front's copies are factored and solved together with the distances
    // copy_stride[s] (s < ns1).  A single problem has ncopy = 1, ns1 = ns.
    int32_t ncopy = 1, ns1 = 0;
    std::vector<CopyStride> copy_stride;
    // chains (see select_chains in plan.cpp): components of small fronts on the narrow upper levels
    // of deep trees, one workgroup each; levels >= chain_L0 list their chain fronts last, and the
    // level kernels stop at ent_lvl_mid / zseg_lvl_mid
    int32_t chain_L0 = 0, chain_maxr = 0;
    std::vector<int8_t> in_chain;
    std::vector<int32_t> chain_comp_ptr;  // components -> groups
    std::vector<int32_t> chain_grp_ptr;   // groups (one level of a component) -> fronts
    std::vector<int32_t> chain_sn;
    std::vector<int64_t> ent_lvl_mid, zseg_lvl_mid;
    std::vector<int64_t> ent_front;       // 2 per front: its range of assembly entries
};

struct Device {
    // problem data (original ordering)
    DBuf<double> kval;          // unregularized K upper values (nnz_K)
    DBuf<int64_t> blk33;        // positions of (3,3) entries in kval
    DBuf<int64_t> blk_off;      // per SOC: offset of its entries in blk33 (after the orthant)
    DBuf<int32_t> soc_off;      // nsoc + 1 row offsets in z
    DBuf<int32_t> big_cones;    // indices of the SOCs with q >= QBIG (one wavefront each)
    DBuf<int32_t> big_chunk_cone;   // per BIG_CHUNK chunk of a big cone's block: position in big_cones
    DBuf<int64_t> big_chunk_start;  //   and first entry of the chunk within that cone's block
    DBuf<double> bigsc;         // 2 per big cone: z1'z1, z1's1 (derivative block)
    DBuf<int64_t> kr_ptr;       // full symmetric CSR of K without the (3,3) block
    DBuf<int32_t> kr_col;
    DBuf<double> kr_val;
    DBuf<double> c, b, h;
    // Ruiz equilibration (settings.ruiz_iters > 0): the caller's c, b, h (c, b, h above hold the scaled
    // ones), the scalings [D (n); E (p); F (m)] and, per KKT row, the factor that takes a residual
    // entry back to the caller's units (1 / (k D) for x rows, 1 / E for y rows, 1 / F for z rows)
    DBuf<double> craw, braw, hraw, rz_dsc, rz_rsc;
    DBuf<int64_t> Pp; DBuf<int32_t> Pi;   // P upper pattern (for dL/dP)
    DBuf<int64_t> Ap, Gp; DBuf<int32_t> Ai, Gi;   // A and G patterns (for dL/dA, dL/dG)
    DBuf<int64_t> posG;         // position of each G entry among the K values (G' g_s in the adjoint)
    DBuf<int32_t> perm, iperm;
    // plan
    DBuf<int32_t> sn_first, sn_rows, task_sn, task_col, ch_ptr, ch_list, lvl_small_sn;
    DBuf<int64_t> sn_rptr, fr_off, task_ptr, ctb_ptr, ctb_src, uv_off;
    DBuf<int8_t> reg_sign;
    DBuf<int64_t> ent_dst, ent_sptr, ent_src, zseg_off;   // numeric assembly map (see Plan)
    DBuf<int8_t> ent_reg;
    DBuf<int32_t> zseg_len;
    DBuf<int32_t> chain_comp_ptr, chain_grp_ptr, chain_sn;   // chains (Plan)
    DBuf<int64_t> ent_front;
    DBuf<double> front64;
    DBuf<float> front32;
    DBuf<double> uvec;          // update vectors of the triangular solves
    DBuf<double> vwork;         // per (front, row) task: gathered solve vector
    DBuf<int64_t> task0;
    DBuf<double> dinv64;        // inverses of the NB x NB diagonal blocks of large fronts
    DBuf<float> dinv32;
    DBuf<double> sinv64;        // inverses of the SB x SB diagonal blocks (and transposes)
    DBuf<float> sinv32;
    DBuf<double> w64;           // W_J blocks of the large fronts (solves only)
    DBuf<float> w32;
    DBuf<double> ubuf;          // max_r: X' v of every super-block in the backward large-front solve
    DBuf<double> vbuf;          // work vector of length max_r (large-front solves)
    DBuf<int32_t> col2sn;
    DBuf<int32_t> nreg;         // dynamic regularization counter
    // iterate and work vectors
    DBuf<double> x, y, s, z;
    DBuf<double> rx, ry, rz;    // residuals (rz excludes s)
    DBuf<double> kx;            // N: K_static * [x;y;z] parts
    DBuf<double> rhs, sol, res, corr, xp;   // N
    DBuf<double> dsa, ds, t, lam, w;        // m
    DBuf<double> wbar, beta;                // SOC scaling
    DBuf<double> scal;          // reduction scalars
    DBuf<double> scal_inst;     // residual scalars of each problem of a batch (NSCAL each)
    DBuf<double> partials;      // per-block reduction partials
    DBuf<int32_t> zcone;        // per z row: SOC index (-1 on the orthant)
    DBuf<double> alpha;         // step lengths of the last iteration (affine, combined)
    DBuf<unsigned long long> amin;          // step-length minima (ordered bits), 4 per problem of a batch
    DBuf<double> mu;            // complementarity measure of each problem of a batch, then its step gate
                                // (1 while it iterates, 0 once its own stopping test has passed)
    DBuf<int32_t> flag;         // count of non-finite entries (qg_update_vectors)
};

// Timing helper around HIP events on the handle's stream.
struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace qg

struct qg_handle {
    qg_settings st;
    hipStream_t stream = nullptr;
    // Side streams of the large-front factorization (default priority, non-blocking):
    // bulk = trailing updates beyond the next super-panel, prep = inverses and W blocks
    // for the solves; ordered against `stream` with the events below.
    hipStream_t bulk = nullptr, prep = nullptr;
    hipStream_t cap = nullptr;          // graph capture only (nothing runs on it)
    hipEvent_t ev_panel = nullptr, ev_bulk = nullptr, ev_prep = nullptr;
    hipEvent_t ev_sync = nullptr;       // host waits on the handle's stream (polled, see stream_wait)
    double *pin = nullptr;              // pinned host memory for small read-backs (PIN_DOUBLES doubles)
    // the factorization and the triangular solve (between the permutations) as HIP graphs, one per
    // factor precision (0 FP64, 1 FP32), captured at first use and replayed (settings.graphs)
    hipGraphExec_t g_factor[2] = {nullptr, nullptr}, g_solve[2] = {nullptr, nullptr};
    int last_hip = 0;
    int device = 0;
    // device memory of the handle: the caller's allocator (qg_setup), or hipMalloc when NULL
    qg_alloc_fn alloc = nullptr;
    qg_free_fn free_fn = nullptr;
    void *alloc_ctx = nullptr;
    bool alloc_refused = false;
    qg::ProblemPattern pp;
    qg::KktPattern kp;
    qg::Symbolic sym;                  // the analysis (supernodes, permutation)
    qg::Symbolic fronts;               // device fronts: the analysis with small-k children merged
    qg::Plan plan;
    qg::Device d;
    std::vector<double> kval_static;   // K upper values without (3,3) entries
    std::vector<double> hc, hb, hh;    // c, b, h on the host
    int64_t nnzK = 0;
    int64_t kr_nnz = 0;         // entries of the static full CSR of K (kr_*)
    int32_t n = 0, m = 0, p = 0, N = 0;
    int32_t ncopy = 1;                 // problems in the batch (qg_setup_batch), 1 for qg_setup
    int32_t n1 = 0, m1 = 0, p1 = 0, l1 = 0;   // sizes of one problem of the batch
    int32_t nbig = 0;                  // SOCs handled one wavefront per cone
    int32_t grp_q = 0;                 // > 0: every SOC has this many entries (<= 16): lane groups
    int ruiz = 0;                      // Ruiz passes (settings.ruiz_iters at setup; 0: no scaling)
    double ruiz_k = 1.0;               // objective scaling
    std::vector<double> ruiz_dsc;      // host copy of [D; E; F]
    int64_t nbigchunk = 0;             // workgroups of the big cones' block writes
    bool solved = false;               // a solve finished (x, s, y, z valid)
    bool final_factor = false;         // the derivative system is factored (FP64)
    int last_precision = -1;           // precision of the current factor
    int last_status = QG_UNSOLVED;
    double ms_setup = 0, ms_analyze = 0;
    int64_t small_lds_bytes = 0;
    std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, int>> prof_events;   // settings.profile
    double prof_flops[4] = {0.0, 0.0, 0.0, 0.0};
};

namespace qg {

// error plumbing
int hip_fail(qg_handle *h, hipError_t e);
#define QG_HIP(h, call)                                  \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return qg::hip_fail(h, e_); \
    } while (0)

void *dmem_alloc(qg_handle *h, size_t bytes);
// Replay exec on the handle's stream, capturing it first from enqueue() (which launches work on the
// handle's stream and on side streams joined to it by events) when it is not there yet.
int graph_replay(qg_handle *h, hipGraphExec_t &exec, int (*enqueue)(qg_handle *, void *), void *arg);
void drop_graphs(qg_handle *h);
void dmem_free(qg_handle *h, void *p);
template <typename T>
int dalloc(qg_handle *h, DBuf<T> &b, size_t n);
template <typename T>
int dupload(qg_handle *h, DBuf<T> &b, const std::vector<T> &v);
void dfree_all(qg_handle *h);

int group_fronts(const Symbolic &sym, Symbolic &fronts);
int build_plan(qg_handle *h);
int upload_static_values(qg_handle *h, bool vectors);
// Ruiz equilibration: scaled c, b, h from the caller's copies on the device (after a change of
// either), and the caller's x, s, y, z from the scaled iterate (qg_solve's outputs).
int launch_scale_vectors(qg_handle *h);
int launch_unscale_outputs(qg_handle *h, double *x, double *s, double *y, double *z);

// device phases (all enqueue on h->stream)
int launch_scaling(qg_handle *h, const double *s, const double *z, double *lam, int block);
int launch_factor(qg_handle *h, int precision);
int launch_solve(qg_handle *h, const double *rhs, double *x, int precision);
int refined_solve(qg_handle *h, const double *rhs, double *x, int precision, int ir_max, int *steps,
                  bool *ok = nullptr);
int launch_kkt_residual(qg_handle *h, const double *rhs, const double *x, double *res, double *norms);
int launch_max_step(qg_handle *h, const double *u, const double *du, int slot);
int launch_cone_op(qg_handle *h, int op, const double *u, const double *v, double *out);
int launch_corrector(qg_handle *h, const double *dsa, const double *dza, double sigma_mu,
                     const double *mu_dev, double *t);
int read_nreg(qg_handle *h, int *nreg);
// Pinned read-back slots (doubles): the residual scalars of each problem, then the refinement norms,
// then the dynamic-regularization count of the last factorization.
constexpr int PIN_DOUBLES = 512;
// Wait on the host for everything enqueued on the handle's stream so far, polling an event (a
// blocking wait sleeps and wakes up tens of microseconds late, once or more per Newton step).
int stream_wait(qg_handle *h);
// Copy the dynamic-regularization count of the last factorization to the pinned slot (read after the
// next wait), and read it.
int nreg_async(qg_handle *h);
int nreg_pinned(const qg_handle *h);
int factor_init_attributes(qg_handle *h);
void prof_collect(qg_handle *h, int64_t *launches, double *ms, double *flops);

int ipm_solve(qg_handle *h, double *x, double *s, double *y, double *z, qg_info *info);
int adjoint_backward(qg_handle *h, const double *g, const double *gy, const double *gz, const double *gs,
                     double *dc, double *dh, double *db, double *dP, double *dA, double *dG);

}  // namespace qg
