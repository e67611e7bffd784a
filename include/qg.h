/*
 * qg.h -- C ABI of the MI355X Newton-step library for quadratic-objective
 * second-order cone programs (the problem class of QOCO-GPU, arXiv 2603.29197).
 *
 * Problem (paper Sec. 1, eq. 1):
 *     minimize 1/2 x'Px + c'x   s.t.  h - Gx in K,  Ax = b,
 * x in R^n, P (n x n, positive semidefinite, given as its upper triangle,
 * as the paper's size count does in Sec. 3), A (p x n), G (m x n).
 * K = C_1 x ... x C_K: the nonnegative orthant of dimension l (rows 0..l-1
 * of G) followed by nsoc second-order cones of dimensions q[0..nsoc-1] in
 * row order (the argument order of the paper's setup call, Sec. 2.1,
 * Listing 1); l + sum(q) must equal m.
 *
 * Each interior-point iteration factors the KKT matrix of eq. (2),
 *     [ P  A'  G'    ]
 *     [ A  0   0     ]
 *     [ G  0  -W'W   ]
 * once (LDL', after a one-time analysis of its sparsity pattern, Sec. 2.2)
 * and solves with the factor twice; the cone operations (Nesterov-Todd
 * scaling, Jordan products, maximum step) run per cone in parallel
 * (Sec. 2.1, 2.3).  All data lives on the device between setup and the
 * return of the solution (Sec. 2.3).
 *
 * Conventions for every entry point:
 *  - indices are 0-based; sparse matrices are CSC with strictly increasing
 *    row indices inside each column (no duplicates);
 *  - pointers documented as "host" are read (or written) before the call
 *    returns and are never retained; "device" pointers are HIP device
 *    memory owned by the caller (e.g. float64 torch tensors);
 *  - all device work is ordered on the stream given to qg_setup, and every
 *    call returns after the work it enqueued has completed;
 *  - a handle is not thread-safe; distinct handles are independent;
 *  - functions return QG_OK (0) or a negative QG_ERR_* code; the solver
 *    outcome is not an error and is reported in qg_info.status.
 */
#ifndef QG_H
#define QG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qg_int;
typedef int64_t qg_nnz;

/* return codes */
#define QG_OK 0
#define QG_ERR_ARG (-1)        /* NULL pointer, bad dimension, l + sum(q) != m, q[k] < 1 */
#define QG_ERR_PATTERN (-2)    /* unsorted/duplicate/out-of-range indices, P not upper, changed nnz */
#define QG_ERR_NONFINITE (-3)  /* NaN or Inf in the data */
#define QG_ERR_OOM (-4)        /* device or host allocation failed */
#define QG_ERR_HIP (-5)        /* a HIP call failed (code kept in the handle) */
#define QG_ERR_STATE (-6)      /* call out of order (e.g. backward before a solve) */
#define QG_ERR_DEVICE (-7)     /* no usable gfx950 device */
#define QG_ERR_SIZE (-8)       /* input larger than a fixed capacity (qg_max_step_noalloc; at setup,
                                  a front of more than 8388607 rows) */

/* qg_info.status */
#define QG_UNSOLVED 0
#define QG_SOLVED 1
#define QG_SOLVED_INACCURATE 2
#define QG_MAX_ITER (-1)
#define QG_NUMERICAL_ERROR (-2)

/* qg_settings.precision */
#define QG_FP64 0     /* every factor in FP64 */
#define QG_FP32_IR 1  /* FP32 factors + FP64 refinement while gap >= switch_gap, then FP64 */

/* qg_settings.ordering: the fill-reducing order of the analysis (paper Sec. 2.2 leaves the
 * reordering to its sparse solver) */
#define QG_ORDER_MD 0  /* minimum degree with the approximate external degree */
#define QG_ORDER_ND 1  /* nested dissection by breadth-first level structures, minimum degree on
                          pieces of at most 256 nodes: shallow elimination trees for banded and
                          grid-like patterns (long chains of small fronts under minimum degree) */

typedef struct {
    qg_int nrow, ncol;
    const qg_nnz *colptr;   /* host, ncol + 1 */
    const qg_int *rowind;   /* host, colptr[ncol] */
    const double *val;      /* host, colptr[ncol] */
} qg_csc;

typedef struct {
    double eps_abs, eps_rel;   /* stopping tolerances (default 1e-8) */
    double eps_inacc;          /* tolerance for SOLVED_INACCURATE at max_iter (1e-5) */
    int max_iter;              /* 100 */
    int precision;             /* QG_FP64 or QG_FP32_IR */
    double switch_gap;         /* FP32 factors while the scaled gap >= switch_gap (1e-6) */
    double static_reg;         /* +delta on the (1,1), -delta on the (2,2) diagonal, FP64 factors (1e-8) */
    double dyn_eps, dyn_delta; /* pivot d with sign*d <= dyn_eps becomes sign*dyn_delta (1e-13, 1e-7) */
    double static_reg32, dyn_eps32, dyn_delta32;  /* the same for FP32 factors (1e-4, 1e-8, 1e-4) */
    int ir_max;                /* refinement steps per solve with an FP64 factor (3) */
    int ir_max32;              /* ... with an FP32 factor (10) */
    double ir_tol;             /* stop when |r - K x|_inf <= ir_tol (1 + |r|_inf) (1e-12) */
    double step_frac;          /* fraction of the maximum step (0.99) */
    int differentiable;        /* 1: factor the derivative system after convergence (qg_backward) */
    int verbose;               /* 1: one line per iteration on stderr */
    int profile;               /* 1: time every launch of the trailing-update kernel (qg_info.kern_*) */
    int chains;                /* 1: the narrow upper levels of deep elimination trees are factored and
                                  solved by one workgroup per tree instead of one launch per level (1);
                                  read by qg_setup only, the arithmetic is the same either way */
    double fp32_min_flops;     /* QG_FP32_IR: FP32 factors only when the fronts factored on the matrix
                                  cores (more than 128 rows) take at least this many flops per
                                  factorization (1e10); below it the factorization is latency-bound,
                                  FP32 saves nothing and its refinement corrections cost extra solves, so
                                  every factor is FP64 (qg_info.switch_iter = 0) */
    int ordering;              /* QG_ORDER_MD (default) or QG_ORDER_ND; read by qg_setup only */
    int cone_lanes;            /* 1: when every second-order cone of a single problem has the same
                                  2 <= q <= 16 entries, NT scaling and the (3,3) block run one lane per
                                  cone entry (lane groups of 2, 4, 8 or 16); 0: one thread per cone (1) */
    int tiny_groups;           /* 1: elimination-tree levels with at least 2048 fronts of at most 16 rows
                                  factor and solve those fronts 16 lanes per front; 0: one workgroup or
                                  wavefront per front (1); read by qg_setup only, same arithmetic */
    int graphs;                /* 1: the triangular solves, and the factorization when no front has more
                                  than 1024 rows (no bulk trailing updates on a side stream), are captured
                                  once per factor precision as HIP graphs and replayed (the factorization
                                  not with profile = 1); 0: launched kernel by kernel (1); same arithmetic */
    int ruiz_iters;            /* 1..QG_RUIZ_MAX: Ruiz equilibration of the data with this many passes;
                                  0: none (0).  Columns of [P A' G'; A; G] and rows of A and G are divided
                                  by the square roots of their largest magnitudes (one factor per
                                  second-order cone), the objective by max(1, |D c|_inf).  The
                                  interior-point method runs on the scaled problem; the stopping test,
                                  qg_info and qg_solve's outputs are in the caller's units, while the
                                  step-level calls see the scaled KKT matrix.  Read by qg_setup only (the
                                  scalings are formed again by qg_update with new matrix values); not with
                                  qg_setup_batch or differentiable = 1 (QG_ERR_ARG) */
} qg_settings;

#define QG_STEP_MS_MAX 256
#define QG_RUIZ_MAX 100

typedef struct {
    int status;                /* QG_SOLVED, ... */
    int iters;                 /* Newton steps taken */
    int switch_iter;           /* first iteration with an FP64 factor (-1: none) */
    int ir_steps;              /* refinement steps over the whole solve */
    int nreg;                  /* dynamic-regularization events over the whole solve */
    int nfactor, nsolve;       /* factorizations (incl. the initial one), solves (excl. refinement) */
    double pobj, dobj, pres, dres, gap;
    double ms_setup, ms_analyze;             /* qg_setup wall time and its analysis part */
    double ms_solve;                         /* qg_solve wall time */
    double ms_factor, ms_trisolve, ms_cone;  /* summed device times (HIP events) */
    double ms_step_median;                   /* median Newton-step time over all iterations */
    double ms_step_median_fp32;              /* ... over iterations with an FP32 factor (0 if none) */
    double ms_step_median_fp64;              /* ... over iterations with an FP64 factor (0 if none) */
    int64_t nnz_L;                           /* entries of L incl. diagonal (exact symbolic count) */
    double factor_flops;                     /* sum_j (c_j - 1)^2 + 3 (c_j - 1), c_j column counts */
    /* with settings.profile: the trailing-update kernel of large fronts (MFMA), HIP events per
     * launch; index 0 = FP64 launches, 1 = FP32 launches on 64 x 64 tiles, 2 and 3 the same
     * on 128 x 128 tiles */
    int64_t kern_launches[4];
    double kern_ms[4];                       /* summed launch durations */
    double kern_flops[4];                    /* algorithmic flops: 2 b (C M - C (C - 1) / 2) per launch
                                                (rank b, M rows by C columns of the lower part) */
    double ms_step_p90;                      /* 90th percentile of the Newton-step times */
    int64_t ntrisolve[2];                    /* triangular solves incl. refinement corrections:
                                                [0] with an FP64 factor, [1] with an FP32 factor */
    int64_t nresidual;                       /* refinement residuals r - K x (FP64, unregularized K) */
    int32_t nstep_ms;                        /* entries of step_ms: min(iters, QG_STEP_MS_MAX) */
    int32_t step_fp32[QG_STEP_MS_MAX];       /* 1 where that step's factor was FP32, 0 for FP64 */
    double step_ms[QG_STEP_MS_MAX];          /* Newton-step times of the first iterations (HIP events) */
} qg_info;

/* Integer pattern of the analysis; pointers stay valid until the object
 * that produced them is destroyed. */
typedef struct {
    qg_int N;                  /* n + p + m */
    qg_int nsuper_fund, nsuper;
    const qg_int *perm;        /* N: perm[k] = original KKT index of pivot k */
    const qg_int *iperm;       /* N */
    const qg_int *parent;      /* N: elimination tree of the permuted matrix, -1 for roots */
    const int64_t *colcount;   /* N: entries of each column of L incl. the diagonal */
    const qg_int *super_fund;  /* nsuper_fund + 1: fundamental supernode first columns, then N */
    const qg_int *super_ptr;   /* nsuper + 1: relaxed supernode first columns, then N */
    const qg_nnz *rows_ptr;    /* nsuper + 1 */
    const qg_int *rows;        /* rows_ptr[nsuper]: sorted row list of each relaxed supernode */
    /* Fronts the device factors on: the relaxed supernodes, with each child of at most 16
     * columns whose front would exceed 128 rows merged into its parent's front as leading
     * pivots.  Numbered in the front order: column k of the fronts is original KKT index
     * front_perm[k], a reordering of the elimination tree that keeps every column after its
     * descendants (so L is the same matrix with renamed rows and columns). */
    qg_int nfront;
    const qg_int *front_perm;      /* N */
    const qg_int *front_ptr;       /* nfront + 1: first column of each front, then N */
    const qg_nnz *front_rows_ptr;  /* nfront + 1 */
    const qg_int *front_rows;      /* sorted rows of each front (front numbering) */
    /* Fronts on the narrow upper levels of deep elimination trees that one workgroup per tree
     * factors and solves (a handle's schedule; 0 from qg_symbolic_pattern or with chains off) */
    qg_int nchain_front;
} qg_pattern;

typedef struct qg_handle qg_handle;      /* device solver state */
typedef struct qg_symbolic qg_symbolic;  /* host-only analysis result */

/*
 * Device-memory hooks of qg_setup.  alloc(ctx, bytes) returns device memory
 * of at least `bytes` bytes, aligned to 256 bytes, usable on the handle's
 * stream, or NULL when it refuses (qg_setup then fails with QG_ERR_OOM after
 * returning everything it obtained through free).  free(ctx, ptr) gives back
 * one pointer alloc returned.  The hooks are called from the thread that
 * calls qg_setup, qg_update and qg_cleanup only, never from device work.
 */
typedef void *(*qg_alloc_fn)(void *ctx, size_t bytes);
typedef void (*qg_free_fn)(void *ctx, void *ptr);

/* Fill *s with the defaults listed in qg_settings. */
int qg_default_settings(qg_settings *s);

/*
 * Host-only analysis of the KKT pattern of eq. (2) (paper Sec. 2.2: the
 * reordering, permutation and symbolic factorization that run once per
 * sparsity pattern).  No device is touched.  Arguments as in qg_setup
 * (values are ignored; P, A, G may be NULL when they have no columns with
 * entries, i.e. are empty); ordering: QG_ORDER_MD or QG_ORDER_ND (anything
 * else is QG_ERR_ARG).  *out is owned by the caller: qg_symbolic_free.
 */
int qg_analyze(qg_symbolic **out, qg_int n, qg_int m, qg_int p,
               const qg_csc *P, const qg_csc *A, const qg_csc *G,
               qg_int l, qg_int nsoc, const qg_int *q, int ordering);
int qg_symbolic_pattern(const qg_symbolic *sym, qg_pattern *out);
void qg_symbolic_free(qg_symbolic *sym);

/*
 * Setup (paper Sec. 2.1 Listing 1, Sec. 2.3): validates and copies the
 * problem data (host pointers, read before return), runs the analysis and
 * uploads everything to the current HIP device.
 * P: n x n upper triangle incl. diagonal, or NULL for P = 0.  A: p x n, may
 * be NULL iff p == 0.  G: m x n, may be NULL iff m == 0.  q: nsoc cone
 * dimensions (host).  s: NULL for defaults.  hip_stream: the stream all
 * work is ordered on (NULL = the default stream).
 * alloc, free, alloc_ctx: where the handle's device memory comes from (all
 * of it: data, analysis maps, factor storage, work vectors); both NULL means
 * hipMalloc / hipFree, exactly one NULL is QG_ERR_ARG.  The handle owns what
 * it obtained and returns it through free in qg_cleanup.
 * Errors: QG_ERR_ARG, QG_ERR_PATTERN, QG_ERR_NONFINITE (checked before any
 * device call), QG_ERR_OOM (including a refusing alloc), QG_ERR_HIP,
 * QG_ERR_DEVICE.  On error *out is NULL and nothing is left allocated.
 */
int qg_setup(qg_handle **out, qg_int n, qg_int m, qg_int p,
             const qg_csc *P, const double *c,
             const qg_csc *A, const double *b,
             const qg_csc *G, const double *h,
             qg_int l, qg_int nsoc, const qg_int *q,
             const qg_settings *s, void *hip_stream,
             qg_alloc_fn alloc, qg_free_fn free, void *alloc_ctx);

/*
 * Replace values on the fixed pattern (host pointers, NULL = unchanged);
 * the analysis is reused (paper Sec. 3.2: the reordering can be reused
 * when only values change).  Pval/Aval/Gval follow the CSC entry order of
 * the matrices given to qg_setup.  Invalidates the stored final factor.
 */
int qg_update(qg_handle *h, const double *Pval, const double *c, const double *Aval,
              const double *b, const double *Gval, const double *hvec);

/*
 * The same for the vectors only, from device memory (e.g. float64 torch
 * tensors): c (n), b (p), hvec (m), NULL = unchanged.  Copied on the handle's
 * stream before return; no host round trip.  QG_ERR_NONFINITE (values left
 * unchanged) if any given entry is NaN or Inf.
 */
int qg_update_vectors(qg_handle *h, const double *c, const double *b, const double *hvec);

/* Replace the settings (the analysis is kept). */
int qg_set_settings(qg_handle *h, const qg_settings *s);

/*
 * Solve (paper Sec. 2.3: the whole interior-point loop runs on the device).
 * x (n), s (m), y (p), z (m): device output buffers.  info: host, may be
 * NULL.  With settings.differentiable the derivative system is factored
 * once after convergence and kept for qg_backward.
 */
int qg_solve(qg_handle *h, double *x, double *s, double *y, double *z, qg_info *info);

/*
 * Gradients of a loss L(x*) through the last solve by implicit
 * differentiation of the optimality conditions (the linearised KKT system,
 * eq. (2) at the final iterate): with u solving K_fin u = [dl_dx; 0; 0] on
 * the stored final factor (FP64 refinement): dl_dc = -u_x (n),
 * dl_db = u_y (p), dl_dh = u_z (m); on P's upper pattern
 * dl_dPval[t] = -(u_i x_j + u_j x_i) (i < j), -u_i x_i (i == j); on the
 * patterns of A and G (entries in the CSC order given to qg_setup)
 * dl_dAval[t] = -(y_i u_x,j + u_y,i x_j), dl_dGval[t] = -(z_i u_x,j + u_z,i x_j).
 * All device pointers; any output may be NULL.  Requires a previous
 * qg_solve with settings.differentiable = 1 whose status was QG_SOLVED or
 * QG_SOLVED_INACCURATE (QG_ERR_STATE otherwise).
 */
int qg_backward(qg_handle *h, const double *dl_dx, double *dl_dc, double *dl_dh,
                double *dl_db, double *dl_dPval, double *dl_dAval, double *dl_dGval);

/*
 * The same for a loss of the whole solution L(x*, y*, z*, s*): dl_dy (p),
 * dl_dz (m), dl_ds (m) are device pointers, NULL meaning zero.  With the
 * primal equality ds = dh - G dx - dG x, u solves
 * K_fin u = [dl_dx - G' dl_ds; dl_dy; dl_dz] and the formulas of qg_backward
 * hold with u_z + dl_ds in place of u_z in dl_dh and dl_dGval.  qg_backward
 * is this call with the three NULL.  Errors as for qg_backward.
 */
int qg_backward_full(qg_handle *h, const double *dl_dx, const double *dl_dy, const double *dl_dz,
                     const double *dl_ds, double *dl_dc, double *dl_dh, double *dl_db,
                     double *dl_dPval, double *dl_dAval, double *dl_dGval);

/*
 * Gradients of k losses through the same solve.  The k adjoint systems
 * share the one stored final factorization and run one after another on the
 * handle's stream.  Each input and output holds k blocks stored one after
 * another: dl_dx (k x n), dl_dy (k x p), dl_dz and dl_ds (k x m), dl_dc
 * (k x n), dl_dh (k x m), dl_db (k x p), dl_dPval (k x nnz(P)), dl_dAval
 * (k x nnz(A)), dl_dGval (k x nnz(G)).  Block j is what qg_backward_full
 * gives for the j-th blocks of the inputs.  NULL inputs mean zero and NULL
 * outputs are not written.  k = 0 does nothing.  k < 0 gives QG_ERR_ARG;
 * other errors are as for qg_backward.
 */
int qg_backward_batch(qg_handle *h, int32_t k, const double *dl_dx, const double *dl_dy,
                      const double *dl_dz, const double *dl_ds, double *dl_dc, double *dl_dh,
                      double *dl_db, double *dl_dPval, double *dl_dAval, double *dl_dGval);

/*
 * Batches of problems on one pattern (paper Sec. 3.2: the analysis is reused
 * when only the values change, for parametric problems).  The k problems
 * share n, m, p, the patterns of P, A, G and the cones; their values differ.
 * P, A, G: the shared pattern (as in qg_setup) whose val arrays hold k value
 * sets one after another (k x nnz, problem 0 first; P may be NULL for P = 0).
 * c (k x n), b (k x p), hvec (k x m): host, problem by problem.  The analysis
 * of one problem runs once and is replicated; the problems are solved
 * together as one separable problem (the block-diagonal KKT matrix of the
 * stack: every factorization and triangular solve of an iteration covers all
 * k, identical fronts of the k problems in one launch), so they share one
 * step length and one centering parameter per iteration, and the stopping
 * test of qg_solve applies to the stack (residual norms over all k problems,
 * the sum of the complementarity gaps against the summed objectives).  The
 * stack's optimum is the k problems' optima.  The handle takes qg_solve_batch
 * and the step-level calls; qg_solve, qg_update, qg_update_vectors and the
 * backward calls return QG_ERR_STATE on it.  Other arguments, ownership and
 * errors as for qg_setup; QG_ERR_ARG also for k < 1 or k (n + m + p) beyond
 * 32-bit indices.
 */
int qg_setup_batch(qg_handle **out, qg_int k, qg_int n, qg_int m, qg_int p,
                   const qg_csc *P, const double *c, const qg_csc *A, const double *b,
                   const qg_csc *G, const double *hvec, qg_int l, qg_int nsoc, const qg_int *q,
                   const qg_settings *s, void *hip_stream, qg_alloc_fn alloc, qg_free_fn free,
                   void *alloc_ctx);

/*
 * Solve the batch of qg_setup_batch.  x (k x n), s (k x m), y (k x p),
 * z (k x m): device outputs, problem by problem (any may be NULL).  info
 * (host, may be NULL) describes the stacked solve.
 */
int qg_solve_batch(qg_handle *h, double *x, double *s, double *y, double *z, qg_info *info);

/* Host copies of the analysis; valid until qg_cleanup. */
int qg_get_pattern(const qg_handle *h, qg_pattern *out);

/* Last error detail (HIP error code or 0). */
int qg_last_hip_error(const qg_handle *h);

/* Release every device buffer and the handle (NULL is a no-op). */
void qg_cleanup(qg_handle *h);

const char *qg_strerror(int code);

/* ---------------------------------------------------------------------
 * Step-level entry points.  Each runs one step of the Newton iteration on
 * the handle's device state so that it can be checked in isolation; the
 * solver uses the same kernels.  Vectors are device pointers of the
 * documented lengths.
 * --------------------------------------------------------------------- */

/*
 * Nesterov-Todd scaling of (s, z) (both strictly inside K; paper Sec. 2.1,
 * the scaling W of the (3,3) block of eq. 2, Sec. 2.2): stores W in
 * the handle, writes lambda = W z (m) if lam != NULL, and writes the (3,3)
 * block -W'W into the handle's KKT values.  block = 1 instead writes the
 * derivative-system block -sym(Arw(z)^-1 Arw(s)) (see qg_backward).
 */
int qg_step_scaling(qg_handle *h, const double *s, const double *z, double *lam, int block);

/* Host copy of the KKT values (upper CSC of eq. 2 in the original ordering,
 * unregularized), nnz_K entries; *nnz receives the count if kval == NULL. */
int qg_step_get_kkt(const qg_handle *h, double *kval, int64_t *nnz);

/* Numeric LDL' of the current KKT values (paper Sec. 2.2 "factor" phase)
 * in QG_FP64 or QG_FP32_IR (FP32) precision; *nreg (host, may be NULL)
 * receives the number of dynamic-regularization events. */
int qg_step_factor(qg_handle *h, int precision, int *nreg);

/*
 * Factor values on the analysis' column pattern: for the permuted
 * strictly-lower pattern (Lp: N+1, Li: Lp[N]; host) writes L's values
 * (Lx, host, Lp[N]) and D (host, N) from the last factor (FP32 factors are
 * widened).  Host-side extraction: meant for small test sizes.
 */
int qg_step_get_factor(const qg_handle *h, const int64_t *Lp, const int32_t *Li,
                       double *Lx, double *D);

/* Solve K x = rhs with the last factor (paper Sec. 2.2 "solve" phase);
 * refine = number of FP64 refinement steps against the unregularized K
 * (stopping early on the ir_tol test).  rhs, x: device, N.
 * *steps (host, may be NULL): refinement steps taken. */
int qg_step_solve(qg_handle *h, const double *rhs, double *x, int refine, int *steps);

/* alpha = sup{a >= 0 : u + a du in K} over all cones (+inf if unbounded),
 * written to *alpha (host). u strictly inside K. */
int qg_step_max_step(qg_handle *h, const double *u, const double *du, double *alpha);

/* Cone operation with the scaling of the last qg_step_scaling:
 * op 0: out = W u;  1: out = W^-1 u;  2: out = W'W u;  3: out = u o v;
 * op 4: out = u \ v (the w with u o w = v). */
int qg_step_cone_op(qg_handle *h, int op, const double *u, const double *v, double *out);

/* Corrector right-hand side (with the last scaling and its lambda):
 * t = W'(lambda \ d),  d = -lambda o lambda - (W^-T ds_a) o (W dz_a) + sigma_mu e. */
int qg_step_corrector(qg_handle *h, const double *ds_a, const double *dz_a, double sigma_mu,
                      double *t);

/* ---------------------------------------------------------------------
 * Entry point that allocates nothing.
 * --------------------------------------------------------------------- */

/* Capacity of qg_max_step_noalloc: at most this many cone units (l + nsoc). */
#define QG_NOALLOC_MAX_UNITS 4194304

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * maximum step of qg_step_max_step without a handle and without any
 * allocation.  alpha = sup{a >= 0 : u + a du in K} (+inf if unbounded) for
 * K = the orthant of dimension l times nsoc second-order cones.
 * soc_off: device, nsoc + 1 increasing row offsets of the cones in u
 * (soc_off[0] = l, cone k is rows soc_off[k] .. soc_off[k+1]-1, each of at
 * least one row); may be NULL when nsoc == 0.  u (strictly inside K), du:
 * device, soc_off[nsoc] entries (l when nsoc == 0).  alpha: host.
 * hip_stream: the stream the work is ordered on (NULL = default stream);
 * returns after it completed.
 * Its only device memory is a fixed array in the library, one per device
 * for the life of the process (QG_NOALLOC_MAX_UNITS / 256 + 1 doubles,
 * 128 KiB); every call on a device shares it, so calls that overlap on one
 * device (other host threads, or streams running concurrently) race and
 * must be serialized by the caller.  No state carries over between calls.
 * Errors: QG_ERR_ARG (negative sizes, NULL alpha, NULL soc_off with
 * nsoc > 0, NULL u or du with l + nsoc > 0), QG_ERR_SIZE
 * (l + nsoc > QG_NOALLOC_MAX_UNITS), QG_ERR_DEVICE, QG_ERR_HIP.
 */
int qg_max_step_noalloc(qg_int l, qg_int nsoc, const qg_int *soc_off, const double *u,
                        const double *du, double *alpha, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* QG_H */
