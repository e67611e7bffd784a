// Numeric LDL' of the KKT matrix (paper Sec. 2.2 "factor" phase), once per
// interior-point iteration, on the fixed pattern from the analysis.
//
// Multifrontal, level by level over the supernodal elimination tree:
//  * assemble_cols: one wavefront per front column; zero the column, scatter
//    the K entries that belong to it (+ static regularization on the
//    diagonal), then add every child's update column that maps onto it, in
//    child order (deterministic, no atomics);
//  * factor_small: fronts with r <= SMALL_R, one workgroup per front in LDS:
//    k right-looking pivot steps over the whole front, which leaves L in the
//    first k columns and the Schur complement (update) in the trailing block;
//  * large fronts: blocked right-looking steps of NB columns:
//      diag_block   (1 workgroup)  LDL' of the NB x NB diagonal block in LDS
//                                  and the inverse of its unit-lower factor;
//      panel_solve  (rows/64 WGs)  L21 = A21 L11^-T D^-1;
//      trail_update (lower tiles)  A22 -= L21 D L21' on MFMA 16x16x4 tiles.
// Dynamic regularization: pivot d with sign*d <= eps becomes sign*dyn.
#include "kernels.hpp"
#include "solver.hpp"

namespace qg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma16x16x4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16x16x4(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T> struct Acc4;
template <> struct Acc4<double> { typedef d4 type; };
template <> struct Acc4<float> { typedef f4 type; };

// Row of the 16 x 16 MFMA output held by lane group lk (= lane / 16) in
// accumulator register v: the f32 instruction keeps four consecutive rows
// per lane group, the f64 instruction interleaves them (rows lk, lk+4, ...).
// Both checked on gfx950 against a product with known entries.
template <typename T> __device__ inline int mfma_out_row(int lk, int v);
template <> __device__ inline int mfma_out_row<float>(int lk, int v) { return 4 * lk + v; }
template <> __device__ inline int mfma_out_row<double>(int lk, int v) { return lk + 4 * v; }

// ---------------------------------------------------------------------------
// assembly: one 64-thread workgroup per (front, column) task
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) assemble_cols(
    int64_t t0, const int32_t *__restrict__ task_sn, const int32_t *__restrict__ task_col,
    const int32_t *__restrict__ sn_first, const int64_t *__restrict__ sn_rptr,
    const int64_t *__restrict__ fr_off, T *__restrict__ front,
    const int64_t *__restrict__ asm_ptr, const int64_t *__restrict__ asm_src,
    const int32_t *__restrict__ asm_row, const double *__restrict__ kval,
    const int8_t *__restrict__ kind, double delta,
    const int64_t *__restrict__ ctb_ptr, const int32_t *__restrict__ ctb_child,
    const int32_t *__restrict__ ctb_col, const int64_t *__restrict__ rel_ptr,
    const int32_t *__restrict__ rel) {
    const int64_t task = t0 + blockIdx.x;
    const int lane = threadIdx.x;
    const int32_t s = task_sn[task];
    const int32_t j = task_col[task];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - sn_first[s];
    T *col = front + fr_off[s] + (int64_t)j * r;
    for (int32_t i = j + lane; i < r; i += 64) col[i] = T(0);
    __syncthreads();
    for (int64_t t = asm_ptr[task] + lane; t < asm_ptr[task + 1]; t += 64)
        col[asm_row[t]] = (T)kval[asm_src[t]];
    __syncthreads();
    if (lane == 0 && j < k) col[j] = (T)((double)col[j] + static_reg(kind[sn_first[s] + j], delta));
    for (int64_t u = ctb_ptr[task]; u < ctb_ptr[task + 1]; ++u) {
        __syncthreads();
        const int32_t c = ctb_child[u];
        const int32_t jc = ctb_col[u];
        const int32_t rc = (int32_t)(sn_rptr[c + 1] - sn_rptr[c]);
        const int32_t kc = sn_first[c + 1] - sn_first[c];
        const int32_t mc = rc - kc;
        const T *ucol = front + fr_off[c] + (int64_t)(kc + jc) * rc + kc;   // update block column jc
        const int32_t *rl = rel + rel_ptr[c];
        for (int32_t i = jc + lane; i < mc; i += 64) col[rl[i]] += ucol[i];
    }
}

// ---------------------------------------------------------------------------
// pivot with dynamic regularization
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline T regularize(T d, int8_t kind_j, double eps, double dyn, int32_t *nreg) {
    const double sg = pivot_sign(kind_j);
    if (!(sg * (double)d > eps)) {   // also catches NaN
        atomicAdd(nreg, 1);
        return (T)(sg * dyn);
    }
    return d;
}

// ---------------------------------------------------------------------------
// small fronts: one 256-thread workgroup per front, front in LDS
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) factor_small(
    const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, T *__restrict__ front,
    const int8_t *__restrict__ kind, double eps, double dyn, int32_t *nreg) {
    __shared__ T F[SMALL_R * SMALL_R];
    __shared__ T dsh;
    const int32_t s = sn_list[blockIdx.x];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - sn_first[s];
    T *G = front + fr_off[s];
    const int tid = threadIdx.x;
    for (int32_t idx = tid; idx < r * r; idx += 256) {
        const int32_t i = idx % r, c = idx / r;
        F[idx] = (i >= c) ? G[idx] : T(0);
    }
    __syncthreads();
    for (int32_t jj = 0; jj < k; ++jj) {
        if (tid == 0) {
            T d = regularize(F[jj * r + jj], kind[sn_first[s] + jj], eps, dyn, nreg);
            F[jj * r + jj] = d;
            dsh = d;
        }
        __syncthreads();
        const T d = dsh;
        const int32_t R = r - jj - 1;
        for (int32_t idx = tid; idx < R * R; idx += 256) {
            const int32_t i = jj + 1 + idx % R, c = jj + 1 + idx / R;
            if (i >= c) F[c * r + i] -= F[jj * r + i] * F[jj * r + c] / d;
        }
        __syncthreads();
        for (int32_t i = jj + 1 + tid; i < r; i += 256) F[jj * r + i] /= d;
        __syncthreads();
    }
    for (int32_t idx = tid; idx < r * r; idx += 256) {
        const int32_t i = idx % r, c = idx / r;
        if (i >= c) G[idx] = F[idx];
    }
}

// ---------------------------------------------------------------------------
// large fronts
// ---------------------------------------------------------------------------
// LDL' of the b x b diagonal block at (j0, j0) of the front F (ld r), in
// place; the inverse of the unit lower factor goes to Xg (ld NB).
template <typename T>
__global__ void __launch_bounds__(256) diag_block(T *__restrict__ F, int32_t r, int32_t j0, int32_t b,
                                                  const int8_t *__restrict__ kind_cols, double eps,
                                                  double dyn, int32_t *nreg, T *__restrict__ Xg) {
    __shared__ T Ls[NB * NB];     // Ls[c * NB + i] = L(i, c)
    __shared__ T tmp[NB];
    __shared__ T dsh;
    const int tid = threadIdx.x;
    for (int32_t idx = tid; idx < b * b; idx += 256) {
        const int32_t i = idx % b, c = idx / b;
        Ls[c * NB + i] = (i >= c) ? F[(int64_t)(j0 + c) * r + j0 + i] : T(0);
    }
    __syncthreads();
    for (int32_t jj = 0; jj < b; ++jj) {
        if (tid == 0) {
            T d = regularize(Ls[jj * NB + jj], kind_cols[j0 + jj], eps, dyn, nreg);
            Ls[jj * NB + jj] = d;
            dsh = d;
        }
        __syncthreads();
        const T d = dsh;
        const int32_t R = b - jj - 1;
        for (int32_t idx = tid; idx < R * R; idx += 256) {
            const int32_t i = jj + 1 + idx % R, c = jj + 1 + idx / R;
            if (i >= c) Ls[c * NB + i] -= Ls[jj * NB + i] * Ls[jj * NB + c] / d;
        }
        __syncthreads();
        for (int32_t i = jj + 1 + tid; i < b; i += 256) Ls[jj * NB + i] /= d;
        __syncthreads();
    }
    for (int32_t idx = tid; idx < b * b; idx += 256) {
        const int32_t i = idx % b, c = idx / b;
        if (i >= c) F[(int64_t)(j0 + c) * r + j0 + i] = Ls[c * NB + i];
    }
    __syncthreads();
    // in-place inverse of the unit lower factor, last column first:
    // X(j+1:, j) = -X(j+1:, j+1:) L(j+1:, j)
    for (int32_t j = b - 2; j >= 0; --j) {
        if (tid < b) tmp[tid] = (tid > j) ? Ls[j * NB + tid] : T(0);
        __syncthreads();
        if (tid > j && tid < b) {
            T acc = tmp[tid];                       // X(i,i) = 1
            for (int32_t t = j + 1; t < tid; ++t) acc += Ls[t * NB + tid] * tmp[t];
            Ls[j * NB + tid] = -acc;
        }
        __syncthreads();
    }
    for (int32_t idx = tid; idx < b * b; idx += 256) {
        const int32_t i = idx % b, c = idx / b;
        Xg[c * NB + i] = (i > c) ? Ls[c * NB + i] : (i == c ? T(1) : T(0));
    }
}

// L21 = A21 X' D^-1 for 64 rows per workgroup (rows j0+b .. r-1).
template <typename T>
__global__ void __launch_bounds__(256) panel_solve(T *__restrict__ F, int32_t r, int32_t j0, int32_t b,
                                                   const T *__restrict__ Xg) {
    __shared__ T Xs[NB * NB];
    __shared__ T Ds[NB];
    const int tid = threadIdx.x;
    for (int32_t idx = tid; idx < NB * NB; idx += 256) Xs[idx] = Xg[idx];
    if (tid < b) Ds[tid] = F[(int64_t)(j0 + tid) * r + j0 + tid];
    __syncthreads();
    const int32_t row = j0 + b + blockIdx.x * 64 + (tid & 63);
    const int32_t cg = tid >> 6;                 // column group 0..3
    const bool active = row < r;
    T out[NB / 4];
#pragma unroll
    for (int u = 0; u < NB / 4; ++u) out[u] = T(0);
    for (int32_t t = 0; t < b && active; ++t) {
        const T a = F[(int64_t)(j0 + t) * r + row];
#pragma unroll
        for (int u = 0; u < NB / 4; ++u) {
            const int32_t c = cg + 4 * u;        // X(c, t) nonzero for t <= c
            out[u] += a * Xs[t * NB + c];
        }
    }
    __syncthreads();   // every thread of this row has read A21 before it is overwritten
#pragma unroll
    for (int u = 0; u < NB / 4; ++u) {
        const int32_t c = cg + 4 * u;
        if (active && c < b) F[(int64_t)(j0 + c) * r + row] = out[u] / Ds[c];
    }
}

// A22 -= L21 D L21' over the lower 64 x 64 tiles of the trailing block
// starting at j1 = j0 + b.  Four wavefronts per tile, 2 x 2 MFMA 16x16
// blocks each; the product is formed transposed so that each lane's four
// accumulators run along a column of the column-major front.
template <typename T>
__global__ void __launch_bounds__(256) trail_update(T *__restrict__ F, int32_t r, int32_t j0, int32_t b) {
    __shared__ T As[NB * 64];    // As[kk * 64 + i] = L(j1 + 64 ti + i, j0 + kk)
    __shared__ T Bs[NB * 64];    // Bs[kk * 64 + j] = L(j1 + 64 tj + j, j0 + kk) * D(kk)
    const int32_t j1 = j0 + b;
    const int64_t x = blockIdx.x;
    int32_t ti = (int32_t)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while ((int64_t)ti * (ti + 1) / 2 > x) --ti;
    while ((int64_t)(ti + 1) * (ti + 2) / 2 <= x) ++ti;
    const int32_t tj = (int32_t)(x - (int64_t)ti * (ti + 1) / 2);
    const int32_t r0 = j1 + 64 * ti, c0 = j1 + 64 * tj;
    const int tid = threadIdx.x;
    {
        const int32_t i = tid & 63;
        for (int32_t kk = tid >> 6; kk < NB; kk += 4) {
            T av = T(0), bv = T(0);
            if (kk < b) {
                const T *colp = F + (int64_t)(j0 + kk) * r;
                if (r0 + i < r) av = colp[r0 + i];
                if (c0 + i < r) bv = colp[c0 + i] * colp[j0 + kk];
            }
            As[kk * 64 + i] = av;
            Bs[kk * 64 + i] = bv;
        }
    }
    __syncthreads();
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    typedef typename Acc4<T>::type V;
    V acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = V{0, 0, 0, 0};
    const int lr = lane & 15, lk = lane >> 4;
    for (int32_t kk = 0; kk < b; kk += 4) {
        const int32_t kq = kk + lk;
        T a_op[2], b_op[2];
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) a_op[bj] = Bs[kq * 64 + wc + 16 * bj + lr];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) b_op[bi] = As[kq * 64 + wr + 16 * bi + lr];
#pragma unroll
        for (int bi = 0; bi < 2; ++bi)
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma16x16x4(a_op[bj], b_op[bi], acc[bi][bj]);
    }
    // lane holds D(mfma_out_row(lk, v), lr) = C(row = wr + 16 bi + lr, col = wc + 16 bj + mfma_out_row(lk, v))
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t row = r0 + wr + 16 * bi + lr;
                const int32_t col = c0 + wc + 16 * bj + mfma_out_row<T>(lk, v);
                if (row < r && col < r && row >= col) F[(int64_t)col * r + row] -= acc[bi][bj][v];
            }
}

// Per-launch HIP events of the trailing-update kernel (settings.profile).
static void prof_begin(qg_handle *h, hipEvent_t *e0, hipEvent_t *e1) {
    if (hipEventCreate(e0) != hipSuccess || hipEventCreate(e1) != hipSuccess) { *e0 = *e1 = nullptr; return; }
    (void)hipEventRecord(*e0, h->stream);
}
static void prof_end(qg_handle *h, hipEvent_t e0, hipEvent_t e1, double flops, int fp32) {
    if (!e0) return;
    (void)hipEventRecord(e1, h->stream);
    h->prof_events.push_back({{e0, e1}, fp32});
    h->prof_flops[fp32] += flops;
}

void prof_collect(qg_handle *h, int64_t *launches, double *ms, double *flops) {
    for (int q = 0; q < 2; ++q) { launches[q] = 0; ms[q] = 0.0; flops[q] = h->prof_flops[q]; }
    for (auto &pr : h->prof_events) {
        float t = 0.f;
        if (hipEventSynchronize(pr.first.second) == hipSuccess &&
            hipEventElapsedTime(&t, pr.first.first, pr.first.second) == hipSuccess)
            ms[pr.second] += t;
        launches[pr.second] += 1;
        (void)hipEventDestroy(pr.first.first);
        (void)hipEventDestroy(pr.first.second);
    }
    h->prof_events.clear();
    h->prof_flops[0] = h->prof_flops[1] = 0.0;
}

template <typename T>
static int factor_large(qg_handle *h, int32_t s, T *front, T *dinv, const RegParams &rp) {
    const Plan &pl = h->plan;
    const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
    const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
    T *F = front + pl.fr_off[s];
    const int8_t *kinds = h->d.reg_sign.p + pl.sn_first[s];
    for (int32_t j0 = 0; j0 < k; j0 += NB) {
        const int32_t b = std::min(NB, k - j0);
        T *ws = dinv + pl.dinv_off[s] + (int64_t)(j0 / NB) * NB * NB;
        diag_block<T><<<1, 256, 0, h->stream>>>(F, r, j0, b, kinds, rp.eps, rp.dyn, h->d.nreg.p, ws);
        const int32_t mb = r - j0 - b;
        if (mb > 0) {
            panel_solve<T><<<(mb + 63) / 64, 256, 0, h->stream>>>(F, r, j0, b, ws);
            const int64_t T_ = (mb + 63) / 64;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (h->st.profile) prof_begin(h, &e0, &e1);
            trail_update<T><<<(unsigned)(T_ * (T_ + 1) / 2), 256, 0, h->stream>>>(F, r, j0, b);
            if (h->st.profile) prof_end(h, e0, e1, (double)b * (double)mb * (double)(mb + 1), sizeof(T) == 4);
        }
    }
    return QG_OK;
}

template <typename T>
static int factor_all(qg_handle *h, T *front, T *dinv, const RegParams &rp) {
    const Plan &pl = h->plan;
    Device &d = h->d;
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        const int64_t t0 = pl.task_ptr[L], nt = pl.task_ptr[L + 1] - t0;
        if (nt > 0)
            assemble_cols<T><<<(unsigned)nt, 64, 0, h->stream>>>(
                t0, d.task_sn.p, d.task_col.p, d.sn_first.p, d.sn_rptr.p, d.fr_off.p, front,
                d.asm_ptr.p, d.asm_src.p, d.asm_row.p, d.kval.p, d.reg_sign.p, rp.delta, d.ctb_ptr.p,
                d.ctb_child.p, d.ctb_col.p, d.rel_ptr.p, d.rel.p);
        const int32_t s0 = pl.lvl_small_ptr[L], s1 = pl.lvl_small_ptr[L + 1];
        if (s1 > s0)
            factor_small<T><<<s1 - s0, 256, 0, h->stream>>>(d.lvl_small_sn.p + s0, d.sn_first.p,
                                                             d.sn_rptr.p, d.fr_off.p, front,
                                                             d.reg_sign.p, rp.eps, rp.dyn, d.nreg.p);
        for (int32_t u = pl.lvl_large_ptr[L]; u < pl.lvl_large_ptr[L + 1]; ++u)
            factor_large<T>(h, pl.lvl_large_sn[u], front, dinv, rp);
    }
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

__global__ void zero_int(int32_t *p) { *p = 0; }

int launch_factor(qg_handle *h, int precision) {
    const qg_settings &st = h->st;
    zero_int<<<1, 1, 0, h->stream>>>(h->d.nreg.p);
    int rc;
    if (precision == QG_FP32_IR) {
        RegParams rp{st.static_reg32, st.dyn_eps32, st.dyn_delta32};
        rc = factor_all<float>(h, h->d.front32.p, h->d.dinv32.p, rp);
    } else {
        RegParams rp{st.static_reg, st.dyn_eps, st.dyn_delta};
        rc = factor_all<double>(h, h->d.front64.p, h->d.dinv64.p, rp);
    }
    h->last_precision = precision;
    return rc;
}

int read_nreg(qg_handle *h, int *nreg) {
    int32_t v = 0;
    QG_HIP(h, hipMemcpyAsync(&v, h->d.nreg.p, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
    QG_HIP(h, hipStreamSynchronize(h->stream));
    if (nreg) *nreg = v;
    return QG_OK;
}

}  // namespace qg
