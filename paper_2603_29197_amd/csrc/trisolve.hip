// Triangular solves with the multifrontal factor (paper Sec. 2.2 "solve"
// phase, twice per interior-point iteration): x = Pi' L^-T D^-1 L^-1 Pi b.
//
// Forward (leaves to root): each supernode gathers its own right-hand side
// entries plus the update vectors of its children (through the same relative
// indices as the factorization, in child order: deterministic), solves with
// its unit-lower diagonal block, and leaves u_s = v_below - L21 y for its
// parent.  Backward (root to leaves): v = D^-1 y - L21' x_below, then the
// unit-upper solve with L11'.  Arithmetic is FP64; L is read in the factor's
// precision (FP32 factors are widened on load).
//
// Small fronts: one 128-thread workgroup per supernode, per level.  Large
// fronts: per SB-column super-block, one kernel applies the stored inverse of
// its unit-lower diagonal block (or its transpose) and a second one updates
// the rows below it (forward) or the columns before it (backward).
#include "kernels.hpp"
#include "solver.hpp"

namespace qg {

// ------------------------------- small -------------------------------------
// Gather of one level: RL lanes per (front s, row j) task:
// v = [j < k_s ? x_perm(first_s + j) : 0] + sum over the child columns that map
// onto row j of their update-vector entries (contribution lists of the
// assembly, with the position of each entry in the work vector precomputed).
// Lane l sums contributions l, l + RL, ...; the RL partial sums are combined
// by a fixed butterfly, so the result does not depend on scheduling.  Update
// vectors live in the children's own task slots (rows k_c .. r_c - 1).
__global__ void __launch_bounds__(256) fwd_gather_level(
    int64_t t0, int64_t nt, const int32_t *__restrict__ task_sn, const int32_t *__restrict__ task_col,
    const int32_t *__restrict__ sn_first, const int64_t *__restrict__ ctb_ptr,
    const int64_t *__restrict__ ctb_src, const double *__restrict__ xp, double *__restrict__ vwork) {
    const int sub = threadIdx.x & (RL - 1);
    const int64_t t = t0 + (int64_t)blockIdx.x * (256 / RL) + (threadIdx.x / RL);
    const bool live = t < t0 + nt;
    const int64_t tt = live ? t : t0;
    double v = 0.0;
    const int64_t u0 = ctb_ptr[tt], u1 = live ? ctb_ptr[tt + 1] : u0;
    for (int64_t u = u0 + sub; u < u1; u += 4 * RL) {     // four independent loads per lane in flight
        double a[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t uu = u + q * RL;
            const double x = vwork[ctb_src[uu < u1 ? uu : u]];   // u < u1: always a valid entry
            a[q] = uu < u1 ? x : 0.0;
        }
        v += (a[0] + a[1]) + (a[2] + a[3]);
    }
#pragma unroll
    for (int off = RL / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (live && sub == 0) {
        const int32_t s = task_sn[t], j = task_col[t];
        const int32_t f = sn_first[s], k = sn_first[s + 1] - f;
        vwork[t] = (j < k ? xp[f + j] : 0.0) + v;
    }
}

template <typename T>
__global__ void __launch_bounds__(SMALL_R) fwd_small(
    const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, const T *__restrict__ front,
    const int64_t *__restrict__ task0, double *__restrict__ vwork, double *__restrict__ xp) {
    __shared__ double v[SMALL_R];
    const int32_t s = sn_list[blockIdx.x];
    const int lane = threadIdx.x;
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    double *vs = vwork + task0[s];
    if (lane < r) v[lane] = vs[lane];
    __syncthreads();
    const T *F = front + fr_off[s];
    for (int32_t jj = 0; jj < k; ++jj) {
        const double yj = v[jj];
        if (lane > jj && lane < r) v[lane] -= (double)F[(int64_t)jj * r + lane] * yj;
        __syncthreads();
    }
    if (lane < k) xp[f + lane] = v[lane];
    else if (lane < r) vs[lane] = v[lane];
}

template <typename T>
__global__ void __launch_bounds__(SMALL_R) bwd_small(
    const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int32_t *__restrict__ sn_rows,
    const int64_t *__restrict__ fr_off, const T *__restrict__ front, double *__restrict__ xp) {
    __shared__ double g[SMALL_R];
    __shared__ double v[SMALL_R];
    const int32_t s = sn_list[blockIdx.x];
    const int lane = threadIdx.x;
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    const T *F = front + fr_off[s];
    if (lane >= k && lane < r) g[lane] = xp[sn_rows[sn_rptr[s] + lane]];
    __syncthreads();
    if (lane < k) {
        double acc = xp[f + lane] / (double)F[(int64_t)lane * r + lane];
        for (int32_t i = k; i < r; ++i) acc -= (double)F[(int64_t)lane * r + i] * g[i];
        v[lane] = acc;
    }
    __syncthreads();
    for (int32_t i = k - 1; i >= 0; --i) {
        const double xi = v[i];
        if (lane < i) v[lane] -= (double)F[(int64_t)lane * r + i] * xi;
        __syncthreads();
    }
    if (lane < k) xp[f + lane] = v[lane];
}

// ------------------------------- large -------------------------------------
// y = X v (forward, X the stored inverse of the unit-lower diagonal block of
// a super-block) or y = X' v (backward, the stored transpose), kb <= SB;
// the result goes to y and to the solution.  Workgroup g forms entries
// 64 g .. 64 g + 63; wavefront w sums over columns q in [64 w, 64 w + 64) of
// the column-major operand (lanes along rows: coalesced), then the four
// partial sums are added in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) sblock_apply(const T *__restrict__ X, int32_t ld, int32_t kb,
                                                    const double *__restrict__ vin, double *__restrict__ y,
                                                    double *__restrict__ xp_out, int32_t upper) {
    __shared__ double vs[SB];
    __shared__ double red[4][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t g = blockIdx.x;
    if (tid < kb) vs[tid] = vin[tid];
    __syncthreads();
    const int32_t t = g * 64 + lane;
    // lower operand: columns q <= t; upper operand: columns q >= t
    const bool live = upper ? (w >= g) : (w <= g);
    double acc = 0.0;
    if (live && t < kb) {
        const int32_t q1 = min(kb, 64 * w + 64);
        const T *Xr = X + t;
#pragma unroll 16
        for (int32_t q = 64 * w; q < q1; ++q) acc += (double)Xr[(int64_t)q * ld] * vs[q];
    }
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && t < kb) {
        const double v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        y[t] = v;
        xp_out[t] = v;
    }
}

// Forward update of the rows below a super-block: v[row] -= L(row, J0:J0+kb) y
// for 64 rows per workgroup; wavefront w takes columns [64 w, 64 w + 64)
// (lanes along rows: coalesced), fixed-order sum over wavefronts.
template <typename T>
__global__ void __launch_bounds__(256) sblock_rows(const T *__restrict__ F, int32_t r, int32_t J0, int32_t kb,
                                                   const double *__restrict__ y, double *__restrict__ vbuf) {
    __shared__ double ys[SB];
    __shared__ double red[4][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < kb) ys[tid] = y[tid];
    __syncthreads();
    const int32_t row = J0 + kb + blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (row < r) {
        const int32_t q1 = min(kb, 64 * w + 64);
        const T *p = F + (int64_t)J0 * r + row;
#pragma unroll 16
        for (int32_t q = 64 * w; q < q1; ++q) acc += (double)p[(int64_t)q * r] * ys[q];
    }
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && row < r) vbuf[row] -= ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// v[0:k] = D^-1 x_own - L21' g with g = x at the rows below (one column per
// wavefront, reduction over rows).
template <typename T>
__global__ void __launch_bounds__(256) bwd_init(int32_t s, const int32_t *__restrict__ sn_first,
                                                const int64_t *__restrict__ sn_rptr,
                                                const int32_t *__restrict__ sn_rows,
                                                const T *__restrict__ F, const double *__restrict__ xp,
                                                double *__restrict__ vbuf) {
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    const int32_t *rows = sn_rows + sn_rptr[s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int32_t c = blockIdx.x * 4 + wave;
    if (c >= k) return;
    double acc = 0.0;
    for (int32_t i = k + lane; i < r; i += 64) acc += (double)F[(int64_t)c * r + i] * xp[rows[i]];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) vbuf[c] = xp[f + c] / (double)F[(int64_t)c * r + c] - acc;
}

// Backward update of the columns before a super-block:
// v[c] -= L(J0:J0+kb, c)' y for 64 columns per workgroup, 16 per wavefront;
// lanes run along the contiguous rows of each column (coalesced), all loads
// of a wavefront are issued before its 16 shuffle reductions, and lanes
// 0..15 then update the 16 entries at once.
template <typename T>
__global__ void __launch_bounds__(256) sblock_cols(const T *__restrict__ F, int32_t r, int32_t J0, int32_t kb,
                                                   const double *__restrict__ y, double *__restrict__ vbuf) {
    __shared__ double ys[SB];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < kb) ys[tid] = y[tid];
    __syncthreads();
    const int32_t c0 = blockIdx.x * NB + w * 16;
    double part[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
        const int32_t c = c0 + cc;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < SB / 64; ++m) {
            const int32_t t = lane + 64 * m;
            const bool ok = c < J0 && t < kb;
            s += (double)ld_or0(F, (int64_t)c * r + J0 + t, ok) * ys[ok ? t : 0];
        }
        part[cc] = s;
    }
    // after the butterfly every lane holds the sum; lane cc updates column c0 + cc
    double mine = 0.0;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
        double s = part[cc];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        mine = lane == cc ? s : mine;
    }
    if (lane < 16 && c0 + lane < J0) vbuf[c0 + lane] -= mine;
}

// ------------------------------- driver ------------------------------------
template <typename T>
static int solve_perm(qg_handle *h, const T *front, const T *sinv) {
    const Plan &pl = h->plan;
    Device &d = h->d;
    double *xp = d.xp.p;
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        const int64_t t0 = pl.task_ptr[L], nt = pl.task_ptr[L + 1] - t0;
        if (nt > 0)
            fwd_gather_level<<<(unsigned)((nt + 256 / RL - 1) / (256 / RL)), 256, 0, h->stream>>>(
                t0, nt, d.task_sn.p, d.task_col.p, d.sn_first.p, d.ctb_ptr.p, d.ctb_src.p, xp, d.vwork.p);
        const int32_t s0 = pl.lvl_small_ptr[L], s1 = pl.lvl_small_ptr[L + 1];
        if (s1 > s0)
            fwd_small<T><<<s1 - s0, SMALL_R, 0, h->stream>>>(d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
                                                               d.fr_off.p, front, d.task0.p, d.vwork.p, xp);
        for (int32_t u = pl.lvl_large_ptr[L]; u < pl.lvl_large_ptr[L + 1]; ++u) {
            const int32_t s = pl.lvl_large_sn[u];
            const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
            const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
            const T *F = front + pl.fr_off[s];
            double *vs = d.vwork.p + pl.task0[s];
            for (int32_t J0 = 0; J0 < k; J0 += SB) {
                const int32_t kb = std::min(SB, k - J0);
                const int32_t ld = (kb + NB - 1) / NB * NB;
                const T *Xsb = sinv + pl.sinv_off[s] + (int64_t)(J0 / SB) * 2 * SB * SB;
                sblock_apply<T><<<(kb + 63) / 64, 256, 0, h->stream>>>(Xsb, ld, kb, vs + J0, d.ybuf.p,
                                                                     xp + pl.sn_first[s] + J0, 0);
                const int32_t rows = r - J0 - kb;
                if (rows > 0)
                    sblock_rows<T><<<(rows + 63) / 64, 256, 0, h->stream>>>(F, r, J0, kb, d.ybuf.p, vs);
            }
        }
    }
    for (int32_t L = pl.nlevels - 1; L >= 0; --L) {
        for (int32_t u = pl.lvl_large_ptr[L + 1] - 1; u >= pl.lvl_large_ptr[L]; --u) {
            const int32_t s = pl.lvl_large_sn[u];
            const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
            const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
            const T *F = front + pl.fr_off[s];
            bwd_init<T><<<(k + 3) / 4, 256, 0, h->stream>>>(s, d.sn_first.p, d.sn_rptr.p, d.sn_rows.p, F, xp,
                                                            d.vbuf.p);
            const int32_t nsb = (k + SB - 1) / SB;
            for (int32_t bi = nsb - 1; bi >= 0; --bi) {
                const int32_t J0 = bi * SB;
                const int32_t kb = std::min(SB, k - J0);
                const int32_t ld = (kb + NB - 1) / NB * NB;
                const T *XTsb = sinv + pl.sinv_off[s] + (int64_t)(J0 / SB) * 2 * SB * SB + (int64_t)ld * ld;
                sblock_apply<T><<<(kb + 63) / 64, 256, 0, h->stream>>>(XTsb, ld, kb, d.vbuf.p + J0, d.ybuf.p,
                                                                     xp + pl.sn_first[s] + J0, 1);
                if (J0 > 0)
                    sblock_cols<T><<<(J0 + NB - 1) / NB, 256, 0, h->stream>>>(F, r, J0, kb, d.ybuf.p, d.vbuf.p);
            }
        }
        const int32_t s0 = pl.lvl_small_ptr[L], s1 = pl.lvl_small_ptr[L + 1];
        if (s1 > s0)
            bwd_small<T><<<s1 - s0, SMALL_R, 0, h->stream>>>(d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
                                                          d.sn_rows.p, d.fr_off.p, front, xp);
    }
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

// xp[k] = b[perm[k]]  /  x[perm[k]] = xp[k]
__global__ void gather_perm(const double *__restrict__ b, const int32_t *__restrict__ perm,
                            double *__restrict__ xp, int32_t N) {
    const int32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < N) xp[k] = b[perm[k]];
}
__global__ void scatter_perm(const double *__restrict__ xp, const int32_t *__restrict__ perm,
                             double *__restrict__ x, int32_t N) {
    const int32_t k = blockIdx.x * 256 + threadIdx.x;
    if (k < N) x[perm[k]] = xp[k];
}

int launch_solve(qg_handle *h, const double *rhs, double *x, int precision) {
    const int32_t N = h->N;
    const unsigned g = (unsigned)((N + 255) / 256);
    gather_perm<<<g, 256, 0, h->stream>>>(rhs, h->d.perm.p, h->d.xp.p, N);
    int rc = precision == QG_FP32_IR ? solve_perm<float>(h, h->d.front32.p, h->d.sinv32.p)
                                     : solve_perm<double>(h, h->d.front64.p, h->d.sinv64.p);
    if (rc) return rc;
    scatter_perm<<<g, 256, 0, h->stream>>>(h->d.xp.p, h->d.perm.p, x, N);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

}  // namespace qg
