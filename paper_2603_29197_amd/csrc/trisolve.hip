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
// fronts: a gather kernel, then one kernel per SB-column super-block that
// solves with the diagonal block (stored inverses of its 64 x 64 diagonal
// blocks) and updates the rows below (forward), or the transposed sequence
// (backward).
#include "kernels.hpp"
#include "solver.hpp"

namespace qg {

// ------------------------------- small -------------------------------------
// Gather of one level: one thread per (front s, row j) task:
// v = [j < k_s ? x_perm(first_s + j) : 0] + sum over the child columns that map
// onto row j of their update-vector entries (contribution lists of the
// assembly, in child order).  Update vectors live in the children's own
// task slots (rows k_c .. r_c - 1).
__global__ void __launch_bounds__(256) fwd_gather_level(
    int64_t t0, int64_t nt, const int32_t *__restrict__ task_sn, const int32_t *__restrict__ task_col,
    const int32_t *__restrict__ sn_first, const int64_t *__restrict__ task0,
    const int64_t *__restrict__ ctb_ptr, const int32_t *__restrict__ ctb_child,
    const int32_t *__restrict__ ctb_col, const double *__restrict__ xp, double *__restrict__ vwork) {
    const int64_t t = t0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= t0 + nt) return;
    const int32_t s = task_sn[t], j = task_col[t];
    const int32_t f = sn_first[s], k = sn_first[s + 1] - f;
    double v = j < k ? xp[f + j] : 0.0;
    for (int64_t u = ctb_ptr[t]; u < ctb_ptr[t + 1]; ++u) {
        const int32_t c = ctb_child[u];
        v += vwork[task0[c] + (sn_first[c + 1] - sn_first[c]) + ctb_col[u]];
    }
    vwork[t] = v;
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
// Super-block [J0, J0+kb) (kb <= SB): y = X v[J0:J0+kb) with the stored
// inverse X of the unit-lower diagonal block (one dot product per thread,
// lanes along rows of the column-major X, leading dimension ld:
// coalesced); workgroup 0 writes y
// to the solution; each workgroup then updates 256 rows below:
// v[row] -= L(row, J0:J0+kb) y (lanes along rows: coalesced).
template <typename T>
__global__ void __launch_bounds__(256) fwd_sblock(const T *__restrict__ F, int32_t r, int32_t J0, int32_t kb,
                                                  const T *__restrict__ Xsb, int32_t ld, double *__restrict__ vbuf,
                                                  double *__restrict__ xp_own) {
    __shared__ double yin[SB];
    __shared__ double y[SB];
    const int tid = threadIdx.x;
    if (tid < kb) yin[tid] = vbuf[J0 + tid];
    __syncthreads();
    if (tid < kb) {
        const int32_t qend = min(kb, ((tid >> 6) + 1) * NB);    // X is lower: blocks right of the wave's are 0
        const T *Xr = Xsb + tid;
        double acc = 0.0;
#pragma unroll 8
        for (int32_t q = 0; q < qend; ++q) acc += (double)Xr[(int64_t)q * ld] * yin[q];
        y[tid] = acc;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < kb) xp_own[J0 + tid] = y[tid];
    const int32_t row = J0 + kb + blockIdx.x * 256 + tid;
    if (row < r) {
        double acc = 0.0;
        const T *p = F + (int64_t)J0 * r + row;
#pragma unroll 16
        for (int32_t q = 0; q < kb; ++q) acc += (double)p[(int64_t)q * r] * y[q];
        vbuf[row] -= acc;
    }
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

// Super-block [J0, J0+kb), processed last to first: y = X' v[J0:J0+kb) with
// the stored transpose of the diagonal block's inverse (coalesced as in the
// forward case); workgroup 0 writes y to the solution; each workgroup then
// updates 64 earlier entries: v[c] -= L(J0:J0+kb, c)' y, with lanes running
// along the contiguous rows t of each column (coalesced) and a wavefront
// reduction.
template <typename T>
__global__ void __launch_bounds__(256) bwd_sblock(const T *__restrict__ F, int32_t r, int32_t J0, int32_t kb,
                                                  const T *__restrict__ XTsb, int32_t ld, double *__restrict__ vbuf,
                                                  double *__restrict__ xp_own) {
    __shared__ double yin[SB];
    __shared__ double y[SB];
    const int tid = threadIdx.x;
    if (tid < kb) yin[tid] = vbuf[J0 + tid];
    __syncthreads();
    if (tid < kb) {
        const int32_t qbeg = (tid >> 6) * NB;                   // X' is upper: blocks left of the wave's are 0
        const T *Xr = XTsb + tid;
        double acc = 0.0;
#pragma unroll 8
        for (int32_t q = qbeg; q < kb; ++q) acc += (double)Xr[(int64_t)q * ld] * yin[q];
        y[tid] = acc;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < kb) xp_own[J0 + tid] = y[tid];
    // columns c0 .. c0+63 before the super-block: wave w handles 16 of them
    const int32_t c0 = blockIdx.x * NB;
    if (c0 >= J0) return;
    const int lane = tid & 63, w = tid >> 6;
    for (int32_t cc = 0; cc < 16; ++cc) {
        const int32_t c = c0 + w * 16 + cc;
        if (c >= J0) break;
        const T *col = F + (int64_t)c * r + J0;
        double s = 0.0;
        for (int32_t t = lane; t < kb; t += 64) s += (double)col[t] * y[t];
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) vbuf[c] -= s;
    }
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
            fwd_gather_level<<<(unsigned)((nt + 255) / 256), 256, 0, h->stream>>>(
                t0, nt, d.task_sn.p, d.task_col.p, d.sn_first.p, d.task0.p, d.ctb_ptr.p, d.ctb_child.p,
                d.ctb_col.p, xp, d.vwork.p);
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
                const int32_t rows = r - J0 - kb;
                const unsigned grid = (unsigned)std::max(1, (rows + 255) / 256);
                const int32_t ld = (kb + NB - 1) / NB * NB;
                const T *Xsb = sinv + pl.sinv_off[s] + (int64_t)(J0 / SB) * 2 * SB * SB;
                fwd_sblock<T><<<grid, 256, 0, h->stream>>>(F, r, J0, kb, Xsb, ld, vs, xp + pl.sn_first[s]);
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
                const unsigned grid = (unsigned)std::max(1, (J0 + NB - 1) / NB);
                const int32_t ld = (kb + NB - 1) / NB * NB;
                const T *XTsb = sinv + pl.sinv_off[s] + (int64_t)(J0 / SB) * 2 * SB * SB + (int64_t)ld * ld;
                bwd_sblock<T><<<grid, 256, 0, h->stream>>>(F, r, J0, kb, XTsb, ld, d.vbuf.p, xp + pl.sn_first[s]);
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
