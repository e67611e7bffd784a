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
// Small fronts: one wavefront per supernode, per level.  Large fronts: a
// gather kernel, then one kernel per NB-column block that applies the stored
// inverse of the diagonal block and updates the rows below (forward), or the
// transposed sequence (backward).
#include "kernels.hpp"
#include "solver.hpp"

namespace qg {

// ------------------------------- small -------------------------------------
template <typename T>
__global__ void __launch_bounds__(64) fwd_small(
    const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, const T *__restrict__ front,
    const int32_t *__restrict__ ch_ptr, const int32_t *__restrict__ ch_list,
    const int64_t *__restrict__ rel_ptr, const int32_t *__restrict__ rel,
    const int64_t *__restrict__ uv_off, double *__restrict__ uvec, double *__restrict__ xp) {
    __shared__ double v[SMALL_R];
    const int32_t s = sn_list[blockIdx.x];
    const int lane = threadIdx.x;
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    if (lane < r) v[lane] = lane < k ? xp[f + lane] : 0.0;
    __syncthreads();
    for (int32_t u = ch_ptr[s]; u < ch_ptr[s + 1]; ++u) {
        const int32_t c = ch_list[u];
        const int64_t m0 = rel_ptr[c], mc = rel_ptr[c + 1] - m0;
        for (int64_t i = lane; i < mc; i += 64) v[rel[m0 + i]] += uvec[uv_off[c] + i];
        __syncthreads();
    }
    const T *F = front + fr_off[s];
    for (int32_t jj = 0; jj < k; ++jj) {
        const double yj = v[jj];
        if (lane > jj && lane < r) v[lane] -= (double)F[(int64_t)jj * r + lane] * yj;
        __syncthreads();
    }
    if (lane < k) xp[f + lane] = v[lane];
    else if (lane < r) uvec[uv_off[s] + lane - k] = v[lane];
}

template <typename T>
__global__ void __launch_bounds__(64) bwd_small(
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
// v = [own entries; 0] + children's update vectors (one workgroup).
__global__ void __launch_bounds__(256) fwd_gather(
    int32_t s, const int32_t *__restrict__ sn_first, const int64_t *__restrict__ sn_rptr,
    const int32_t *__restrict__ ch_ptr, const int32_t *__restrict__ ch_list,
    const int64_t *__restrict__ rel_ptr, const int32_t *__restrict__ rel,
    const int64_t *__restrict__ uv_off, const double *__restrict__ uvec,
    const double *__restrict__ xp, double *__restrict__ vbuf) {
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    for (int32_t i = threadIdx.x; i < r; i += 256) vbuf[i] = i < k ? xp[f + i] : 0.0;
    for (int32_t u = ch_ptr[s]; u < ch_ptr[s + 1]; ++u) {
        __syncthreads();
        const int32_t c = ch_list[u];
        const int64_t m0 = rel_ptr[c], mc = rel_ptr[c + 1] - m0;
        for (int64_t i = threadIdx.x; i < mc; i += 256) vbuf[rel[m0 + i]] += uvec[uv_off[c] + i];
    }
}

// Block j0 (b columns): y = X v[j0:j0+b] (X = inverse of the unit diagonal
// block); block 0 writes y to xp; every block updates 256 rows below.
template <typename T>
__global__ void __launch_bounds__(256) fwd_block(const T *__restrict__ F, int32_t r, int32_t j0, int32_t b,
                                                 const T *__restrict__ X, double *__restrict__ vbuf,
                                                 double *__restrict__ xp_own) {
    __shared__ double y[NB];
    const int tid = threadIdx.x;
    if (tid < b) {
        double acc = 0.0;
        for (int32_t t = 0; t <= tid; ++t) acc += (double)X[t * NB + tid] * vbuf[j0 + t];
        y[tid] = acc;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < b) xp_own[j0 + tid] = y[tid];
    const int32_t row = j0 + b + blockIdx.x * 256 + tid;
    if (row < r) {
        double acc = 0.0;
        for (int32_t t = 0; t < b; ++t) acc += (double)F[(int64_t)(j0 + t) * r + row] * y[t];
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

// Block j0 (b columns, processed last to first): y = X' v[j0:j0+b]; block 0
// writes y; every block updates 256 earlier entries: v[c] -= L(j0:j0+b, c)' y.
template <typename T>
__global__ void __launch_bounds__(256) bwd_block(const T *__restrict__ F, int32_t r, int32_t j0, int32_t b,
                                                 const T *__restrict__ X, double *__restrict__ vbuf,
                                                 double *__restrict__ xp_own) {
    __shared__ double y[NB];
    const int tid = threadIdx.x;
    if (tid < b) {
        double acc = 0.0;
        for (int32_t t = tid; t < b; ++t) acc += (double)X[tid * NB + t] * vbuf[j0 + t];
        y[tid] = acc;
    }
    __syncthreads();
    if (blockIdx.x == 0 && tid < b) xp_own[j0 + tid] = y[tid];
    const int32_t c = blockIdx.x * 256 + tid;
    if (c < j0) {
        double acc = 0.0;
        const T *col = F + (int64_t)c * r + j0;
        for (int32_t t = 0; t < b; ++t) acc += (double)col[t] * y[t];
        vbuf[c] -= acc;
    }
}

__global__ void copy_tail(const double *__restrict__ src, double *__restrict__ dst, int32_t n) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------- driver ------------------------------------
template <typename T>
static int solve_perm(qg_handle *h, const T *front, const T *dinv) {
    const Plan &pl = h->plan;
    Device &d = h->d;
    double *xp = d.xp.p;
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        const int32_t s0 = pl.lvl_small_ptr[L], s1 = pl.lvl_small_ptr[L + 1];
        if (s1 > s0)
            fwd_small<T><<<s1 - s0, 64, 0, h->stream>>>(d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
                                                          d.fr_off.p, front, d.ch_ptr.p, d.ch_list.p,
                                                          d.rel_ptr.p, d.rel.p, d.uv_off.p, d.uvec.p, xp);
        for (int32_t u = pl.lvl_large_ptr[L]; u < pl.lvl_large_ptr[L + 1]; ++u) {
            const int32_t s = pl.lvl_large_sn[u];
            const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
            const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
            const T *F = front + pl.fr_off[s];
            fwd_gather<<<1, 256, 0, h->stream>>>(s, d.sn_first.p, d.sn_rptr.p, d.ch_ptr.p, d.ch_list.p,
                                                 d.rel_ptr.p, d.rel.p, d.uv_off.p, d.uvec.p, xp, d.vbuf.p);
            for (int32_t j0 = 0; j0 < k; j0 += NB) {
                const int32_t b = std::min(NB, k - j0);
                const int32_t rows = r - j0 - b;
                const unsigned grid = (unsigned)std::max(1, (rows + 255) / 256);
                fwd_block<T><<<grid, 256, 0, h->stream>>>(F, r, j0, b, dinv + pl.dinv_off[s] + (int64_t)(j0 / NB) * NB * NB,
                                                            d.vbuf.p, xp + pl.sn_first[s]);
            }
            if (r > k)
                copy_tail<<<(r - k + 255) / 256, 256, 0, h->stream>>>(d.vbuf.p + k, d.uvec.p + pl.uv_off[s], r - k);
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
            const int32_t nblk = (k + NB - 1) / NB;
            for (int32_t bi = nblk - 1; bi >= 0; --bi) {
                const int32_t j0 = bi * NB;
                const int32_t b = std::min(NB, k - j0);
                const unsigned grid = (unsigned)std::max(1, (j0 + 255) / 256);
                bwd_block<T><<<grid, 256, 0, h->stream>>>(F, r, j0, b, dinv + pl.dinv_off[s] + (int64_t)bi * NB * NB,
                                                            d.vbuf.p, xp + pl.sn_first[s]);
            }
        }
        const int32_t s0 = pl.lvl_small_ptr[L], s1 = pl.lvl_small_ptr[L + 1];
        if (s1 > s0)
            bwd_small<T><<<s1 - s0, 64, 0, h->stream>>>(d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
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
    int rc = precision == QG_FP32_IR ? solve_perm<float>(h, h->d.front32.p, h->d.dinv32.p)
                                     : solve_perm<double>(h, h->d.front64.p, h->d.dinv64.p);
    if (rc) return rc;
    scatter_perm<<<g, 256, 0, h->stream>>>(h->d.xp.p, h->d.perm.p, x, N);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

}  // namespace qg
