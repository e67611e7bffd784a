// Vector work of the Newton step: KKT residuals of problem (1), the
// refinement residual against the unregularized KKT matrix of eq. (2),
// right-hand sides and the iterate update.  Reductions are two-pass (per
// block partials, then one block in fixed order), so results do not depend
// on scheduling.  The sparse residual kernels walk the rows in a grid-stride
// loop over at most RED_BLOCKS blocks per problem (the partials of a block
// are formed once, at its end), with R lanes per row: 4 when the rows hold 8
// entries or fewer on average, else 16.
#include "vec.hpp"

#include <cmath>
#include <cstring>

namespace qg {

// Per-block reduction helper: NS slots, each either a sum or a max-abs; slot
// q of block b goes to partials[q * nblk + b].
template <int NS>
__device__ inline void block_reduce_store(double (&val)[NS], const uint32_t maxmask, double *partials,
                                          int32_t nblk, int32_t block) {
    __shared__ double sh[NS][4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
        double v = val[q];
        const bool ismax = (maxmask >> q) & 1u;
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off);
            v = ismax ? nan_max(v, o) : v + o;
        }
        if (lane == 0) sh[q][wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        const int q = threadIdx.x;
        const bool ismax = (maxmask >> q) & 1u;
        double v = sh[q][0];
        for (int w = 1; w < 4; ++w) v = ismax ? nan_max(v, sh[q][w]) : v + sh[q][w];
        partials[(int64_t)q * nblk + block] = v;
    }
}

template <int NS>
__device__ inline void accumulate(double (&val)[NS], const uint32_t maxmask, int q, double x) {
    val[q] = ((maxmask >> q) & 1u) ? nan_max(val[q], x) : val[q] + x;
}

// Second pass: workgroup g reduces the g-th run of nblk x ns partials (one
// run per problem of a batch; slot-major) into out[g ns ..]: wavefront w of W takes
// the slots w, w + W, ..., each lane a fixed strided subset of the blocks in a
// fixed order, then a fixed butterfly (deterministic).
__global__ void __launch_bounds__(FINISH_THREADS) finish_reduce(const double *__restrict__ partials, int32_t nblk,
                                                     int32_t ns, uint32_t maxmask, double *__restrict__ out) {
    partials += (int64_t)blockIdx.x * nblk * ns;
    out += (int64_t)blockIdx.x * ns;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = wave; q < ns; q += (int)(blockDim.x >> 6)) {
        const bool ismax = (maxmask >> q) & 1u;
        const double *pq = partials + (int64_t)q * nblk;
        const double id = ismax ? -INFINITY : 0.0;
        double v = id;
        // 16 loads per lane in flight at a time (the partials were just written by other compute
        // units: each round waits for memory once)
        for (int32_t b0 = lane; b0 < nblk; b0 += 64 * 16) {
            double t[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) t[u] = b0 + 64 * u < nblk ? pq[b0 + 64 * u] : id;
#pragma unroll
            for (int u = 0; u < 16; ++u) v = ismax ? nan_max(v, t[u]) : v + t[u];
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double o = __shfl_xor(v, off);
            v = ismax ? nan_max(v, o) : v + o;
        }
        if (lane == 0) out[q] = v;
    }
}

// Residuals of problem (1): rx = Px + A'y + G'z + c, ry = Ax - b,
// rz = Gx + s - h, and the scalars of the stopping test (slots in vec.hpp).
// A batch of kb problems (sizes n1, p1, m1, l1 each; n = kb n1, ...) is one
// stacked problem: blockIdx.y is the problem, whose rows (its x, y and cone
// rows, see batch.cpp) the x-blocks walk, so that every block's partial
// scalars belong to one problem.  kb = 1 is the plain problem.
__device__ inline int32_t stacked_row(int32_t kb, int32_t n1, int32_t p1, int32_t m1, int32_t l1, int32_t inst,
                                      int32_t loc) {
    if (loc < n1) return inst * n1 + loc;
    if (loc < n1 + p1) return kb * n1 + inst * p1 + (loc - n1);
    const int32_t w = loc - n1 - p1;
    return kb * (n1 + p1) + (w < l1 ? inst * l1 + w : kb * l1 + inst * (m1 - l1) + (w - l1));
}

template <int R>
__global__ void __launch_bounds__(256) residual_kernel(
    int32_t n, int32_t p, int32_t m, const int64_t *__restrict__ kr_ptr, const int32_t *__restrict__ kr_col,
    const double *__restrict__ kr_val, const double *__restrict__ x, const double *__restrict__ y,
    const double *__restrict__ z, const double *__restrict__ s, const double *__restrict__ c,
    const double *__restrict__ b, const double *__restrict__ hv, double *__restrict__ rx,
    double *__restrict__ ry, double *__restrict__ rz, double *__restrict__ partials, int32_t kb, int32_t n1,
    int32_t p1, int32_t m1, int32_t l1, const double *__restrict__ rsc) {
    double val[NSCAL];
#pragma unroll
    for (int q = 0; q < NSCAL; ++q) val[q] = 0.0;
    const int sub = threadIdx.x & (R - 1);
    const int32_t N = n + p + m;
    const int32_t rows1 = n1 + p1 + m1, stride = (int32_t)gridDim.x * (256 / R);
    // the R lanes of a row run the loop together, so the shuffles below stay inside the row's lanes
    for (int32_t loc = blockIdx.x * (256 / R) + (threadIdx.x / R); loc < rows1; loc += stride) {
        const int32_t i = stacked_row(kb, n1, p1, m1, l1, blockIdx.y, loc);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t t = kr_ptr[i] + sub; t < kr_ptr[i + 1]; t += R) {
            const int32_t j = kr_col[t];
            const double v = kr_val[t];
            if (j < n) a0 += v * x[j];
            else if (j < n + p) a1 += v * y[j - n];
            else a2 += v * z[j - n - p];
        }
#pragma unroll
        for (int off = R / 2; off > 0; off >>= 1) {
            a0 += __shfl_xor(a0, off);
            a1 += __shfl_xor(a1, off);
            a2 += __shfl_xor(a2, off);
        }
        if (sub == 0 && i < N) {
            // equilibrated data: the max-norm terms in the caller's units (u = 1 / the row's scaling)
            const double u = rsc ? rsc[i] : 1.0;
            if (i < n) {
                const double r_ = a0 + a1 + a2 + c[i];
                rx[i] = r_;
                accumulate(val, SCAL_MAXMASK, S_PX, u * fabs(a0)); accumulate(val, SCAL_MAXMASK, S_ATY, u * fabs(a1));
                accumulate(val, SCAL_MAXMASK, S_GTZ, u * fabs(a2)); accumulate(val, SCAL_MAXMASK, S_RX, u * fabs(r_));
                accumulate(val, SCAL_MAXMASK, S_XPX, x[i] * a0); accumulate(val, SCAL_MAXMASK, S_CX, c[i] * x[i]);
                accumulate(val, SCAL_MAXMASK, S_C, u * fabs(c[i]));
            } else if (i < n + p) {
                const int32_t e = i - n;
                const double r_ = a0 - b[e];
                ry[e] = r_;
                accumulate(val, SCAL_MAXMASK, S_AX, u * fabs(a0)); accumulate(val, SCAL_MAXMASK, S_RY, u * fabs(r_));
                accumulate(val, SCAL_MAXMASK, S_BY, b[e] * y[e]); accumulate(val, SCAL_MAXMASK, S_B, u * fabs(b[e]));
            } else {
                const int32_t e = i - n - p;
                const double r_ = a0 + s[e] - hv[e];
                rz[e] = r_;
                accumulate(val, SCAL_MAXMASK, S_GX, u * fabs(a0)); accumulate(val, SCAL_MAXMASK, S_RZ, u * fabs(r_));
                accumulate(val, SCAL_MAXMASK, S_HZ, hv[e] * z[e]); accumulate(val, SCAL_MAXMASK, S_SZ, s[e] * z[e]);
                accumulate(val, SCAL_MAXMASK, S_S, u * fabs(s[e])); accumulate(val, SCAL_MAXMASK, S_H, u * fabs(hv[e]));
            }
        }
    }
    block_reduce_store<NSCAL>(val, SCAL_MAXMASK, partials + (int64_t)blockIdx.y * NSCAL * gridDim.x,
                              (int32_t)gridDim.x, (int32_t)blockIdx.x);
}

// res = rhs - K sol, K = static part + (3,3) block from kval; slot 0 of the
// partials: max |res|, slot 1: max |rhs|.
template <int R>
__global__ void __launch_bounds__(256) kkt_residual_kernel(
    int32_t n, int32_t p, int32_t m, int32_t l, const int64_t *__restrict__ kr_ptr,
    const int32_t *__restrict__ kr_col, const double *__restrict__ kr_val, const double *__restrict__ kval,
    const int64_t *__restrict__ blk33, const int64_t *__restrict__ blk_off, const int32_t *__restrict__ soc_off,
    const int32_t *__restrict__ zcone, const double *__restrict__ rhs, const double *__restrict__ sol,
    double *__restrict__ res, double *__restrict__ partials) {
    double val[2] = {0.0, 0.0};
    const int32_t N = n + p + m;
    const int sub = threadIdx.x & (R - 1);
    const int32_t stride = (int32_t)gridDim.x * (256 / R);
    for (int32_t i = blockIdx.x * (256 / R) + (threadIdx.x / R); i < N; i += stride) {
        double acc = 0.0;
        for (int64_t t = kr_ptr[i] + sub; t < kr_ptr[i + 1]; t += R) acc += kr_val[t] * sol[kr_col[t]];
        if (i >= n + p) {
            const int32_t e = i - n - p;
            const double *zs = sol + n + p;
            if (e < l) {
                if (sub == 0) acc += kval[blk33[e]] * zs[e];
            } else {
                const int32_t k = zcone[e];
                const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
                const int32_t a = e - off;
                const int64_t base = l + blk_off[k];
                for (int32_t bb = sub; bb < q; bb += R) {
                    const int32_t lo = a < bb ? a : bb, hi = a < bb ? bb : a;
                    acc += kval[blk33[base + (int64_t)hi * (hi + 1) / 2 + lo]] * zs[bb + off];
                }
            }
        }
#pragma unroll
        for (int off = R / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
        if (sub == 0) {
            const double r_ = rhs[i] - acc;
            res[i] = r_;
            val[0] = nan_max(val[0], fabs(r_));
            val[1] = nan_max(val[1], fabs(rhs[i]));
        }
    }
    block_reduce_store<2>(val, 3u, partials, (int32_t)gridDim.x, (int32_t)blockIdx.x);
}

__global__ void build_rhs_kernel(int32_t n, int32_t p, int32_t m, const double *__restrict__ rx,
                                 const double *__restrict__ ry, const double *__restrict__ rz,
                                 const double *__restrict__ zpart, double zsign, double *__restrict__ rhs) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    const int32_t N = n + p + m;
    if (i >= N) return;
    if (i < n) rhs[i] = -rx[i];
    else if (i < n + p) rhs[i] = -ry[i - n];
    else rhs[i] = -rz[i - n - p] + zsign * zpart[i - n - p];
}

__global__ void axpy_kernel(int32_t len, double a, const double *__restrict__ xv, double *__restrict__ yv) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < len) yv[i] += a * xv[i];
}

// (x, y, z, s) += alpha (dx, dy, dz, ds), alpha = min(1, frac * min(a_s, a_z)); in a batch of kb
// problems (sizes n1, p1, m1, l1 each; the stacked layout of batch.cpp) each row takes its problem's alpha
__global__ void update_kernel(int32_t n, int32_t p, int32_t m, const double *__restrict__ d,
                              const double *__restrict__ ds, const unsigned long long *__restrict__ amin,
                              double frac, double *__restrict__ x, double *__restrict__ y,
                              double *__restrict__ z, double *__restrict__ s, double *__restrict__ alpha_out,
                              int32_t kb, int32_t n1, int32_t p1, int32_t m1, int32_t l1,
                              const double *__restrict__ gate) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    int32_t inst = 0;
    if (kb > 1) {
        if (i < n) inst = i / n1;
        else if (i < n + p) inst = (i - n) / p1;
        else {
            const int32_t e = i - n - p, l = kb * l1;
            inst = e < l ? e / l1 : (m1 > l1 ? (e - l) / (m1 - l1) : 0);
        }
        inst = inst < kb ? inst : kb - 1;
    }
    const double as = __longlong_as_double((long long)amin[4 * inst + 2]);
    const double az = __longlong_as_double((long long)amin[4 * inst + 3]);
    // a problem of a batch whose own stopping test has passed keeps its iterate (gate 0)
    const double g = kb > 1 ? gate[inst] : 1.0;
    const double alpha = g * fmin(1.0, frac * fmin(as, az));
    if (i == 0 && alpha_out) *alpha_out = alpha;
    if (g == 0.0) return;
    if (i < n) x[i] += alpha * d[i];
    else if (i < n + p) y[i - n] += alpha * d[i];
    else if (i < n + p + m) {
        const int32_t e = i - n - p;
        z[e] += alpha * d[i];
        s[e] += alpha * ds[e];
    }
}

__global__ void fill_kernel(int32_t len, double v, double *__restrict__ out) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < len) out[i] = v;
}
__global__ void scale_copy_kernel(int32_t len, double a, const double *__restrict__ xv, double *__restrict__ out) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < len) out[i] = a * xv[i];
}

int launch_fill(qg_handle *h, int32_t len, double v, double *out) {
    if (len <= 0) return QG_OK;
    fill_kernel<<<(len + 255) / 256, 256, 0, h->stream>>>(len, v, out);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}
int launch_scale_copy(qg_handle *h, int32_t len, double a, const double *xv, double *out) {
    if (len <= 0) return QG_OK;
    scale_copy_kernel<<<(len + 255) / 256, 256, 0, h->stream>>>(len, a, xv, out);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

// Lanes per row of the sparse residual kernels and their block count (at most RED_BLOCKS per
// problem, fewer when the rows run out).
static int lanes_per_row(const qg_handle *h) { return h->kr_nnz <= 8 * (int64_t)h->N ? 4 : 16; }
static int32_t red_blocks(int32_t rows, int R) {
    const int32_t need = (rows + 256 / R - 1) / (256 / R);
    return need < 1 ? 1 : (need < RED_BLOCKS ? need : RED_BLOCKS);
}

int launch_residual(qg_handle *h, const double *x, const double *y, const double *z, const double *s,
                    double *scal_host) {
    Device &d = h->d;
    const int32_t kb = h->ncopy;
    const int32_t n1 = h->n / kb, p1 = h->p / kb, m1 = h->m / kb, l1 = h->pp.l / kb;
    const int R = lanes_per_row(h);
    const int32_t nblk = red_blocks(n1 + p1 + m1, R);
    const dim3 grid((unsigned)nblk, (unsigned)kb);
    const double *rsc = h->ruiz > 0 ? d.rz_rsc.p : nullptr;
    if (R == 4)
        residual_kernel<4><<<grid, 256, 0, h->stream>>>(
            h->n, h->p, h->m, d.kr_ptr.p, d.kr_col.p, d.kr_val.p, x, y, z, s, d.c.p, d.b.p, d.h.p, d.rx.p, d.ry.p,
            d.rz.p, d.partials.p, kb, n1, p1, m1, l1, rsc);
    else
        residual_kernel<16><<<grid, 256, 0, h->stream>>>(
            h->n, h->p, h->m, d.kr_ptr.p, d.kr_col.p, d.kr_val.p, x, y, z, s, d.c.p, d.b.p, d.h.p, d.rx.p, d.ry.p,
            d.rz.p, d.partials.p, kb, n1, p1, m1, l1, rsc);
    finish_reduce<<<(unsigned)kb, FINISH_THREADS, 0, h->stream>>>(d.partials.p, nblk, NSCAL, SCAL_MAXMASK, d.scal_inst.p);
    QG_HIP(h, hipGetLastError());
    const size_t nv = (size_t)kb * NSCAL;
    double *dst = nv + 4 <= (size_t)PIN_DOUBLES ? h->pin : scal_host;   // large batches: pageable
    QG_HIP(h, hipMemcpyAsync(dst, d.scal_inst.p, nv * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (int rc = stream_wait(h)) return rc;
    if (dst != scal_host) std::memcpy(scal_host, dst, nv * sizeof(double));
    return QG_OK;
}

// Equilibrated vectors from the caller's: c^ = k D c, b^ = E b, h^ = F h (dsc = D, E, F back to back).
__global__ void ruiz_scale_kernel(int32_t n, int32_t p, int32_t m, double k, const double *__restrict__ dsc,
                                  const double *__restrict__ craw, const double *__restrict__ braw,
                                  const double *__restrict__ hraw, double *__restrict__ c, double *__restrict__ b,
                                  double *__restrict__ hv) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) c[i] = k * dsc[i] * craw[i];
    else if (i < n + p) b[i - n] = dsc[i] * braw[i - n];
    else if (i < n + p + m) hv[i - n - p] = dsc[i] * hraw[i - n - p];
}

// The caller's solution from the equilibrated one: x = D x^, y = E y^ / k, z = F z^ / k, s = s^ / F.
// Every output pointer may be null.
__global__ void ruiz_unscale_kernel(int32_t n, int32_t p, int32_t m, double k, const double *__restrict__ dsc,
                                    const double *__restrict__ xs, const double *__restrict__ ss,
                                    const double *__restrict__ ys, const double *__restrict__ zs,
                                    double *__restrict__ x, double *__restrict__ s, double *__restrict__ y,
                                    double *__restrict__ z) {
    const int32_t i = (int32_t)(blockIdx.x * 256 + threadIdx.x);
    if (i < n) {
        if (x) x[i] = dsc[i] * xs[i];
    } else if (i < n + p) {
        if (y) y[i - n] = dsc[i] * ys[i - n] / k;
    } else if (i < n + p + m) {
        const int32_t e = i - n - p;
        if (z) z[e] = dsc[i] * zs[e] / k;
        if (s) s[e] = ss[e] / dsc[i];
    }
}

int launch_scale_vectors(qg_handle *h) {
    Device &d = h->d;
    const int32_t N = h->N;
    if (N == 0) return QG_OK;
    ruiz_scale_kernel<<<(unsigned)((N + 255) / 256), 256, 0, h->stream>>>(h->n, h->p, h->m, h->ruiz_k,
                                                                          d.rz_dsc.p, d.craw.p, d.braw.p,
                                                                          d.hraw.p, d.c.p, d.b.p, d.h.p);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int launch_unscale_outputs(qg_handle *h, double *x, double *s, double *y, double *z) {
    Device &d = h->d;
    const int32_t N = h->N;
    if (N == 0 || (!x && !s && !y && !z)) return QG_OK;
    ruiz_unscale_kernel<<<(unsigned)((N + 255) / 256), 256, 0, h->stream>>>(
        h->n, h->p, h->m, h->ruiz_k, d.rz_dsc.p, d.x.p, d.s.p, d.y.p, d.z.p, x, s, y, z);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int launch_kkt_residual(qg_handle *h, const double *rhs, const double *sol, double *res, double *norms) {
    Device &d = h->d;
    const int32_t N = h->N;
    const int R = lanes_per_row(h);
    const int32_t nblk = red_blocks(N, R);
    if (R == 4)
        kkt_residual_kernel<4><<<nblk, 256, 0, h->stream>>>(h->n, h->p, h->m, h->pp.l, d.kr_ptr.p, d.kr_col.p,
                                                            d.kr_val.p, d.kval.p, d.blk33.p, d.blk_off.p,
                                                            d.soc_off.p, d.zcone.p, rhs, sol, res, d.partials.p);
    else
        kkt_residual_kernel<16><<<nblk, 256, 0, h->stream>>>(h->n, h->p, h->m, h->pp.l, d.kr_ptr.p, d.kr_col.p,
                                                             d.kr_val.p, d.kval.p, d.blk33.p, d.blk_off.p,
                                                             d.soc_off.p, d.zcone.p, rhs, sol, res, d.partials.p);
    finish_reduce<<<1, 128, 0, h->stream>>>(d.partials.p, nblk, 2, 3u, d.scal.p + NSCAL);
    QG_HIP(h, hipGetLastError());
    double *pn = h->pin + PIN_DOUBLES - 4;
    QG_HIP(h, hipMemcpyAsync(pn, d.scal.p + NSCAL, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if (int rc = stream_wait(h)) return rc;
    norms[0] = pn[0];
    norms[1] = pn[1];
    return QG_OK;
}

int launch_build_rhs(qg_handle *h, const double *zpart, double zsign, double *rhs) {
    const int32_t N = h->N;
    build_rhs_kernel<<<(N + 255) / 256, 256, 0, h->stream>>>(h->n, h->p, h->m, h->d.rx.p, h->d.ry.p,
                                                             h->d.rz.p, zpart, zsign, rhs);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int launch_axpy(qg_handle *h, int32_t len, double a, const double *xv, double *yv) {
    if (len <= 0) return QG_OK;
    axpy_kernel<<<(len + 255) / 256, 256, 0, h->stream>>>(len, a, xv, yv);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int launch_update(qg_handle *h, const double *dvec, const double *ds, double frac, double *alpha_dev) {
    Device &d = h->d;
    const int32_t N = h->N;
    const int32_t kb = h->ncopy;
    update_kernel<<<(N + 255) / 256, 256, 0, h->stream>>>(h->n, h->p, h->m, dvec, ds, d.amin.p, frac, d.x.p,
                                                          d.y.p, d.z.p, d.s.p, alpha_dev, kb, h->n / kb,
                                                          h->p / kb, h->m / kb, h->pp.l / kb, d.mu.p + kb);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int stream_wait(qg_handle *h) {
    QG_HIP(h, hipEventRecord(h->ev_sync, h->stream));
    hipError_t e;
    while ((e = hipEventQuery(h->ev_sync)) == hipErrorNotReady) {
    }
    QG_HIP(h, e);
    return QG_OK;
}

int nreg_async(qg_handle *h) {
    QG_HIP(h, hipMemcpyAsync(h->pin + PIN_DOUBLES - 2, h->d.nreg.p, sizeof(int32_t), hipMemcpyDeviceToHost,
                             h->stream));
    return QG_OK;
}

int nreg_pinned(const qg_handle *h) {
    int32_t v;
    std::memcpy(&v, h->pin + PIN_DOUBLES - 2, sizeof(int32_t));
    return v;
}

// HIP graphs of fixed launch sequences (no memset or copy nodes: kernels and event joins only)
int graph_replay(qg_handle *h, hipGraphExec_t &exec, int (*enqueue)(qg_handle *, void *), void *arg) {
    if (!exec) {
        // captured on the handle's private stream (the caller's may be the legacy default stream, which
        // cannot be captured), replayed on the caller's
        hipGraph_t g = nullptr;
        hipStream_t caller = h->stream;
        QG_HIP(h, hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
        h->stream = h->cap;
        const int rc = enqueue(h, arg);
        h->stream = caller;
        const hipError_t e = hipStreamEndCapture(h->cap, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(h, e);
        const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            exec = nullptr;
            return hip_fail(h, ei);
        }
    }
    QG_HIP(h, hipGraphLaunch(exec, h->stream));
    return QG_OK;
}

void drop_graphs(qg_handle *h) {
    for (int i = 0; i < 2; ++i) {
        if (h->g_factor[i]) (void)hipGraphExecDestroy(h->g_factor[i]);
        if (h->g_solve[i]) (void)hipGraphExecDestroy(h->g_solve[i]);
        h->g_factor[i] = h->g_solve[i] = nullptr;
    }
}

int refined_solve(qg_handle *h, const double *rhs, double *x, int precision, int ir_max, int *steps,
                  bool *ok) {
    int rc = launch_solve(h, rhs, x, precision);
    if (rc) return rc;
    int k = 0;
    double nrm[2];
    bool passed = false;
    for (; k < ir_max; ++k) {
        if ((rc = launch_kkt_residual(h, rhs, x, h->d.res.p, nrm))) return rc;
        if (nrm[0] <= h->st.ir_tol * (1.0 + nrm[1])) { passed = true; break; }
        if (!std::isfinite(nrm[0])) break;     // a non-finite solve never passes
        if ((rc = launch_solve(h, h->d.res.p, h->d.corr.p, precision))) return rc;
        if ((rc = launch_axpy(h, h->N, 1.0, h->d.corr.p, x))) return rc;
    }
    if (ok) {
        if (!passed) {   // test the last correction
            if ((rc = launch_kkt_residual(h, rhs, x, h->d.res.p, nrm))) return rc;
            passed = nrm[0] <= h->st.ir_tol * (1.0 + nrm[1]);
        }
        *ok = passed;
    }
    if (steps) *steps = k;
    return QG_OK;
}

}  // namespace qg
