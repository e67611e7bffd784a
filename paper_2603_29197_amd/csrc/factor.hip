// Numeric LDL' of the KKT matrix (paper Sec. 2.2 "factor" phase), once per
// interior-point iteration, on the fixed pattern from the analysis.
//
// Multifrontal, level by level over the supernodal elimination tree:
//  * zero_segments + gather_entries: clear the level's fronts, then form each
//    entry that receives a value from the K entry (+ static regularization on
//    a pivot diagonal) and every child update entry that maps onto it, in
//    child order, one thread per entry (deterministic, no atomics);
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
// assembly (extend-add), one level at a time: the level's fronts are cleared,
// then every entry that receives a value is formed by one thread from its
// sources in a fixed order -- the K entry, the static regularization of a
// pivot diagonal, then the children's update entries in child order -- so no
// two threads write the same entry and the sum does not depend on scheduling.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) zero_segments(const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ len, T *__restrict__ front) {
    const int64_t o = off[blockIdx.x];
    const int32_t n = len[blockIdx.x];
    for (int32_t i = threadIdx.x; i < n; i += 256) front[o + i] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(256) gather_entries(int64_t e0, int64_t ne, const int64_t *__restrict__ dst,
                                                      const int64_t *__restrict__ sptr,
                                                      const int8_t *__restrict__ reg,
                                                      const int64_t *__restrict__ src,
                                                      const double *__restrict__ kval, double delta,
                                                      T *__restrict__ front) {
    const int64_t e = e0 + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= e0 + ne) return;
    int64_t u = sptr[e];
    const int64_t u1 = sptr[e + 1];
    T v = T(0);
    if (u < u1) {
        const int64_t s0 = src[u];
        if (s0 < 0) { v = (T)kval[-s0 - 1]; ++u; }
    }
    const int8_t kd = reg[e];
    if (kd >= 0) v = (T)((double)v + static_reg(kd, delta));
    for (; u < u1; ++u) v += front[src[u]];
    front[dst[e]] = v;
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
// The k pivot steps of one assembled front F (r x r, column-major, in LDS;
// lower part) by the whole 256-thread workgroup, then F's lower part back to
// the front storage G: L in the first k columns, the update block after them.
template <typename T>
__device__ inline void factor_front_lds(T *F, T *__restrict__ G, int32_t r, int32_t k,
                                        const int8_t *__restrict__ kind, double eps, double dyn, int32_t *nreg,
                                        T &dsh) {
    const int tid = threadIdx.x;
    for (int32_t jj = 0; jj < k; ++jj) {
        if (tid == 0) {
            T d = regularize(F[jj * r + jj], kind[jj], eps, dyn, nreg);
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

template <typename T>
__global__ void __launch_bounds__(256) factor_small(
    const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, T *__restrict__ front,
    const int8_t *__restrict__ kind, double eps, double dyn, int32_t *nreg) {
    extern __shared__ double smem_small[];          // r_max * r_max entries of T (launch size)
    T *F = reinterpret_cast<T *>(smem_small);
    __shared__ T dsh;
    const int32_t s = sn_list[blockIdx.x];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - sn_first[s];
    T *G = front + fr_off[s];
    const int tid = threadIdx.x;
    const int32_t rr = r * r;
    for (int32_t base = 0; base < rr; base += 256 * 8) {   // 8 loads in flight per thread
        T g[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) g[u] = ld_or0(G, base + tid + 256 * u, base + tid + 256 * u < rr);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t idx = base + tid + 256 * u;
            if (idx < rr) F[idx] = (idx % r >= idx / r) ? g[u] : T(0);
        }
    }
    __syncthreads();
    factor_front_lds(F, G, r, k, kind + sn_first[s], eps, dyn, nreg, dsh);
}

// The k pivot steps of one front F (r <= CHAIN_R, column-major in LDS, lower
// part) by one wavefront, with the arithmetic of factor_front_lds (pivot,
// rank-1 update of the trailing lower part, column scaling); the steps are
// separated by wavefront barriers only (the LDS operations of one wavefront
// complete in order).
template <typename T>
__device__ inline void factor_tile_wave(T *F, int32_t r, int32_t k, const int8_t *__restrict__ kd_s, double eps,
                                        double dyn, int32_t *nreg, T &dsh) {
    const int lane = threadIdx.x & 63;
    for (int32_t jj = 0; jj < k; ++jj) {
        if (lane == 0) {
            const T d = regularize(F[jj * r + jj], kd_s[jj], eps, dyn, nreg);
            F[jj * r + jj] = d;
            dsh = d;
        }
        __builtin_amdgcn_wave_barrier();
        const T d = dsh;
        const int32_t R = r - jj - 1;
        for (int32_t idx = lane; idx < R * R; idx += 64) {
            const int32_t i = jj + 1 + idx % R, cc = jj + 1 + idx / R;
            if (i >= cc) F[cc * r + i] -= F[jj * r + i] * F[jj * r + cc] / d;
        }
        __builtin_amdgcn_wave_barrier();
        for (int32_t i = jj + 1 + lane; i < r; i += 64) F[jj * r + i] /= d;
        __builtin_amdgcn_wave_barrier();
    }
}

// Small fronts of a level whose fronts all have at most CHAIN_R rows and 12 on
// average: one wavefront per front, four per workgroup, each front (assembled
// in the front storage by the level's gather) in its own LDS tile.  The same
// arithmetic as factor_small, a quarter of the workgroups and no workgroup
// barriers.  (On levels of larger fronts, 16 rows and more on average, the
// workgroup per front of factor_small was measured faster.)
template <typename T>
__global__ void __launch_bounds__(256) factor_small_wave(
    int32_t nfront, const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, T *__restrict__ front,
    const int8_t *__restrict__ kind, double eps, double dyn, int32_t *nreg) {
    __shared__ T tile[4][CHAIN_R * CHAIN_R];
    __shared__ T dsh[4];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int32_t q = blockIdx.x * 4 + w;
    if (q >= nfront) return;                         // whole wavefront
    const int32_t s = sn_list[q];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - sn_first[s];
    T *F = tile[w];
    T *G = front + fr_off[s];
    const int32_t rr = r * r;
    T g[CHAIN_R * CHAIN_R / 64];                     // all loads in flight at once
#pragma unroll
    for (int u = 0; u < CHAIN_R * CHAIN_R / 64; ++u) g[u] = ld_or0(G, lane + 64 * u, lane + 64 * u < rr);
#pragma unroll
    for (int u = 0; u < CHAIN_R * CHAIN_R / 64; ++u) {
        const int32_t idx = lane + 64 * u;
        if (idx < rr) F[idx] = (idx % r >= idx / r) ? g[u] : T(0);
    }
    __builtin_amdgcn_wave_barrier();
    factor_tile_wave<T>(F, r, k, kind + sn_first[s], eps, dyn, nreg, dsh[w]);
    for (int32_t idx = lane; idx < rr; idx += 64) {
        const int32_t i = idx % r, cc = idx / r;
        if (i >= cc) G[idx] = F[idx];
    }
}

// Tiny fronts (r <= TR, TR = TINY_R8 or TINY_R, one launch for each):
// 16 lanes per front, 16 fronts per workgroup, each front (assembled in the
// front storage by the level's gather) in its own TR x TR LDS tile, with the
// arithmetic of factor_front_lds.  The four fronts of a wavefront run their
// pivot loops together (masked past a front's own pivot count); a wavefront's
// LDS operations complete in order, so the steps need no barrier.  (With
// 16 x 16 tiles a workgroup holds 32 KB of LDS and five fit on a compute unit;
// most leaf fronts of nested dissection, about four rows, take 8 x 8.)
template <typename T, int TR>
__global__ void __launch_bounds__(256) factor_tiny(
    int32_t nfront, const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, T *__restrict__ front,
    const int8_t *__restrict__ kind, double eps, double dyn, int32_t *nreg) {
    static_assert(TR <= TINY_R && TR * TR % 16 == 0, "tile of the lane-group fronts");
    __shared__ T tile[16][TR * TR];   // sized for the level's largest front: more workgroups per CU
    __shared__ T dsh[16];
    const int g = threadIdx.x >> 4, gl = threadIdx.x & 15;
    const int32_t q = blockIdx.x * 16 + g;
    const bool has = q < nfront;
    const int32_t s = has ? sn_list[q] : 0;
    const int32_t r = has ? (int32_t)(sn_rptr[s + 1] - sn_rptr[s]) : 0;
    const int32_t k = has ? sn_first[s + 1] - sn_first[s] : 0;
    T *F = tile[g];
    T *G = front + (has ? fr_off[s] : 0);
    const int8_t *kd_s = kind + (has ? sn_first[s] : 0);
    const int32_t rr = r * r;
    T v[TR * TR / 16];                               // all loads in flight at once
#pragma unroll
    for (int u = 0; u < TR * TR / 16; ++u) v[u] = ld_or0(G, gl + 16 * u, gl + 16 * u < rr);
#pragma unroll
    for (int u = 0; u < TR * TR / 16; ++u) {
        const int32_t idx = gl + 16 * u;
        if (idx < rr) F[idx] = (idx % r >= idx / r) ? v[u] : T(0);
    }
    __builtin_amdgcn_wave_barrier();
    for (int32_t jj = 0; jj < k; ++jj) {
        if (gl == 0) {
            const T d = regularize(F[jj * r + jj], kd_s[jj], eps, dyn, nreg);
            F[jj * r + jj] = d;
            dsh[g] = d;
        }
        __builtin_amdgcn_wave_barrier();
        const T d = dsh[g];
        const int32_t R = r - jj - 1;
        for (int32_t idx = gl; idx < R * R; idx += 16) {
            const int32_t i = jj + 1 + idx % R, cc = jj + 1 + idx / R;
            if (i >= cc) F[cc * r + i] -= F[jj * r + i] * F[jj * r + cc] / d;
        }
        __builtin_amdgcn_wave_barrier();
        for (int32_t i = jj + 1 + gl; i < r; i += 16) F[jj * r + i] /= d;
        __builtin_amdgcn_wave_barrier();
    }
    for (int32_t idx = gl; idx < rr; idx += 16) {
        const int32_t i = idx % r, cc = idx / r;
        if (i >= cc) G[idx] = F[idx];
    }
}

// Chains (the narrow upper levels of deep elimination trees): one workgroup
// per component walks the component's levels; the fronts of a level are
// factored one per wavefront, each in its own LDS tile, with the same
// arithmetic as factor_small (pivot, rank-1 update of the trailing lower
// part, column scaling), the steps separated by wavefront barriers only (the
// LDS operations of one wavefront complete in order).  A front is assembled
// in its tile from the entries of the numeric assembly map (the same sources
// in the same order as gather_entries: the K entry, the static regularization
// of a pivot diagonal, then the children's update entries).  Children below
// the chain levels were factored by the level kernels before this launch;
// children inside the component by this workgroup, before the workgroup
// barrier that ends their level.  (Keeping one row per lane in registers was
// measured slower: the update of a 32-row front then costs each lane up to 31
// divisions per pivot instead of about R*R/128.)
template <typename T>
__global__ void __launch_bounds__(256) factor_chain(
    const int32_t *__restrict__ comp_ptr, const int32_t *__restrict__ grp_ptr, const int32_t *__restrict__ chain_sn,
    const int64_t *__restrict__ ent_front, const int64_t *__restrict__ dst, const int64_t *__restrict__ sptr,
    const int8_t *__restrict__ reg, const int64_t *__restrict__ src, const double *__restrict__ kval,
    double delta, const int32_t *__restrict__ sn_first, const int64_t *__restrict__ sn_rptr,
    const int64_t *__restrict__ fr_off, T *__restrict__ front, const int8_t *__restrict__ kind, double eps,
    double dyn, int32_t *nreg) {
    __shared__ T tile[4][CHAIN_R * CHAIN_R];
    __shared__ T dsh[4];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: the front indices below too
    const int lane = threadIdx.x & 63;
    T *F = tile[w];
    const int32_t c = blockIdx.x;
    for (int32_t g = comp_ptr[c]; g < comp_ptr[c + 1]; ++g) {
        for (int32_t t = grp_ptr[g] + w; t < grp_ptr[g + 1]; t += 4) {
            const int32_t s = chain_sn[t];
            const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
            const int32_t k = sn_first[s + 1] - sn_first[s];
            const int64_t base = fr_off[s];
            const int8_t *kd_s = kind + sn_first[s];
            for (int32_t idx = lane; idx < r * r; idx += 64) F[idx] = T(0);
            __builtin_amdgcn_wave_barrier();
            for (int64_t e = ent_front[2 * s] + lane; e < ent_front[2 * s + 1]; e += 64) {
                int64_t u = sptr[e];
                const int64_t u1 = sptr[e + 1];
                T v = T(0);
                if (u < u1) {
                    const int64_t s0 = src[u];
                    if (s0 < 0) { v = (T)kval[-s0 - 1]; ++u; }
                }
                const int8_t kd = reg[e];
                if (kd >= 0) v = (T)((double)v + static_reg(kd, delta));
                for (; u < u1; ++u) v += front[src[u]];
                F[dst[e] - base] = v;
            }
            __builtin_amdgcn_wave_barrier();
            factor_tile_wave<T>(F, r, k, kd_s, eps, dyn, nreg, dsh[w]);
            T *G = front + base;
            for (int32_t idx = lane; idx < r * r; idx += 64) {
                const int32_t i = idx % r, cc = idx / r;
                if (i >= cc) G[idx] = F[idx];
            }
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// large fronts
// ---------------------------------------------------------------------------
// Reciprocal of a pivot: the hardware reciprocal (1 ulp) for FP32 factors,
// whose errors the FP64 refinement removes; correctly rounded for FP64.
__device__ inline float recip(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ inline double recip(double d) { return 1.0 / d; }


// One 16 x 16 tile of C = sum_k A(i, k) B(k, j), k = 0..15, on MFMA 16x16x4:
// a(i, k) and b(k, j) return the operands; the result is in the lane layout
// of mfma_out_row (row mfma_out_row(lane / 16, v), column lane % 16).
template <typename T, typename FA, typename FB>
__device__ inline typename Acc4<T>::type tile16(FA a, FB b) {
    const int lane = threadIdx.x & 63;
    const int i = lane & 15, kq = lane >> 4;
    typename Acc4<T>::type acc = {0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) acc = mfma16x16x4(a(i, k0 + kq), b(k0 + kq, i), acc);
    return acc;
}

// LDL' of the b x b diagonal block at (j0, j0) of the front F (ld r), in
// place; the inverse of its unit lower factor goes to Xg (ld NB, zeros above
// the diagonal).  The block is staged in LDS and factored 16 columns at a
// time.  Wavefront 0 holds the rows of the block from the sub-block down in
// registers (lane i holds row i) and runs the 16 pivot steps on them, reading
// each pivot column with lane broadcasts, so a pivot step has no barrier and
// the rows below the sub-block come out as rows of L at no extra cost.  Then
// wavefront 3 inverts the sub-block's unit lower factor while wavefronts 0-2
// apply its rank-16 update to the rest of the block on 16 x 16 MFMA tiles.
// The inverse of the whole unit lower factor is assembled from the 16 x 16
// inverses, X_pq = -X_pp sum_{m=q}^{p-1} L_pm X_mq on MFMA tiles: block row p
// by wavefronts 1..p while wavefront 0 pivots sub-block p + 1, the last block
// row at the end.
template <typename T>
__global__ void __launch_bounds__(256) diag_block(T *__restrict__ F, int32_t r, int32_t j0, int32_t b,
                                                  const int8_t *__restrict__ kind_cols, double eps,
                                                  double dyn, int32_t *nreg, T *__restrict__ Xg, CopyStride cs) {
    F += blockIdx.z * cs.f;
    kind_cols += blockIdx.z * cs.col;
    Xg += blockIdx.z * cs.dinv;
    // the panel chain is the critical path of a large front: its waves win issue
    // arbitration against the concurrent bulk update on a shared compute unit
    __builtin_amdgcn_s_setprio(3);
    constexpr int LD = NB + 1;           // padded leading dimension of the LDS tiles
    constexpr int PB = 16;               // sub-block width
    __shared__ T S[NB * LD];             // S[c * LD + i]: block, becomes L (strictly lower) and D (diagonal)
    __shared__ T X[NB * LD];             // inverse of the unit lower factor
    __shared__ T Tm[4][PB * PB];         // partial sums of off-diagonal inverse blocks, one per wavefront
    __shared__ T Dd[NB];
    __shared__ double sgn[NB];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    {
        T v[NB * NB / 256];
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int idx = tid + 256 * u, i = idx & 63, c = idx >> 6;
            v[u] = ld_or0(F, (int64_t)(j0 + c) * r + j0 + i, i < b && c < b && i >= c);
        }
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int idx = tid + 256 * u, i = idx & 63, c = idx >> 6;
            S[c * LD + i] = v[u];
            X[c * LD + i] = T(0);
        }
    }
    if (tid < NB) sgn[tid] = tid < b ? pivot_sign(kind_cols[j0 + tid]) : 1.0;
    __syncthreads();
    int events = 0;
    const int lr = lane & 15, lk = lane >> 4;
    // off-diagonal block X_pq (p > q) of the inverse, by the calling wavefront:
    // X_pq = -X_pp sum_{m=q}^{p-1} L_pm X_mq (block row p's diagonal block and the
    // block rows above it are complete)
    auto x_block = [&](int p, int q) {
        const int n = PB * p, q0 = PB * q;
        typename Acc4<T>::type tacc = {0, 0, 0, 0};
        for (int m0 = q0; m0 < n; m0 += PB) {
            auto acc = tile16<T>([&](int i, int k) { return S[(m0 + k) * LD + n + i]; },
                                 [&](int k, int j) { return X[(q0 + j) * LD + m0 + k]; });
#pragma unroll
            for (int v = 0; v < 4; ++v) tacc[v] += acc[v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Tm[wave][lr * PB + mfma_out_row<T>(lk, v)] = tacc[v];   // T(row, col) at col * 16 + row
        __builtin_amdgcn_wave_barrier();
        auto acc = tile16<T>([&](int i, int k) { return X[(n + k) * LD + n + i]; },
                             [&](int k, int j) { return Tm[wave][j * PB + k]; });
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = n + mfma_out_row<T>(lk, v), j = q0 + lr;
            if (i < b && j < b) X[j * LD + i] = -acc[v];
        }
    };
    for (int p0 = 0; p0 < b; p0 += PB) {
        const int pb = min(PB, b - p0);
        const int ps = p0 / PB;
        if (wave == 0) {
            // lane i: row i, entries in the sub-block's columns p0 .. p0 + 15 (lower part only)
            const int i = lane;
            const bool row_ok = i >= p0 && i < b;
            T a[PB];
#pragma unroll
            for (int m = 0; m < PB; ++m) {
                const T v = S[(p0 + m) * LD + i];
                a[m] = (row_ok && m < pb && i >= p0 + m) ? v : T(0);
            }
            T dmine = T(0);
            double sgv[PB];                            // pivot signs, read before the pivot chain
#pragma unroll
            for (int j = 0; j < PB; ++j) sgv[j] = sgn[p0 + j];
#pragma unroll
            for (int j = 0; j < PB; ++j) {
                if (j < pb) {
                    const int c = p0 + j;
                    const T raw = lane_bcast(a[j], c);
                    const double sg = sgv[j];
                    const bool fix = !(sg * (double)raw > eps);
                    const T d = fix ? (T)(sg * dyn) : raw;
                    events += fix ? 1 : 0;
                    const T inv = recip(d);
                    const T l = i > c ? a[j] * inv : T(0);
                    // A(i, p0 + k) -= L(i, c) A(p0 + k, c); entries above the diagonal are never read
#pragma unroll
                    for (int k = j + 1; k < PB; ++k) a[k] -= l * lane_bcast(a[j], p0 + k);
                    a[j] = i > c ? l : (i == c ? d : a[j]);
                    dmine = i == c ? d : dmine;
                }
            }
            if (row_ok) {
                // columns beyond pb (a partial last sub-block) hold values that are never read
#pragma unroll
                for (int m = 0; m < PB; ++m) S[(p0 + m) * LD + i] = i >= p0 + m ? a[m] : T(0);
                if (i < p0 + pb) Dd[i] = dmine;
            }
        } else if (wave < ps) {
            // meanwhile: block row ps - 1 of the inverse (its diagonal block is done)
            x_block(ps - 1, wave - 1);
        }
        __syncthreads();
        const int i0 = p0 + pb, nb = b - i0;
        if (wave == 3) {
            // inverse of the unit lower sub-block: lane c forms column c by forward
            // substitution; the 120 entries of L it needs are read from LDS up front
            // (broadcast reads, all in flight), so the substitution is a register chain
            T lc[PB][PB];
#pragma unroll
            for (int m = 0; m < PB; ++m)
#pragma unroll
                for (int k = m + 1; k < PB; ++k) lc[m][k] = S[(p0 + m) * LD + p0 + k];
            T x[PB];
#pragma unroll
            for (int k = 0; k < PB; ++k) x[k] = (k == lr) ? T(1) : T(0);
#pragma unroll
            for (int m = 0; m < PB; ++m)
#pragma unroll
                for (int k = m + 1; k < PB; ++k) x[k] -= ((k < pb && m < pb) ? lc[m][k] : T(0)) * x[m];
            if (lane < pb) {
#pragma unroll
                for (int k = 0; k < PB; ++k)
                    if (k < pb && k >= lane) X[(p0 + lane) * LD + p0 + k] = x[k];
            }
        } else if (nb > 0) {
            // rank-pb update of the rest of the block: tiles (ti, tj), ti >= tj
            const int nt = (nb + 15) / 16;
            for (int tt = wave; tt < nt * (nt + 1) / 2; tt += 3) {
                int ti = 0;
                while ((ti + 1) * (ti + 2) / 2 <= tt) ++ti;
                const int tj = tt - ti * (ti + 1) / 2;
                const int ri = i0 + 16 * ti, rj = i0 + 16 * tj;
                auto acc = tile16<T>(
                    [&](int i, int k) { return k < pb ? S[(p0 + k) * LD + ri + i] : T(0); },
                    [&](int k, int j) { return k < pb ? S[(p0 + k) * LD + rj + j] * Dd[p0 + k] : T(0); });
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = ri + mfma_out_row<T>(lk, v), j = rj + lr;
                    if (i < b && j < b && i >= j) S[j * LD + i] -= acc[v];
                }
            }
        }
        __syncthreads();
    }
    // the last block row of the inverse (the earlier ones were formed during the pivot phases)
    const int last = (b + PB - 1) / PB - 1;
    if (wave < last) x_block(last, wave);
    __syncthreads();
    if (tid == 0 && events) atomicAdd(nreg, events);
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
        const int idx = tid + 256 * u, i = idx & 63, c = idx >> 6;
        if (i < b && c < b && i >= c) F[(int64_t)(j0 + c) * r + j0 + i] = S[c * LD + i];
        Xg[c * NB + i] = (i < b && c < b && i >= c) ? X[c * LD + i] : T(0);
    }
}

// Inverse of the unit-lower SB x SB diagonal block of a super-panel
// [J0, J0+kb) from the inverses X_ii of its 64 x 64 diagonal blocks:
// X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj (i > j).  Workgroup j computes block
// column j (independent of the other columns), block row by block row; the
// 64 x 64 products run on MFMA 16x16x4 with operands staged through LDS
// (wavefront w forms rows 16 w .. 16 w + 15).  Writes X and X'
// (column-major, leading dimension ld = kb rounded up to a multiple of 64).
template <typename T>
__global__ void __launch_bounds__(256) sblock_inverse(const T *__restrict__ F, int32_t r, int32_t J0, int32_t kb,
                                                      const T *__restrict__ dinv_s, int32_t ld,
                                                      T *__restrict__ Xs, T *__restrict__ XTs, CopyStride cs) {
    F += blockIdx.z * cs.f;
    dinv_s += blockIdx.z * cs.dinv;
    Xs += blockIdx.z * cs.sinv;
    XTs += blockIdx.z * cs.sinv;
    constexpr int LD = NB + 1;
    __shared__ T A[NB * LD];         // A[k * LD + i] = operand A(i, k)
    __shared__ T B[NB * LD];         // B[j * LD + k] = operand B(k, j)
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
    const int32_t j = blockIdx.x;
    const int32_t nsub = (kb + NB - 1) / NB;
    const int32_t bj = min(NB, kb - j * NB);
    typedef typename Acc4<T>::type V;
    // X_jj
    const T *Xjj = dinv_s + (int64_t)((J0 + j * NB) / NB) * NB * NB;
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int cc = lane, rr = wave + 4 * m;
        const T v = Xjj[cc * NB + rr];
        Xs[(int64_t)(j * NB + cc) * ld + j * NB + rr] = v;
        XTs[(int64_t)(j * NB + rr) * ld + j * NB + cc] = v;
    }
    for (int32_t i = j + 1; i < nsub; ++i) {
        // X_jj, and the X_{i-1,j} stored at the end of the previous pass, were written by other
        // wavefronts of this workgroup and are read below
        __syncthreads();
        const int32_t bi = min(NB, kb - i * NB);
        V acc[4];
#pragma unroll
        for (int bc = 0; bc < 4; ++bc) acc[bc] = V{0, 0, 0, 0};
        for (int32_t k = j; k < i; ++k) {
            const int32_t bk = min(NB, kb - k * NB);
            T la[NB * NB / 256], lb[NB * NB / 256];
#pragma unroll
            for (int u = 0; u < NB * NB / 256; ++u) {
                const int32_t idx = tid + 256 * u, e = idx & 63, f = idx >> 6;
                la[u] = ld_or0(F, (int64_t)(J0 + k * NB + f) * r + J0 + i * NB + e, e < bi && f < bk);   // L_ik(e, f)
                lb[u] = ld_or0(Xs, (int64_t)(j * NB + f) * ld + k * NB + e, e < bk && f < bj);          // X_kj(e, f)
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < NB * NB / 256; ++u) {
                const int32_t idx = tid + 256 * u, e = idx & 63, f = idx >> 6;
                A[f * LD + e] = la[u];       // A(e, f) = L_ik(e, f)
                B[f * LD + e] = lb[u];       // B(e, f) = X_kj(e, f)
            }
            __syncthreads();
#pragma unroll 4
            for (int k0 = 0; k0 < NB; k0 += 4) {
                const T a = A[(k0 + lk) * LD + 16 * wave + lr];
#pragma unroll
                for (int bc = 0; bc < 4; ++bc) acc[bc] = mfma16x16x4(a, B[(16 * bc + lr) * LD + k0 + lk], acc[bc]);
            }
        }
        // X_ij = -X_ii S with S = acc (rows 16 wave + mfma_out_row, columns 16 bc + lr)
        __syncthreads();
        const T *Xii = dinv_s + (int64_t)((J0 + i * NB) / NB) * NB * NB;
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int32_t idx = tid + 256 * u, e = idx & 63, f = idx >> 6;
            A[f * LD + e] = Xii[f * NB + e];                 // A(e, f) = X_ii(e, f)
        }
#pragma unroll
        for (int bc = 0; bc < 4; ++bc)
#pragma unroll
            for (int v = 0; v < 4; ++v) B[(16 * bc + lr) * LD + 16 * wave + mfma_out_row<T>(lk, v)] = acc[bc][v];
        __syncthreads();
        V out[4];
#pragma unroll
        for (int bc = 0; bc < 4; ++bc) out[bc] = V{0, 0, 0, 0};
#pragma unroll 4
        for (int k0 = 0; k0 < NB; k0 += 4) {
            const T a = A[(k0 + lk) * LD + 16 * wave + lr];
#pragma unroll
            for (int bc = 0; bc < 4; ++bc) out[bc] = mfma16x16x4(a, B[(16 * bc + lr) * LD + k0 + lk], out[bc]);
        }
#pragma unroll
        for (int bc = 0; bc < 4; ++bc)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = 16 * wave + mfma_out_row<T>(lk, v), cc = 16 * bc + lr;
                const T val = (rr < bi && cc < bj) ? -out[bc][v] : T(0);
                Xs[(int64_t)(j * NB + cc) * ld + i * NB + rr] = val;
                XTs[(int64_t)(i * NB + rr) * ld + j * NB + cc] = val;
            }
    }
}

// L21 = A21 X' D^-1 for 64 rows per workgroup (rows j0+b .. r-1): the 64 x b
// tile of A21 and X are staged through LDS with coalesced loads (all in
// flight at once); the product runs on MFMA 16x16x4, formed transposed
// (X A21', wavefront w forms panel columns 16 w .. 16 w + 15) so that lanes
// run along the contiguous rows of the front in the store.
template <typename T>
__global__ void __launch_bounds__(256) panel_solve(T *__restrict__ F, int32_t r, int32_t j0, int32_t b,
                                                   const T *__restrict__ Xg, CopyStride cs) {
    F += blockIdx.z * cs.f;
    Xg += blockIdx.z * cs.dinv;
    __builtin_amdgcn_s_setprio(3);                      // panel chain: see diag_block
    constexpr int XP = sizeof(T) == 4 ? NB + 16 : NB;   // pitch: MFMA operand rows on disjoint banks
    __shared__ T Xs[NB * XP];        // Xs[t * XP + c] = X(c, t)
    __shared__ T As[NB * (NB + 1)];  // As[t * (NB + 1) + i] = A21(row0 + i, t)
    __shared__ T Ds[NB];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, lr = lane & 15, lk = lane >> 4;
    const int32_t row0 = j0 + b + blockIdx.x * 64;
    {
        T xv[NB * NB / 256], av[NB * NB / 256];
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int32_t idx = tid + 256 * u, i = idx & 63, t = idx >> 6;
            xv[u] = Xg[idx];
            av[u] = ld_or0(F, (int64_t)(j0 + t) * r + row0 + i, row0 + i < r && t < b);
        }
#pragma unroll
        for (int u = 0; u < NB * NB / 256; ++u) {
            const int32_t idx = tid + 256 * u, i = idx & 63, t = idx >> 6;
            Xs[t * XP + i] = xv[u];
            As[t * (NB + 1) + i] = av[u];
        }
    }
    if (tid < NB) Ds[tid] = ld_or0(F, (int64_t)(j0 + tid) * r + j0 + tid, tid < b);
    __syncthreads();
    typedef typename Acc4<T>::type V;
    V acc[4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) acc[bi] = V{0, 0, 0, 0};
#pragma unroll 4
    for (int k0 = 0; k0 < NB; k0 += 4) {
        const T a = Xs[(k0 + lk) * XP + 16 * wave + lr];                  // X(c, t): c = 16 w + lr, t = k0 + lk
#pragma unroll
        for (int bi = 0; bi < 4; ++bi) acc[bi] = mfma16x16x4(a, As[(k0 + lk) * (NB + 1) + 16 * bi + lr], acc[bi]);
    }
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int c = 16 * wave + mfma_out_row<T>(lk, v);
            const int32_t row = row0 + 16 * bi + lr;
            if (row < r && c < b) F[(int64_t)(j0 + c) * r + row] = acc[bi][v] / Ds[c];
        }
}

// Raw buffer resource over nbytes from p, built from wave-uniform values (so
// it lives in scalar registers and every access is a single instruction): a
// load at a byte offset >= nbytes returns 0 and a store there is dropped by the
// hardware range check.  Word 3 selects the 32-bit data format (4 in bits
// 15..18 of a gfx9-family descriptor).
__device__ inline __amdgpu_buffer_rsrc_t uniform_rsrc(const void *p, int32_t nbytes) {
    const uint64_t a = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    return __builtin_amdgcn_make_buffer_rsrc((void *)(((uint64_t)hi << 32) | lo), (short)0,
                                             __builtin_amdgcn_readfirstlane(nbytes), 0x00020000);
}
// byte offset past every range: marks a lane or entry whose access must read 0 / store nothing.  With
// fronts of at most MAX_FRONT_R rows the ranges (at most 32 columns of 8-byte or 64 columns of 4-byte
// entries) and every valid offset stay below it, and it plus the largest in-chunk step stays below 2^32.
constexpr uint32_t OFF_NONE = 0x80000000u;
template <typename T> __device__ inline T buffer_load(__amdgpu_buffer_rsrc_t rs, uint32_t off);
template <> __device__ inline float buffer_load<float>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)off, 0, 0));
}
template <> __device__ inline double buffer_load<double>(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0));
}
template <typename T> __device__ inline void buffer_store(__amdgpu_buffer_rsrc_t rs, uint32_t off, T v);
template <> __device__ inline void buffer_store<float>(__amdgpu_buffer_rsrc_t rs, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), rs, (int)off, 0, 0);
}
template <> __device__ inline void buffer_store<double>(__amdgpu_buffer_rsrc_t rs, uint32_t off, double v) {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rs, (int)off, 0, 0);
}

// C -= L(:, k0:k0+kb) D L(cols, k0:k0+kb)' on the lower part (row >= col) of
// rows [r_lo, r) x cols [r_lo, c_hi) of the front F (ld r), 64 x 64 tiles,
// 1-D grid (see the XCD mapping below).  The rank kb is consumed in chunks of
// KC = 16 columns through double-buffered LDS: the global loads of the next
// chunk are issued before the MFMAs of the current one and are only waited
// for at the LDS store; the old C values are loaded after the last chunk.
// Four wavefronts per tile, 2 x 2 MFMA 16x16x4 blocks each; the product is
// formed transposed so that each lane's accumulators run along a column of
// the column-major front.  Global accesses are buffer instructions on
// wave-uniform resources, as in trail_update_big below: rank columns past kb
// and rows past the end read 0, C entries outside the update are neither
// read nor written.
template <typename T>
__global__ void __launch_bounds__(256) trail_update(T *__restrict__ F, int32_t r, int32_t k0, int32_t kb,
                                                   int32_t r_lo, int32_t c_hi, int32_t urgent, int64_t zstride) {
    F += blockIdx.z * zstride;
    constexpr int KC = 16;
    constexpr int PER = KC / 4;                    // rank columns staged per thread and chunk
    constexpr uint32_t S = sizeof(T);
    // row pitch of the LDS tiles: the four 16-lane groups of an MFMA operand read rows kk .. kk+3;
    // for 4-byte entries a pitch of 80 puts them on disjoint banks
    constexpr int LDT = sizeof(T) == 4 ? 80 : 64;
    __shared__ T As[2][KC * LDT];                  // As[kk * LDT + i] = L(r0 + i, k)
    __shared__ T Bs[2][KC * LDT];                  // Bs[kk * LDT + j] = L(c0 + j, k) * D(k)
    __shared__ T Dk[OB];                           // D(k0 .. k0 + kb - 1), zero past the rank (kb <= OB)
    // Workgroup IDs are dealt to the 8 XCDs in turn; XCD x takes the tile rows ti = x (mod 8)
    // and walks them column tile by column tile, so its concurrent workgroups share the column
    // panel and keep their row panels in that XCD's L2.
    const int32_t TR = (r - r_lo + 63) / 64, TC = (c_hi - r_lo + 63) / 64, NR = (TR + 7) / 8;
    const int32_t xcd = blockIdx.x % 8, sq = blockIdx.x / 8;
    const int32_t tj = sq / NR, ti = (sq % NR) * 8 + xcd;
    if (ti >= TR || tj >= TC || ti < tj) return;   // outside the grid or strictly above the diagonal
    if (urgent) __builtin_amdgcn_s_setprio(2);     // on the panel chain: ahead of the bulk update's waves
    const int32_t r0 = r_lo + 64 * ti, c0 = r_lo + 64 * tj;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    typedef typename Acc4<T>::type V;
    const int32_t i = tid & 63;
    const int kk0 = tid >> 6;                      // this thread stages rank columns kk0, kk0 + 4, ...
    const uint32_t offa = r0 + i < r ? (uint32_t)(kk0 * r + r0 + i) * S : OFF_NONE;
    const uint32_t offb = c0 + i < c_hi ? (uint32_t)(kk0 * r + c0 + i) * S : OFF_NONE;
    const uint32_t ustep = 4u * (uint32_t)r * S;   // four columns
    T ra[PER], rb[PER];
    auto gload = [&](int32_t kc) {
        const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(F + (int64_t)(k0 + kc) * r, min(KC, kb - kc) * r * (int32_t)S);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            ra[u] = buffer_load<T>(rs, offa + u * ustep);
            rb[u] = buffer_load<T>(rs, offb + u * ustep);
        }
    };
    auto lstore = [&](int buf, int32_t kc) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int32_t kk = kk0 + 4 * u;
            As[buf][kk * LDT + i] = ra[u];
            Bs[buf][kk * LDT + i] = rb[u] * Dk[kc + kk];
        }
    };
    V acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = V{0, 0, 0, 0};
    const int32_t nch = (kb + KC - 1) / KC;
    for (int32_t t = tid; t < OB; t += 256) Dk[t] = t < kb ? F[(int64_t)(k0 + t) * r + k0 + t] : T(0);
    gload(0);
    __syncthreads();
    lstore(0, 0);
    __syncthreads();
    for (int32_t c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) gload((c + 1) * KC);
#pragma unroll
        for (int32_t kk = 0; kk < KC; kk += 4) {       // zero-padded past the rank
            const int32_t kq = kk + lk;
            T a_op[2], b_op[2];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) a_op[bj] = Bs[buf][kq * LDT + wc + 16 * bj + lr];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) b_op[bi] = As[buf][kq * LDT + wr + 16 * bi + lr];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma16x16x4(a_op[bj], b_op[bi], acc[bi][bj]);
        }
        if (c + 1 < nch) lstore(buf ^ 1, (c + 1) * KC);
        __syncthreads();
    }
    // lane holds C(row = wr + 16 bi + lr, col = wc + 16 bj + mfma_out_row(lk, v)); the resource spans the
    // wavefront's valid columns, entries below the last row or above the diagonal point past it
    const int32_t cq = c0 + wc;
    if (cq >= c_hi) return;
    const __amdgpu_buffer_rsrc_t rc = uniform_rsrc(F + (int64_t)cq * r, min(32, c_hi - cq) * r * (int32_t)S);
    uint32_t off[2][2][4];
    T cold[2][2][4];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t row = r0 + wr + 16 * bi + lr;
                const int32_t cl = 16 * bj + mfma_out_row<T>(lk, v);
                off[bi][bj][v] = (row < r && row >= cq + cl) ? (uint32_t)(cl * r + row) * S : OFF_NONE;
                cold[bi][bj][v] = buffer_load<T>(rc, off[bi][bj][v]);
            }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) buffer_store<T>(rc, off[bi][bj][v], cold[bi][bj][v] - acc[bi][bj][v]);
}

// The same update (FP32) on 128 x 128 tiles, for the large launches (the
// rank-SB updates of a super-panel across the rest of the front).  Each
// wavefront owns a 64 x 64 quarter as 4 x 4 MFMA 16x16x4 blocks, so every
// operand read from LDS feeds four MFMAs and every entry of the two panel
// blocks staged per chunk serves 128 rows or columns.  The rank is consumed in
// chunks of KC = 16 columns through double-buffered LDS (38 KB per workgroup,
// four workgroups per compute unit), the global loads of the next chunk in
// flight during the MFMAs of the current one; C is read once, after the last
// chunk.  All global accesses are buffer instructions on a resource in scalar
// registers: a chunk's resource spans exactly its valid rank columns, so
// columns past the rank read 0, and lanes on rows past the end point beyond
// every range (OFF_NONE), so no address arithmetic or select sits in the loop.
// On a diagonal tile the quarter strictly above the diagonal computes products
// it never stores.
__global__ void __launch_bounds__(256, 3) trail_update_big(float *__restrict__ F, int32_t r, int32_t k0, int32_t kb,
                                                          int32_t r_lo, int32_t c_hi, int32_t urgent,
                                                          int64_t zstride) {
    F += blockIdx.z * zstride;
    constexpr int TILE = 128;
    constexpr int KC = 16;
    constexpr int PER = KC * TILE / 256;           // rank columns staged per thread and chunk (8)
    // row pitch of the LDS tiles: the four 16-lane groups of an MFMA operand read rows kk .. kk+3;
    // a pitch of 144 (16 mod 32 banks) puts each half-wavefront on disjoint banks
    constexpr int LDT = TILE + 16;
    __shared__ float As[2][KC * LDT];              // As[kk * LDT + i] = L(r0 + i, k)
    __shared__ float Bs[2][KC * LDT];              // Bs[kk * LDT + j] = L(c0 + j, k) * D(k)
    __shared__ float Dk[OB];                       // D(k0 .. k0 + kb - 1), zero past the rank (kb <= OB)
    // XCD-aware order as in trail_update: XCD x takes the tile rows ti = x (mod 8)
    const int32_t TR = (r - r_lo + TILE - 1) / TILE, TC = (c_hi - r_lo + TILE - 1) / TILE, NR = (TR + 7) / 8;
    const int32_t xcd = blockIdx.x % 8, sq = blockIdx.x / 8;
    const int32_t tj = sq / NR, ti = (sq % NR) * 8 + xcd;
    if (ti >= TR || tj >= TC || ti < tj) return;
    if (urgent) __builtin_amdgcn_s_setprio(2);     // on the panel chain: ahead of the bulk update's waves
    const int32_t r0 = r_lo + TILE * ti, c0 = r_lo + TILE * tj;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
    const int lr = lane & 15, lk = lane >> 4;
    // this quarter stores results unless it lies beyond the last row or column, or strictly above the diagonal
    const bool active = r0 + wr < r && c0 + wc < c_hi && r0 + wr + 63 >= c0 + wc;
    typedef typename Acc4<float>::type V;
    const int32_t i = tid & (TILE - 1);
    const int kk0 = tid >> 7;                      // 0 or 1: this thread stages rank columns kk0, kk0 + 2, ...
    // byte offsets of this thread's first staged entries within a chunk (column kk0 of the chunk)
    const uint32_t offa = r0 + i < r ? (uint32_t)(kk0 * r + r0 + i) * 4u : OFF_NONE;
    const uint32_t offb = c0 + i < c_hi ? (uint32_t)(kk0 * r + c0 + i) * 4u : OFF_NONE;
    const uint32_t ustep = 8u * (uint32_t)r;       // two columns
    float ra[PER], rb[PER];
    auto gload = [&](int32_t kc) {
        const __amdgpu_buffer_rsrc_t rs = uniform_rsrc(F + (int64_t)(k0 + kc) * r, min(KC, kb - kc) * r * 4);
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            ra[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(offa + u * ustep), 0, 0));
            rb[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, (int)(offb + u * ustep), 0, 0));
        }
    };
    auto lstore = [&](int buf, int32_t kc) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int32_t kk = kk0 + 2 * u;
            As[buf][kk * LDT + i] = ra[u];
            Bs[buf][kk * LDT + i] = rb[u] * Dk[kc + kk];
        }
    };
    V acc[4][4];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = V{0, 0, 0, 0};
    const int32_t nch = (kb + KC - 1) / KC;
    for (int32_t t = tid; t < OB; t += 256) Dk[t] = t < kb ? F[(int64_t)(k0 + t) * r + k0 + t] : 0.f;
    gload(0);
    __syncthreads();
    lstore(0, 0);
    __syncthreads();
    for (int32_t c = 0; c < nch; ++c) {
        const int buf = c & 1;
        if (c + 1 < nch) gload((c + 1) * KC);
#pragma unroll
        for (int32_t kk = 0; kk < KC; kk += 4) {       // zero-padded past the rank
            const int32_t kq = kk + lk;
            float a_op[4], b_op[4];
#pragma unroll
            for (int bj = 0; bj < 4; ++bj) a_op[bj] = Bs[buf][kq * LDT + wc + 16 * bj + lr];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi) b_op[bi] = As[buf][kq * LDT + wr + 16 * bi + lr];
#pragma unroll
            for (int bi = 0; bi < 4; ++bi)
#pragma unroll
                for (int bj = 0; bj < 4; ++bj) acc[bi][bj] = mfma16x16x4(a_op[bj], b_op[bi], acc[bi][bj]);
        }
        if (c + 1 < nch) lstore(buf ^ 1, (c + 1) * KC);
        __syncthreads();
    }
    if (!active) return;
    // lane holds C(row = wr + 16 bi + lr, col = wc + 16 bj + mfma_out_row(lk, v)); 16 lanes load and store
    // 16 consecutive rows of one column.  The resource spans this quarter's valid columns; entries below
    // the last row or above the diagonal point past it.
    const int32_t cq = c0 + wc;
    const __amdgpu_buffer_rsrc_t rc = uniform_rsrc(F + (int64_t)cq * r, min(64, c_hi - cq) * r * 4);
#pragma unroll
    for (int bi = 0; bi < 4; ++bi) {
        const int32_t row = r0 + wr + 16 * bi + lr;
        uint32_t off[4][4];
        float cold[4][4];
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t cl = 16 * bj + mfma_out_row<float>(lk, v);
                off[bj][v] = (row < r && row >= cq + cl) ? (uint32_t)(cl * r + row) * 4u : OFF_NONE;
                cold[bj][v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rc, (int)off[bj][v], 0, 0));
            }
#pragma unroll
        for (int bj = 0; bj < 4; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, cold[bj][v] - acc[bi][bj][v]), rc,
                                                      (int)off[bj][v], 0, 0);
    }
}

// W_J = L(J1:r, J0:J1) X_J for a super-panel [J0, J1) (X_J the inverse of its
// unit-lower diagonal block, column-major with leading dimension ld), written
// column-major with leading dimension r - J1.  The solves use W_J: the forward
// update of the rows below the super-block is L(below, J) y_J = W_J v_J, which
// needs v_J only, and the backward pushes W_J' x onto the earlier blocks.
// 64 x 64 output tiles, grid (row tile, column tile); since X_J is lower
// triangular, column tile tc only needs ranks >= 64 tc.  MFMA 16x16x4, formed
// transposed so that lanes run along the rows of W in the store.
template <typename T>
__global__ void __launch_bounds__(256) wblock(const T *__restrict__ F, int32_t r, int32_t J0, int32_t kb,
                                             const T *__restrict__ Xs, int32_t ld, T *__restrict__ W,
                                             CopyStride cs) {
    F += blockIdx.z * cs.f;
    Xs += blockIdx.z * cs.sinv;
    W += blockIdx.z * cs.w;
    constexpr int KC = 32, PER = KC * 64 / 256;
    constexpr int AP = sizeof(T) == 4 ? 80 : 64;   // pitch: MFMA operand rows on disjoint banks
    __shared__ T As[KC * AP];          // As[kk * AP + i] = L(J1 + 64 ti + i, J0 + kc + kk)
    __shared__ T Bs[KC * 65];          // Bs[kk * 65 + j] = X(kc + kk, 64 tc + j)
    const int32_t J1 = J0 + kb, m = r - J1;
    const int32_t ti = blockIdx.x, tc = blockIdx.y;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int lr = lane & 15, lk = lane >> 4;
    typedef typename Acc4<T>::type V;
    V acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = V{0, 0, 0, 0};
    // the next chunk's loads are issued before the current chunk's products (one register stage)
    T av[PER], bv[PER];
    auto gload = [&](int32_t kc) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            const int i = e & 63, kk = e >> 6;                        // A: lanes along rows
            av[u] = ld_or0(F, (int64_t)(J0 + kc + kk) * r + J1 + 64 * ti + i, kc + kk < kb && 64 * ti + i < m);
            const int kb_ = e & (KC - 1), j = e / KC;                 // B: lanes along ranks
            bv[u] = ld_or0(Xs, (int64_t)(64 * tc + j) * ld + kc + kb_, kc + kb_ < kb && 64 * tc + j < kb);
        }
    };
    if (64 * tc < kb) gload(64 * tc);
    for (int32_t kc = 64 * tc; kc < kb; kc += KC) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + 256 * u;
            As[(e >> 6) * AP + (e & 63)] = av[u];
            Bs[(e & (KC - 1)) * 65 + e / KC] = bv[u];
        }
        __syncthreads();
        if (kc + KC < kb) gload(kc + KC);
#pragma unroll
        for (int kk = 0; kk < KC; kk += 4) {
            const int kq = kk + lk;
            T a_op[2], b_op[2];
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) a_op[bj] = Bs[kq * 65 + wc + 16 * bj + lr];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi) b_op[bi] = As[kq * AP + wr + 16 * bi + lr];
#pragma unroll
            for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = mfma16x16x4(a_op[bj], b_op[bi], acc[bi][bj]);
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t row = 64 * ti + wr + 16 * bi + lr;
                const int32_t c = 64 * tc + wc + 16 * bj + mfma_out_row<T>(lk, v);
                if (row < m && c < kb) W[(int64_t)c * m + row] = acc[bi][bj][v];
            }
}

// Per-launch HIP events of the trailing-update kernel (settings.profile).
static void prof_begin(hipStream_t st, hipEvent_t *e0, hipEvent_t *e1) {
    if (hipEventCreate(e0) != hipSuccess || hipEventCreate(e1) != hipSuccess) { *e0 = *e1 = nullptr; return; }
    (void)hipEventRecord(*e0, st);
}
// slot = (128 x 128 tiles ? 2 : 0) + (FP32 ? 1 : 0)
static void prof_end(qg_handle *h, hipStream_t st, hipEvent_t e0, hipEvent_t e1, double flops, int slot) {
    if (!e0) return;
    (void)hipEventRecord(e1, st);
    h->prof_events.push_back({{e0, e1}, slot});
    h->prof_flops[slot] += flops;
}

void prof_collect(qg_handle *h, int64_t *launches, double *ms, double *flops) {
    for (int q = 0; q < 4; ++q) { launches[q] = 0; ms[q] = 0.0; flops[q] = h->prof_flops[q]; }
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
    for (double &f : h->prof_flops) f = 0.0;
}

template <typename T>
static void launch_update(qg_handle *h, hipStream_t st, T *F, int32_t r, int32_t k0, int32_t kb, int32_t r_lo,
                          int32_t c_hi, const CopyStride &cs, int32_t ncopy) {
    const int32_t TR = (r - r_lo + 63) / 64, TC = (c_hi - r_lo + 63) / 64;
    if (TR <= 0 || TC <= 0 || kb <= 0) return;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->st.profile) prof_begin(st, &e0, &e1);
    // large launches (at least one 128 x 128 lower tile per compute unit) on the big tiles
    const int64_t TR2 = (r - r_lo + 127) / 128, TC2 = (c_hi - r_lo + 127) / 128;
    const int64_t lower2 = TC2 * TR2 - TC2 * (TC2 - 1) / 2;
    const int urgent = st == h->stream ? 1 : 0;
    // FP32 only: the FP64 variant needs more registers than two wavefronts per SIMD allow and was
    // measured slower than the 64 x 64 tiles (one wavefront per SIMD leaves the loads unhidden)
    const bool big = sizeof(T) == 4 && lower2 * ncopy >= 256 && kb > 64;
    if constexpr (sizeof(T) == 4) {
        if (big)
            trail_update_big<<<dim3((unsigned)(8 * TC2 * ((TR2 + 7) / 8)), 1, (unsigned)ncopy), 256, 0, st>>>(
                F, r, k0, kb, r_lo, c_hi, urgent, cs.f);
    }
    if (!big)
        trail_update<T><<<dim3((unsigned)(8 * TC * ((TR + 7) / 8)), 1, (unsigned)ncopy), 256, 0, st>>>(
            F, r, k0, kb, r_lo, c_hi, urgent, cs.f);
    if (h->st.profile) {
        // lower part of rows [r_lo, r) x cols [r_lo, c_hi): sum over columns of (r - col)
        const double M = (double)(r - r_lo), C = (double)(c_hi - r_lo);
        const double entries = C * M - C * (C - 1.0) / 2.0;
        prof_end(h, st, e0, e1, 2.0 * (double)kb * entries * ncopy, (big ? 2 : 0) + (sizeof(T) == 4 ? 1 : 0));
    }
}

// Large front: outer blocks of OB columns, each made of super-panels of SB
// columns, each factored in NB-column panels (diag_block, panel_solve, update
// of the rest of the super-panel) on the main stream; a finished super-panel
// updates the rest of its outer block (rank SB, main stream).  With
// lookahead: the rank-OB update of an outer block is split into the columns
// of the next outer block (main stream, before that block is factored) and
// everything beyond (bulk stream), so the bulk update of outer block O runs
// while outer block O+1 is factored.  The bulk update of O and the
// next-columns update of O+1 touch the same columns, so the latter waits for
// the former.  Every entry receives its updates in column order.  The inverses and W blocks that only the
// solves need are formed on the prep stream.  Both side streams are joined at
// the end.
template <typename T>
static int factor_large(qg_handle *h, int32_t s, T *front, T *dinv, T *sinv, T *wb, const RegParams &rp,
                        const CopyStride &cs, int32_t ncopy) {
    const Plan &pl = h->plan;
    const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
    const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
    T *F = front + pl.fr_off[s];
    const int8_t *kinds = h->d.reg_sign.p + pl.sn_first[s];
    hipStream_t ms = h->stream;
    bool bulk_pending = false;
    // everything before this front on the main stream is visible to the side streams
    QG_HIP(h, hipEventRecord(h->ev_panel, ms));
    QG_HIP(h, hipStreamWaitEvent(h->bulk, h->ev_panel, 0));
    QG_HIP(h, hipStreamWaitEvent(h->prep, h->ev_panel, 0));
    // outer blocks of OB columns on fronts of at most OB rows (no bulk updates at all) and on fronts
    // wider than OB_WIDE_R (where the rank-OB bulk updates pay for the longer panel chain); one
    // super-panel per outer block in between (same box: the lasso's 10000-row root 1-3 % faster with
    // one super-panel per outer block, the 20000-row root 3.5 % faster in FP32 with outer blocks)
    const int32_t ob = (r <= OB || r > OB_WIDE_R) ? OB : SB;
    for (int32_t O0 = 0; O0 < k; O0 += ob) {
        const int32_t O1 = std::min(k, O0 + ob);
        for (int32_t J0 = O0; J0 < O1; J0 += SB) {
            const int32_t J1 = std::min(O1, J0 + SB);
            for (int32_t j0 = J0; j0 < J1; j0 += NB) {
                const int32_t b = std::min(NB, J1 - j0);
                T *ws = dinv + pl.dinv_off[s] + (int64_t)(j0 / NB) * NB * NB;
                diag_block<T><<<dim3(1, 1, ncopy), 256, 0, ms>>>(F, r, j0, b, kinds, rp.eps, rp.dyn, h->d.nreg.p, ws, cs);
                const int32_t mb = r - j0 - b;
                if (mb > 0) panel_solve<T><<<dim3((mb + 63) / 64, 1, ncopy), 256, 0, ms>>>(F, r, j0, b, ws, cs);
                // rest of this super-panel's columns (rank b)
                if (j0 + b < J1) launch_update<T>(h, ms, F, r, j0, b, j0 + b, J1, cs, ncopy);
            }
            QG_HIP(h, hipEventRecord(h->ev_panel, ms));
            {
                // solve-only data of this super-panel
                QG_HIP(h, hipStreamWaitEvent(h->prep, h->ev_panel, 0));
                const int32_t nsub = (J1 - J0 + NB - 1) / NB, ld = nsub * NB;
                T *Xs = sinv + pl.sinv_off[s] + (int64_t)(J0 / SB) * 2 * SB * SB;
                sblock_inverse<T><<<dim3(nsub, 1, ncopy), 256, 0, h->prep>>>(F, r, J0, J1 - J0, dinv + pl.dinv_off[s],
                                                                            ld, Xs, Xs + (int64_t)ld * ld, cs);
                if (J1 < r)
                    wblock<T><<<dim3((unsigned)((r - J1 + 63) / 64), (unsigned)nsub, ncopy), 256, 0, h->prep>>>(
                        F, r, J0, J1 - J0, Xs, ld, wb + pl.w_off[s] + w_block_offset(r, J0), cs);
            }
            // the rest of this outer block's columns (rank J1 - J0), on the panel chain
            if (J1 < O1) launch_update<T>(h, ms, F, r, J0, J1 - J0, J1, O1, cs, ncopy);
        }
        if (O1 < r) {
            const int32_t O2 = std::min(r, O1 + ob);
            QG_HIP(h, hipEventRecord(h->ev_panel, ms));
            // bulk: columns [O2, r), after this outer block's panels
            if (O2 < r) {
                QG_HIP(h, hipStreamWaitEvent(h->bulk, h->ev_panel, 0));
                launch_update<T>(h, h->bulk, F, r, O0, O1 - O0, O2, r, cs, ncopy);
            }
            // next outer block's columns [O1, O2): after the previous bulk update, which also wrote them
            if (bulk_pending) QG_HIP(h, hipStreamWaitEvent(ms, h->ev_bulk, 0));
            launch_update<T>(h, ms, F, r, O0, O1 - O0, O1, O2, cs, ncopy);
            if (O2 < r) {
                QG_HIP(h, hipEventRecord(h->ev_bulk, h->bulk));
                bulk_pending = true;
            } else {
                bulk_pending = false;
            }
        }
    }
    // join
    if (bulk_pending) QG_HIP(h, hipStreamWaitEvent(ms, h->ev_bulk, 0));
    QG_HIP(h, hipEventRecord(h->ev_prep, h->prep));
    QG_HIP(h, hipStreamWaitEvent(ms, h->ev_prep, 0));
    QG_HIP(h, hipEventRecord(h->ev_bulk, h->bulk));
    QG_HIP(h, hipStreamWaitEvent(ms, h->ev_bulk, 0));
    return QG_OK;
}

template <typename T>
static int factor_all(qg_handle *h, T *front, T *dinv, T *sinv, T *wb, const RegParams &rp) {
    const Plan &pl = h->plan;
    Device &d = h->d;
    const int32_t nchain = (int32_t)pl.chain_comp_ptr.size() - 1;
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        if (L == pl.chain_L0 && nchain > 0) {
            // every level below the chains is factored: the components run now, beside the rest
            factor_chain<T><<<(unsigned)nchain, 256, 0, h->stream>>>(
                d.chain_comp_ptr.p, d.chain_grp_ptr.p, d.chain_sn.p, d.ent_front.p, d.ent_dst.p, d.ent_sptr.p,
                d.ent_reg.p, d.ent_src.p, d.kval.p, rp.delta, d.sn_first.p, d.sn_rptr.p, d.fr_off.p, front,
                d.reg_sign.p, rp.eps, rp.dyn, d.nreg.p);
        }
        // the level's other fronts (its chain fronts come last in its ranges)
        const int64_t z0 = pl.zseg_lvl_ptr[L], nz = pl.zseg_lvl_mid[L] - z0;
        if (nz > 0) zero_segments<T><<<(unsigned)nz, 256, 0, h->stream>>>(d.zseg_off.p + z0, d.zseg_len.p + z0, front);
        const int64_t e0 = pl.ent_lvl_ptr[L], ne = pl.ent_lvl_mid[L] - e0;
        if (ne > 0)
            gather_entries<T><<<(unsigned)((ne + 255) / 256), 256, 0, h->stream>>>(
                e0, ne, d.ent_dst.p, d.ent_sptr.p, d.ent_reg.p, d.ent_src.p, d.kval.p, rp.delta, front);
        int32_t s0 = pl.lvl_small_ptr[L];
        const int32_t s1 = pl.lvl_small_ptr[L + 1], nt = pl.lvl_tiny_cnt[L];
        if (nt > 0) {
            // the fronts of at most TINY_R8 rows lead the level's tiny ones
            const int32_t n8 = pl.lvl_tiny8_cnt[L];
            if (n8 > 0)
                factor_tiny<T, TINY_R8><<<(n8 + 15) / 16, 256, 0, h->stream>>>(n8, d.lvl_small_sn.p + s0, d.sn_first.p,
                                                                               d.sn_rptr.p, d.fr_off.p, front,
                                                                               d.reg_sign.p, rp.eps, rp.dyn, d.nreg.p);
            if (nt > n8)
                factor_tiny<T, TINY_R><<<(nt - n8 + 15) / 16, 256, 0, h->stream>>>(
                    nt - n8, d.lvl_small_sn.p + s0 + n8, d.sn_first.p, d.sn_rptr.p, d.fr_off.p, front, d.reg_sign.p,
                    rp.eps, rp.dyn, d.nreg.p);
            s0 += nt;
        }
        if (s1 > s0 && pl.lvl_small_maxr[L] <= CHAIN_R && pl.lvl_small_rsum[L] <= 12 * (int64_t)(s1 - s0)) {
            factor_small_wave<T><<<(s1 - s0 + 3) / 4, 256, 0, h->stream>>>(
                s1 - s0, d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p, d.fr_off.p, front, d.reg_sign.p, rp.eps,
                rp.dyn, d.nreg.p);
        } else if (s1 > s0) {
            const size_t lds = (size_t)pl.lvl_small_maxr[L] * pl.lvl_small_maxr[L] * sizeof(T);
            factor_small<T><<<s1 - s0, 256, lds, h->stream>>>(d.lvl_small_sn.p + s0, d.sn_first.p,
                                                               d.sn_rptr.p, d.fr_off.p, front,
                                                               d.reg_sign.p, rp.eps, rp.dyn, d.nreg.p);
        }
        // large fronts; in a batch, the copies of a front run in one launch sequence
        for (int32_t u = pl.lvl_large_ptr[L]; u < pl.lvl_large_ptr[L + 1]; ++u) {
            const int32_t s = pl.lvl_large_sn[u];
            if (s >= pl.ns1) continue;
            const int rc = factor_large<T>(h, s, front, dinv, sinv, wb, rp, pl.copy_stride[s], pl.ncopy);
            if (rc) return rc;
        }
    }
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

__global__ void zero_int(int32_t *p) { *p = 0; }

int factor_init_attributes(qg_handle *h) {
    const int bytes = SMALL_R * SMALL_R * (int)sizeof(double);
    QG_HIP(h, hipFuncSetAttribute(reinterpret_cast<const void *>(&factor_small<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    QG_HIP(h, hipFuncSetAttribute(reinterpret_cast<const void *>(&factor_small<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, bytes / 2));
    return QG_OK;
}

static int enqueue_factor(qg_handle *h, void *arg) {
    const int precision = *static_cast<const int *>(arg);
    const qg_settings &st = h->st;
    zero_int<<<1, 1, 0, h->stream>>>(h->d.nreg.p);
    if (precision == QG_FP32_IR) {
        RegParams rp{st.static_reg32, st.dyn_eps32, st.dyn_delta32};
        return factor_all<float>(h, h->d.front32.p, h->d.dinv32.p, h->d.sinv32.p, h->d.w32.p, rp);
    }
    RegParams rp{st.static_reg, st.dyn_eps, st.dyn_delta};
    return factor_all<double>(h, h->d.front64.p, h->d.dinv64.p, h->d.sinv64.p, h->d.w64.p, rp);
}

int launch_factor(qg_handle *h, int precision) {
    int prec = precision;
    // A graph only where no front spans more than one outer block (no bulk trailing updates beside the
    // panel chain): with the bulk stream the replayed graph was measured 2-5 % slower than the stream
    // launches (lasso FP32 87.6 -> 91.9 ms over a solve's factorizations); per-launch timing
    // (settings.profile) records events between the launches.
    const bool graph = h->st.graphs && !h->st.profile && h->plan.max_r <= OB;
    const int rc = graph
                       ? graph_replay(h, h->g_factor[precision == QG_FP32_IR ? 1 : 0], enqueue_factor, &prec)
                       : enqueue_factor(h, &prec);
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
