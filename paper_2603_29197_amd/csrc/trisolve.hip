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
// Small fronts: one wavefront per supernode, four per workgroup, per level.  Large
// fronts, per SB-column super-block J with the stored inverse X_J of its
// unit-lower diagonal block and W_J = L(below J, J) X_J: forward, one kernel
// forms y_J = X_J v_J and, in other workgroups, v_below -= W_J v_J; backward,
// one kernel forms u_J = X_J' v_J for all blocks, then per block (last to
// first) one kernel takes x_J = u_J and pushes W_J' x_J onto the earlier u.
#include "kernels.hpp"
#include "solver.hpp"

namespace qg {

// ------------------------------- small -------------------------------------
// Gather for the rows of a large front: RL lanes per (front s, row j) task:
// v = [j < k_s ? x_perm(first_s + j) : 0] + sum over the child columns that map
// onto row j of their update-vector entries (contribution lists of the
// assembly, with the position of each entry in the work vector precomputed).
// Lane l sums contributions l, l + RL, ...; the RL partial sums are combined
// by a fixed butterfly, so the result does not depend on scheduling.  Update
// vectors live in the children's own task slots (rows k_c .. r_c - 1).
__global__ void __launch_bounds__(256) fwd_gather_level(
    int64_t t0, int64_t nt, const int32_t *__restrict__ task_sn, const int32_t *__restrict__ task_col,
    const int32_t *__restrict__ sn_first, const int64_t *__restrict__ ctb_ptr,
    const int64_t *__restrict__ ctb_src, const double *__restrict__ xp, double *__restrict__ vwork,
    int64_t tstride) {
    t0 += blockIdx.z * tstride;                      // copy z of a batched front: its own task slots
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

// Small fronts (r <= SMALL_R = 128): one wavefront per front, four fronts per
// workgroup; lane l holds rows l and l + 64.  The wavefront's rows live in
// LDS and its LDS operations complete in order, so the elimination steps need
// no workgroup barrier.
constexpr int SW = 4;                       // fronts (wavefronts) per workgroup

// Forward: the row's right-hand side is gathered (own entry plus the
// children's update-vector entries that map onto it, in child order), then k
// elimination steps with L columns read from the front, and the update vector
// is left in the front's own slots for the parent.
template <typename T>
__device__ inline void fwd_front(int32_t s, const int32_t *__restrict__ sn_first,
                                 const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off,
                                 const T *__restrict__ front, const int64_t *__restrict__ task0,
                                 const int64_t *__restrict__ ctb_ptr, const int64_t *__restrict__ ctb_src,
                                 double *__restrict__ vwork, double *__restrict__ xp, double *v) {
    const int lane = threadIdx.x & 63;
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    double *vs = vwork + task0[s];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t row = lane + 64 * h;
        if (row < r) {
            const int64_t tk = task0[s] + row;
            double a = row < k ? xp[f + row] : 0.0;
            for (int64_t u = ctb_ptr[tk]; u < ctb_ptr[tk + 1]; ++u) a += vwork[ctb_src[u]];
            v[row] = a;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const T *F = front + fr_off[s];
    for (int32_t jj = 0; jj < k; ++jj) {
        const double yj = v[jj];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t row = lane + 64 * h;
            const bool act = row > jj && row < r;
            const T l = F[(int64_t)jj * r + (act ? row : jj)];
            if (act) v[row] -= (double)l * yj;
        }
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t row = lane + 64 * h;
        if (row < k) xp[f + row] = v[row];
        else if (row < r) vs[row] = v[row];
    }
    __builtin_amdgcn_wave_barrier();
}

// Backward: v = D^-1 x_own - L21' g (g = solution at the update rows; the
// products with L21' are summed per column over the wavefront with a
// butterfly), then the unit-upper solve with L11'.
template <typename T>
__device__ inline void bwd_front(int32_t s, const int32_t *__restrict__ sn_first,
                                 const int64_t *__restrict__ sn_rptr, const int32_t *__restrict__ sn_rows,
                                 const int64_t *__restrict__ fr_off, const T *__restrict__ front,
                                 double *__restrict__ xp, double *v) {
    const int lane = threadIdx.x & 63;
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    const T *F = front + fr_off[s];
    double g[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t row = lane + 64 * h;
        g[h] = (row >= k && row < r) ? xp[sn_rows[sn_rptr[s] + row]] : 0.0;
    }
    for (int32_t c = 0; c < k; ++c) {
        double p = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t row = lane + 64 * h;
            const bool upd = row >= k && row < r;
            const T lv = F[(int64_t)c * r + (upd ? row : c)];
            p += upd ? (double)lv * g[h] : 0.0;
        }
        for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off);
        if (lane == 0) v[c] = xp[f + c] / (double)F[(int64_t)c * r + c] - p;
    }
    __builtin_amdgcn_wave_barrier();
    for (int32_t i = k - 1; i >= 0; --i) {
        const double xi = v[i];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t row = lane + 64 * h;
            const bool act = row < i;
            const T l = F[(int64_t)(act ? row : i) * r + i];
            if (act) v[row] -= (double)l * xi;
        }
        __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int32_t row = lane + 64 * h;
        if (row < k) xp[f + row] = v[row];
    }
    __builtin_amdgcn_wave_barrier();
}

// Chains (see factor_chain): one workgroup per component, its levels in
// order (forward: lowest first; backward: highest first), the fronts of a
// level one per wavefront, a workgroup barrier between levels.  A chain front
// has at most CHAIN_R = 32 rows, so lane l holds row l in registers: every L
// entry the lane needs is loaded at once when the front starts (one memory
// round trip instead of one per elimination step), and the pivot values are
// broadcast with readlane instead of through LDS, so the elimination steps
// need no barrier.  Same operations in the same order as fwd_front and
// bwd_front, hence the same bits.
template <typename T>
__device__ inline void fwd_front_chain(int32_t s, const int32_t *__restrict__ sn_first,
                                       const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off,
                                       const T *__restrict__ front, const int64_t *__restrict__ task0,
                                       const int64_t *__restrict__ ctb_ptr, const int64_t *__restrict__ ctb_src,
                                       double *__restrict__ vwork, double *__restrict__ xp) {
    const int row = threadIdx.x & 63;
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    const int64_t t0 = task0[s];
    const T *F = front + fr_off[s];
    const bool live = row < r;
    // L(row, jj) from clamped (always valid) positions, all loads in flight at once: the empty asm
    // statements need every value in a register, so no load is deferred to its elimination step.
    // Entries of masked lanes or steps are loaded but never used.
    const int32_t rowc = min(row, r - 1);
    T lc[CHAIN_R];
#pragma unroll
    for (int jj = 0; jj < CHAIN_R; ++jj) lc[jj] = F[(int64_t)min(jj, k - 1) * r + rowc];
#pragma unroll
    for (int jj = 0; jj < CHAIN_R; ++jj) __asm__ volatile("" : "+v"(lc[jj]));
    double a = 0.0;
    if (live) {
        const int64_t tk = t0 + row;
        a = row < k ? xp[f + row] : 0.0;
        for (int64_t u = ctb_ptr[tk]; u < ctb_ptr[tk + 1]; ++u) a += vwork[ctb_src[u]];
    }
#pragma unroll
    for (int jj = 0; jj < CHAIN_R; ++jj) {
        if (jj < k) {                                 // uniform
            const double yj = lane_bcast(a, jj);
            if (row > jj && live) a -= (double)lc[jj] * yj;
        }
    }
    if (row < k) xp[f + row] = a;
    else if (live) vwork[t0 + row] = a;
}

template <typename T>
__device__ inline void bwd_front_chain(int32_t s, const int32_t *__restrict__ sn_first,
                                       const int64_t *__restrict__ sn_rptr, const int32_t *__restrict__ sn_rows,
                                       const int64_t *__restrict__ fr_off, const T *__restrict__ front,
                                       double *__restrict__ xp) {
    const int row = threadIdx.x & 63;
    const int32_t f = sn_first[s];
    const int32_t r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const int32_t k = sn_first[s + 1] - f;
    const T *F = front + fr_off[s];
    const bool upd = row >= k && row < r;
    // L(row, c) and L(c, row) from clamped (always valid) positions, all loads in flight at once (see
    // fwd_front_chain); entries of masked lanes or columns are loaded but never used
    const int32_t rowc = min(row, r - 1);
    T lc[CHAIN_R], lr[CHAIN_R];
#pragma unroll
    for (int c = 0; c < CHAIN_R; ++c) {
        const int32_t cc = min(c, k - 1);
        lc[c] = F[(int64_t)cc * r + rowc];
        lr[c] = F[(int64_t)rowc * r + cc];
    }
#pragma unroll
    for (int c = 0; c < CHAIN_R; ++c) __asm__ volatile("" : "+v"(lc[c]), "+v"(lr[c]));
    const double g = upd ? xp[sn_rows[sn_rptr[s] + row]] : 0.0;
    const double xo = row < k ? xp[f + row] : 0.0;
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < CHAIN_R; ++c) {
        if (c < k) {                                  // uniform
            double p = 0.0;
            p += upd ? (double)lc[c] * g : 0.0;
            p += 0.0;                                 // the rows l + 64 of bwd_front (none here)
            for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off);
            if (row == c) v = xo / (double)lc[c] - p;
        }
    }
#pragma unroll
    for (int i = CHAIN_R - 1; i >= 0; --i) {
        if (i < k) {                                  // uniform
            const double xi = lane_bcast(v, i);
            if (row < i) v -= (double)lr[i] * xi;
        }
    }
    if (row < k) xp[f + row] = v;
}

// Tiny fronts (r <= TINY_R): 16 lanes per front, lane i holding row i, sixteen
// fronts per workgroup; pivot values come from the front's own lanes by
// shuffle.  Same operations in the same order as fwd_front and bwd_front (the
// backward's column sums are the same butterfly restricted to the 16 lanes
// that hold rows), hence the same values.
// Largest of a value over the four 16-lane groups of a wavefront (every lane holds its group's
// value), returned in every lane.
__device__ inline int wave_max4(int v) {
    v = max(v, __shfl_xor(v, 16));
    return max(v, __shfl_xor(v, 32));
}

template <typename T>
__global__ void __launch_bounds__(256) fwd_tiny(
    int32_t nfront, const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, const T *__restrict__ front,
    const int64_t *__restrict__ task0, const int64_t *__restrict__ ctb_ptr, const int64_t *__restrict__ ctb_src,
    double *__restrict__ vwork, double *__restrict__ xp) {
    const int gl = threadIdx.x & 15, gb = (threadIdx.x & 63) & ~15;
    const int32_t q = (blockIdx.x * 256 + threadIdx.x) >> 4;
    const bool has = q < nfront;
    const int32_t s = has ? sn_list[q] : 0;
    const int32_t f = has ? sn_first[s] : 0;
    const int32_t r = has ? (int32_t)(sn_rptr[s + 1] - sn_rptr[s]) : 0;
    const int32_t k = has ? sn_first[s + 1] - f : 0;
    const bool live = gl < r;
    const int64_t t0 = has ? task0[s] : 0;
    const T *F = front + (has ? fr_off[s] : 0);
    // the row's L entries, all loads in flight before the elimination
    double lc[TINY_R];
#pragma unroll
    for (int jj = 0; jj < TINY_R; ++jj) lc[jj] = (jj < k && gl > jj && live) ? (double)F[(int64_t)jj * r + gl] : 0.0;
    double a = 0.0;
    if (live) {
        const int64_t tk = t0 + gl;
        a = gl < k ? xp[f + gl] : 0.0;
        for (int64_t u = ctb_ptr[tk]; u < ctb_ptr[tk + 1]; ++u) a += vwork[ctb_src[u]];
    }
    // steps beyond the wavefront's largest pivot count change nothing: stop there (a bound that is
    // the same in every lane, as the shuffles need)
    const int kw = wave_max4(k);
#pragma unroll
    for (int jj = 0; jj < TINY_R; ++jj) {
        if (jj >= kw) break;
        const double yj = __shfl(a, gb + jj);
        if (jj < k && gl > jj && live) a -= lc[jj] * yj;
    }
    if (gl < k) xp[f + gl] = a;
    else if (live) vwork[t0 + gl] = a;
}

template <typename T>
__global__ void __launch_bounds__(256) bwd_tiny(
    int32_t nfront, const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int32_t *__restrict__ sn_rows,
    const int64_t *__restrict__ fr_off, const T *__restrict__ front, double *__restrict__ xp) {
    const int gl = threadIdx.x & 15, gb = (threadIdx.x & 63) & ~15;
    const int32_t q = (blockIdx.x * 256 + threadIdx.x) >> 4;
    const bool has = q < nfront;
    const int32_t s = has ? sn_list[q] : 0;
    const int32_t f = has ? sn_first[s] : 0;
    const int32_t r = has ? (int32_t)(sn_rptr[s + 1] - sn_rptr[s]) : 0;
    const int32_t k = has ? sn_first[s + 1] - f : 0;
    const T *F = front + (has ? fr_off[s] : 0);
    const bool upd = gl >= k && gl < r;
    const double g = upd ? xp[sn_rows[sn_rptr[s] + gl]] : 0.0;
    const double xo = gl < k ? xp[f + gl] : 0.0;
    // the row's L entries L(gl, c) (update rows) and L(gl, i) (pivot rows, i > gl), and the pivot
    // D(gl): all loads in flight before the sums
    double lc[TINY_R];
#pragma unroll
    for (int c = 0; c < TINY_R; ++c)
        lc[c] = ((c < k && upd) || (c < k && gl < c)) ? (double)F[upd ? (int64_t)c * r + gl : (int64_t)gl * r + c] : 0.0;
    const double dg = gl < k ? (double)F[(int64_t)gl * r + gl] : 1.0;
    double v = 0.0;
    // columns and steps beyond the wavefront's largest pivot count change nothing: skipped (a bound
    // that is the same in every lane, as the shuffles need)
    const int kw = wave_max4(k);
#pragma unroll
    for (int c = 0; c < TINY_R; ++c) {
        if (c >= kw) break;
        double p = 0.0;
        if (c < k && upd) p += lc[c] * g;
        p += 0.0;                                     // the rows l + 64 of bwd_front (none here)
        for (int off = 8; off > 0; off >>= 1) p += __shfl_xor(p, off);
        if (c < k && gl == c) v = xo / dg - p;
    }
#pragma unroll
    for (int i = TINY_R - 1; i >= 0; --i) {
        if (i >= kw) continue;
        const double xi = __shfl(v, gb + i);
        if (i < k && gl < i) v -= lc[i] * xi;
    }
    if (gl < k) xp[f + gl] = v;
}

// The level kernels of small fronts.  (The register path of the chains, all L
// entries of a front loaded at once, was measured slower here: on a level of
// 2e5 fronts of about four rows its 32 loads per lane cost 1.1 ms against
// 0.11 ms for the backward sweep.)
template <typename T>
__global__ void __launch_bounds__(64 * SW) fwd_small(
    int32_t nfront, const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, const T *__restrict__ front,
    const int64_t *__restrict__ task0, const int64_t *__restrict__ ctb_ptr, const int64_t *__restrict__ ctb_src,
    double *__restrict__ vwork, double *__restrict__ xp) {
    __shared__ double vsh[SW][SMALL_R];
    const int w = threadIdx.x >> 6;
    const int32_t q = blockIdx.x * SW + w;
    if (q >= nfront) return;                   // whole wavefront
    fwd_front<T>(sn_list[q], sn_first, sn_rptr, fr_off, front, task0, ctb_ptr, ctb_src, vwork, xp, vsh[w]);
}

template <typename T>
__global__ void __launch_bounds__(64 * SW) bwd_small(
    int32_t nfront, const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int32_t *__restrict__ sn_rows,
    const int64_t *__restrict__ fr_off, const T *__restrict__ front, double *__restrict__ xp) {
    __shared__ double vsh[SW][SMALL_R];
    const int w = threadIdx.x >> 6;
    const int32_t q = blockIdx.x * SW + w;
    if (q >= nfront) return;                   // whole wavefront
    bwd_front<T>(sn_list[q], sn_first, sn_rptr, sn_rows, fr_off, front, xp, vsh[w]);
}

// Forward sweep, small fronts on levels with few of them (fewer than REG_LEVEL_MAX, all of at most
// CHAIN_R rows): the register path of the chains, one wavefront per front, every L entry of a lane's
// row loaded at once instead of one dependent load per elimination step; the same bits as fwd_front.
// (On levels of many small fronts its 32 loads per lane cost more than the steps they save; in the
// backward sweep, whose register path also loads each lane's L row with strided loads, it was
// measured slower on every level: many-SOC 10.9 -> 14.5 us per level on average.)
template <typename T>
__global__ void __launch_bounds__(64 * SW) fwd_small_reg(
    int32_t nfront, const int32_t *__restrict__ sn_list, const int32_t *__restrict__ sn_first,
    const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off, const T *__restrict__ front,
    const int64_t *__restrict__ task0, const int64_t *__restrict__ ctb_ptr, const int64_t *__restrict__ ctb_src,
    double *__restrict__ vwork, double *__restrict__ xp) {
    const int32_t q = blockIdx.x * SW + (threadIdx.x >> 6);
    if (q >= nfront) return;                   // whole wavefront
    fwd_front_chain<T>(sn_list[q], sn_first, sn_rptr, fr_off, front, task0, ctb_ptr, ctb_src, vwork, xp);
}

// Static data of one chain front for the forward solve, per lane (row): everything that does not
// depend on the solve's progress (the L entries, the front's own right-hand side entry, the range of
// the row's contributions in the work vector and the positions of its first two).
template <typename T>
struct FwdStatic {
    int32_t f, r, k;
    int64_t t0;
    T lc[CHAIN_R];
    double xr;
    int64_t u0, u1, q0, q1;
};

// Issue the loads of front s's static data (s < 0: none).  The positions q0 and q1 need u0 and u1,
// so they are completed by fwd_static_sources once those have arrived.
template <typename T>
__device__ inline void fwd_static_load(FwdStatic<T> &st, int32_t s, const int32_t *__restrict__ sn_first,
                                       const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off,
                                       const T *__restrict__ front, const int64_t *__restrict__ task0,
                                       const int64_t *__restrict__ ctb_ptr, const double *__restrict__ xp) {
    if (s < 0) return;
    const int row = threadIdx.x & 63;
    st.f = sn_first[s];
    st.k = sn_first[s + 1] - st.f;
    st.r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    st.t0 = task0[s];
    const T *F = front + fr_off[s];
    const int32_t rowc = min(row, st.r - 1);
#pragma unroll
    for (int jj = 0; jj < CHAIN_R; ++jj) st.lc[jj] = F[(int64_t)min(jj, st.k - 1) * st.r + rowc];
    st.xr = xp[st.f + min(row, st.k - 1)];
    st.u0 = ctb_ptr[st.t0 + rowc];
    st.u1 = ctb_ptr[st.t0 + rowc + 1];
}
template <typename T>
__device__ inline void fwd_static_sources(FwdStatic<T> &st, int32_t s, const int64_t *__restrict__ ctb_src) {
    if (s < 0) return;
    st.q0 = st.u0 < st.u1 ? ctb_src[st.u0] : 0;
    st.q1 = st.u0 + 1 < st.u1 ? ctb_src[st.u0 + 1] : 0;
}

// Chains, forward, one level ahead: while a wavefront solves its front of level g, the static data
// of its front of level g + 1 is in flight, so after the level's barrier only the children's
// update-vector entries remain to be read.  Further fronts of a level (more than SW of them) go
// through fwd_front_chain.  Same operations in the same order as fwd_front.
template <typename T>
__global__ void __launch_bounds__(64 * SW) fwd_chain(
    const int32_t *__restrict__ comp_ptr, const int32_t *__restrict__ grp_ptr, const int32_t *__restrict__ chain_sn,
    const int32_t *__restrict__ sn_first, const int64_t *__restrict__ sn_rptr, const int64_t *__restrict__ fr_off,
    const T *__restrict__ front, const int64_t *__restrict__ task0, const int64_t *__restrict__ ctb_ptr,
    const int64_t *__restrict__ ctb_src, double *__restrict__ vwork, double *__restrict__ xp) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: the front indices below too
    const int row = threadIdx.x & 63;
    const int32_t c = blockIdx.x;
    const int32_t g0 = comp_ptr[c], g1 = comp_ptr[c + 1];
    auto first = [&](int32_t g) {                     // this wavefront's first front of level g, or -1
        if (g >= g1) return -1;
        const int32_t t = grp_ptr[g] + w;
        return t < grp_ptr[g + 1] ? chain_sn[t] : -1;
    };
    FwdStatic<T> cur, nxt;
    int32_t s_cur = first(g0);
    fwd_static_load<T>(cur, s_cur, sn_first, sn_rptr, fr_off, front, task0, ctb_ptr, xp);
    fwd_static_sources<T>(cur, s_cur, ctb_src);
    for (int32_t g = g0; g < g1; ++g) {
        double v0 = 0.0, v1 = 0.0;
        if (s_cur >= 0) {                             // the children's entries (written before the last barrier)
            if (cur.u0 < cur.u1) v0 = vwork[cur.q0];
            if (cur.u0 + 1 < cur.u1) v1 = vwork[cur.q1];
        }
        const int32_t s_nxt = first(g + 1);
        fwd_static_load<T>(nxt, s_nxt, sn_first, sn_rptr, fr_off, front, task0, ctb_ptr, xp);
        if (s_cur >= 0) {
            const bool live = row < cur.r;
            double a = row < cur.k ? cur.xr : 0.0;
            if (cur.u0 < cur.u1) a += v0;
            if (cur.u0 + 1 < cur.u1) a += v1;
            for (int64_t u = cur.u0 + 2; u < cur.u1; ++u) a += vwork[ctb_src[u]];
            if (!live) a = 0.0;
#pragma unroll
            for (int jj = 0; jj < CHAIN_R; ++jj) {
                if (jj < cur.k) {                         // uniform
                    const double yj = lane_bcast(a, jj);
                    if (row > jj && live) a -= (double)cur.lc[jj] * yj;
                }
            }
            if (row < cur.k) xp[cur.f + row] = a;
            else if (live) vwork[cur.t0 + row] = a;
        }
        fwd_static_sources<T>(nxt, s_nxt, ctb_src);
        for (int32_t t = grp_ptr[g] + w + SW; t < grp_ptr[g + 1]; t += SW)
            fwd_front_chain<T>(chain_sn[t], sn_first, sn_rptr, fr_off, front, task0, ctb_ptr, ctb_src, vwork, xp);
        __syncthreads();
        s_cur = s_nxt;
        cur = nxt;
    }
}

// Static data of one chain front for the backward solve, per lane (row): the L entries of its row and
// column, the work-vector position of its update row, and its own entry of the forward result.
template <typename T>
struct BwdStatic {
    int32_t f, r, k;
    T lc[CHAIN_R], lr[CHAIN_R];
    int32_t gi;
    double xo;
};

template <typename T>
__device__ inline void bwd_static_load(BwdStatic<T> &st, int32_t s, const int32_t *__restrict__ sn_first,
                                       const int64_t *__restrict__ sn_rptr, const int32_t *__restrict__ sn_rows,
                                       const int64_t *__restrict__ fr_off, const T *__restrict__ front,
                                       const double *__restrict__ xp) {
    if (s < 0) return;
    const int row = threadIdx.x & 63;
    st.f = sn_first[s];
    st.k = sn_first[s + 1] - st.f;
    st.r = (int32_t)(sn_rptr[s + 1] - sn_rptr[s]);
    const T *F = front + fr_off[s];
    const int32_t rowc = min(row, st.r - 1);
#pragma unroll
    for (int c = 0; c < CHAIN_R; ++c) {
        const int32_t cc = min(c, st.k - 1);
        st.lc[c] = F[(int64_t)cc * st.r + rowc];
        st.lr[c] = F[(int64_t)rowc * st.r + cc];
    }
    st.gi = sn_rows[sn_rptr[s] + rowc];
    st.xo = xp[st.f + min(row, st.k - 1)];
}

// Chains, backward, one level ahead (see fwd_chain): after the level's barrier only the solution
// entries of the front's update rows (solved by its ancestors) remain to be read.  Same operations in
// the same order as bwd_front.
template <typename T>
__global__ void __launch_bounds__(64 * SW) bwd_chain(
    const int32_t *__restrict__ comp_ptr, const int32_t *__restrict__ grp_ptr, const int32_t *__restrict__ chain_sn,
    const int32_t *__restrict__ sn_first, const int64_t *__restrict__ sn_rptr, const int32_t *__restrict__ sn_rows,
    const int64_t *__restrict__ fr_off, const T *__restrict__ front, double *__restrict__ xp) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: the front indices below too
    const int row = threadIdx.x & 63;
    const int32_t c = blockIdx.x;
    const int32_t g0 = comp_ptr[c], g1 = comp_ptr[c + 1];
    auto first = [&](int32_t g) {                     // this wavefront's first front of level g, or -1
        if (g < g0) return -1;
        const int32_t t = grp_ptr[g] + w;
        return t < grp_ptr[g + 1] ? chain_sn[t] : -1;
    };
    BwdStatic<T> cur, nxt;
    int32_t s_cur = first(g1 - 1);
    bwd_static_load<T>(cur, s_cur, sn_first, sn_rptr, sn_rows, fr_off, front, xp);
    for (int32_t g = g1 - 1; g >= g0; --g) {
        double gv = 0.0;
        const bool upd = s_cur >= 0 && row >= cur.k && row < cur.r;
        if (upd) gv = xp[cur.gi];                     // solved by the ancestors, before the last barrier
        const int32_t s_nxt = first(g - 1);
        bwd_static_load<T>(nxt, s_nxt, sn_first, sn_rptr, sn_rows, fr_off, front, xp);
        if (s_cur >= 0) {
            double v = 0.0;
#pragma unroll
            for (int cc = 0; cc < CHAIN_R; ++cc) {
                if (cc < cur.k) {                         // uniform
                    double p = 0.0;
                    p += upd ? (double)cur.lc[cc] * gv : 0.0;
                    p += 0.0;                             // the rows l + 64 of bwd_front (none here)
                    for (int off = 32; off > 0; off >>= 1) p += __shfl_xor(p, off);
                    if (row == cc) v = cur.xo / (double)cur.lc[cc] - p;
                }
            }
#pragma unroll
            for (int i = CHAIN_R - 1; i >= 0; --i) {
                if (i < cur.k) {                          // uniform
                    const double xi = lane_bcast(v, i);
                    if (row < i) v -= (double)cur.lr[i] * xi;
                }
            }
            if (row < cur.k) xp[cur.f + row] = v;
        }
        for (int32_t t = grp_ptr[g] + w + SW; t < grp_ptr[g + 1]; t += SW)
            bwd_front_chain<T>(chain_sn[t], sn_first, sn_rptr, sn_rows, fr_off, front, xp);
        __syncthreads();
        s_cur = s_nxt;
        cur = nxt;
    }
}

// ------------------------------- large -------------------------------------
// Sum over q of the column-major operand M(t, q) u(q) for one entry t per
// lane: wavefront w takes the columns q in [q_lo(w), q_hi(w)) (lanes along
// rows: coalesced), and the four partial sums are added in a fixed order.
// Returns the sum in wavefront 0 (other wavefronts return 0).
template <typename T>
__device__ inline double quarter_gemv(const T *__restrict__ Mt, int64_t ldm, const double *__restrict__ u,
                                      int32_t q_lo, int32_t q_hi, bool live, double (&red)[4][64]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double acc = 0.0;
    if (live) {
#pragma unroll 16
        for (int32_t q = q_lo; q < q_hi; ++q) acc += (double)Mt[(int64_t)q * ldm] * u[q];
    }
    red[w][lane] = acc;
    __syncthreads();
    return w == 0 ? ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane] : 0.0;
}

// Forward step of super-block [J0, J0+kb) of a large front (work vector vs,
// rows 0..r-1 of the front): workgroups 0..G-1 (G = kb / 64 rounded up) form
// y = X_J v_J and write it to the solution; the others update the rows below,
// v[J1 + i] -= sum_q W_J(i, q) v_J(q) (W_J = L(below, J) X_J, so this equals
// L(below, J) y without waiting for y).  One launch per super-block.
template <typename T>
__global__ void __launch_bounds__(256) fwd_block(const T *__restrict__ X, int32_t ld, int32_t kb,
                                                 const T *__restrict__ W, int32_t m, int32_t J0,
                                                 double *__restrict__ vs, double *__restrict__ xp_own,
                                                 CopyStride cs) {
    X += blockIdx.z * cs.sinv;
    W += blockIdx.z * cs.w;
    vs += blockIdx.z * cs.task;
    xp_own += blockIdx.z * cs.col;
    __shared__ double vj[SB];
    __shared__ double red[4][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid < kb) vj[tid] = vs[J0 + tid];
    __syncthreads();
    const int32_t G = (kb + 63) / 64;
    const int32_t g = blockIdx.x;
    if (g < G) {
        // X lower: entry t = 64 g + lane needs columns q <= t
        const int32_t t = 64 * g + lane;
        const double y = quarter_gemv(X + t, ld, vj, 64 * w, min(kb, 64 * w + 64), w <= g && t < kb, red);
        if (w == 0 && t < kb) xp_own[J0 + t] = y;
    } else {
        const int32_t i = 64 * (g - G) + lane;
        const double s = quarter_gemv(W + i, (int64_t)m, vj, 64 * w, min(kb, 64 * w + 64), i < m, red);
        if (w == 0 && i < m) vs[J0 + kb + i] -= s;
    }
}

// Backward, all super-blocks of a large front at once: u_J = X_J' v_J
// (grid (4, super-blocks); X_J' stored column-major, upper triangular).
template <typename T>
__global__ void __launch_bounds__(256) bwd_apply_all(const T *__restrict__ sinv_s, int32_t k,
                                                     const double *__restrict__ v, double *__restrict__ u,
                                                     CopyStride cs, int32_t max_r) {
    sinv_s += blockIdx.z * cs.sinv;
    v += (int64_t)blockIdx.z * max_r;
    u += (int64_t)blockIdx.z * max_r;
    __shared__ double vj[SB];
    __shared__ double red[4][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int32_t g = blockIdx.x, J0 = blockIdx.y * SB;
    const int32_t kb = min(SB, k - J0), ld = (kb + NB - 1) / NB * NB;
    if (64 * g >= kb) return;                       // whole workgroup: nothing in this quarter
    const T *XT = sinv_s + (int64_t)(J0 / SB) * 2 * SB * SB + (int64_t)ld * ld;
    if (tid < kb) vj[tid] = v[J0 + tid];
    __syncthreads();
    const int32_t t = 64 * g + lane;
    const double y = quarter_gemv(XT + t, ld, vj, 64 * w, min(kb, 64 * w + 64), w >= g && t < kb, red);
    if (w == 0 && t < kb) u[J0 + t] = y;
}

// v[0:k] = D^-1 x_own - L21' g with g = x at the rows below (one column per
// wavefront, reduction over rows).
template <typename T>
__global__ void __launch_bounds__(256) bwd_init(int32_t s, const int32_t *__restrict__ sn_first,
                                                const int64_t *__restrict__ sn_rptr,
                                                const int32_t *__restrict__ sn_rows,
                                                const T *__restrict__ F, const double *__restrict__ xp,
                                                double *__restrict__ vbuf, CopyStride cs, int32_t max_r) {
    s += blockIdx.z * cs.front;
    F += blockIdx.z * cs.f;
    vbuf += (int64_t)blockIdx.z * max_r;
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

// Backward step of super-block [K0, K0+kb): x_K = u_K is final (every later
// block has pushed onto it); workgroup 0 writes it to the solution, and every
// workgroup pushes it onto 64 earlier entries: u[c] -= sum_t W_J(K0 - J1 + t,
// c - J0) x_K(t) for the block J = [J0, J1) that holds c.  Wavefront w takes
// 16 columns; lanes run along the contiguous rows of each W column
// (coalesced), and the 64 loads of W and the 4 of x_K of a lane are issued
// together.  The 16 x 64 partial sums of a wavefront are transposed through
// LDS: lane l adds 16 of column l / 4's partials, then two butterfly steps
// combine the four lanes of each column.  No workgroup barrier.
template <typename T>
__global__ void __launch_bounds__(256) bwd_push(const T *__restrict__ W_s, int32_t r, int32_t K0, int32_t kb,
                                                double *__restrict__ u, double *__restrict__ xp_own,
                                                CopyStride cs, int32_t max_r) {
    W_s += blockIdx.z * cs.w;
    u += (int64_t)blockIdx.z * max_r;
    xp_own += blockIdx.z * cs.col;
    __shared__ double red[4][16][65];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const bool pushes = blockIdx.x * NB < K0;        // uniform over the workgroup
    const int32_t c0 = blockIdx.x * NB + w * 16;
    // raw loads from always-valid addresses (zeroing at the use, so that all are in flight at once)
    T wv[16][SB / 64];
    if (pushes) {
        const int32_t J0 = (blockIdx.x * NB) / SB * SB, J1 = J0 + SB;   // a full block: J1 <= K0
        const int64_t m = r - J1;
        const T *Wj = W_s + w_block_offset(r, J0) + (K0 - J1);
#pragma unroll
        for (int cc = 0; cc < 16; ++cc)
#pragma unroll
            for (int q = 0; q < SB / 64; ++q) {
                const int32_t t = lane + 64 * q;
                wv[cc][q] = Wj[c0 + cc < K0 && t < kb ? (int64_t)(c0 + cc - J0) * m + t : 0];
            }
    }
    double xk[SB / 64];
#pragma unroll
    for (int q = 0; q < SB / 64; ++q) xk[q] = u[K0 + (lane + 64 * q < kb ? lane + 64 * q : 0)];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < SB / 64; ++q) xk[q] = lane + 64 * q < kb ? xk[q] : 0.0;
    if (blockIdx.x == 0 && w == 0) {
#pragma unroll
        for (int q = 0; q < SB / 64; ++q)
            if (lane + 64 * q < kb) xp_own[K0 + lane + 64 * q] = xk[q];
    }
    if (!pushes) return;
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < SB / 64; ++q)
            s += (double)(c0 + cc < K0 && lane + 64 * q < kb ? wv[cc][q] : T(0)) * xk[q];
        red[w][cc][lane] = s;
    }
    __builtin_amdgcn_wave_barrier();                 // LDS operations of one wavefront complete in order
    const int cc = lane >> 2, qq = lane & 3;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < 16; ++e) s += red[w][cc][16 * qq + e];
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    if (qq == 0 && c0 + cc < K0) u[c0 + cc] -= s;
}

// ------------------------------- driver ------------------------------------
template <typename T>
static int solve_perm(qg_handle *h, const T *front, const T *sinv, const T *wbuf) {
    const Plan &pl = h->plan;
    Device &d = h->d;
    double *xp = d.xp.p;
    const int32_t nchain = (int32_t)pl.chain_comp_ptr.size() - 1;
    for (int32_t L = 0; L < pl.nlevels; ++L) {
        if (L == pl.chain_L0 && nchain > 0)
            fwd_chain<T><<<(unsigned)nchain, 64 * SW, 0, h->stream>>>(
                d.chain_comp_ptr.p, d.chain_grp_ptr.p, d.chain_sn.p, d.sn_first.p, d.sn_rptr.p, d.fr_off.p, front,
                d.task0.p, d.ctb_ptr.p, d.ctb_src.p, d.vwork.p, xp);
        int32_t s0 = pl.lvl_small_ptr[L];
        const int32_t s1 = pl.lvl_small_ptr[L + 1], nt = pl.lvl_tiny_cnt[L];
        if (nt > 0) {
            fwd_tiny<T><<<(nt + 15) / 16, 256, 0, h->stream>>>(nt, d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
                                                                d.fr_off.p, front, d.task0.p, d.ctb_ptr.p,
                                                                d.ctb_src.p, d.vwork.p, xp);
            s0 += nt;
        }
        const bool reg = s1 - s0 < REG_LEVEL_MAX && pl.lvl_small_maxr[L] <= CHAIN_R;
        if (s1 > s0 && reg)
            fwd_small_reg<T><<<(s1 - s0 + SW - 1) / SW, 64 * SW, 0, h->stream>>>(
                s1 - s0, d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p, d.fr_off.p, front, d.task0.p, d.ctb_ptr.p,
                d.ctb_src.p, d.vwork.p, xp);
        else if (s1 > s0)
            fwd_small<T><<<(s1 - s0 + SW - 1) / SW, 64 * SW, 0, h->stream>>>(s1 - s0, d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
                                                               d.fr_off.p, front, d.task0.p, d.ctb_ptr.p,
                                                               d.ctb_src.p, d.vwork.p, xp);
        for (int32_t u = pl.lvl_large_ptr[L]; u < pl.lvl_large_ptr[L + 1]; ++u) {
            const int32_t s = pl.lvl_large_sn[u];
            if (s >= pl.ns1) continue;                 // copies of a batch run with copy 0 (blockIdx.z)
            const CopyStride &cs = pl.copy_stride[s];
            const unsigned nc = (unsigned)pl.ncopy;
            const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
            const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
            double *vs = d.vwork.p + pl.task0[s];
            // gather of this front's rows (its tasks are contiguous)
            fwd_gather_level<<<dim3((unsigned)((r + 256 / RL - 1) / (256 / RL)), 1, nc), 256, 0, h->stream>>>(
                pl.task0[s], r, d.task_sn.p, d.task_col.p, d.sn_first.p, d.ctb_ptr.p, d.ctb_src.p, xp, d.vwork.p,
                cs.task);
            for (int32_t J0 = 0; J0 < k; J0 += SB) {
                const int32_t kb = std::min(SB, k - J0);
                const int32_t ld = (kb + NB - 1) / NB * NB;
                const int32_t m = r - J0 - kb;
                const T *Xsb = sinv + pl.sinv_off[s] + (int64_t)(J0 / SB) * 2 * SB * SB;
                const T *Wj = wbuf + pl.w_off[s] + w_block_offset(r, J0);
                const unsigned grid = (unsigned)((kb + 63) / 64 + (m + 63) / 64);
                fwd_block<T><<<dim3(grid, 1, nc), 256, 0, h->stream>>>(Xsb, ld, kb, Wj, m, J0, vs,
                                                                      xp + pl.sn_first[s], cs);
            }
        }
    }
    for (int32_t L = pl.nlevels - 1; L >= 0; --L) {
        for (int32_t u = pl.lvl_large_ptr[L + 1] - 1; u >= pl.lvl_large_ptr[L]; --u) {
            const int32_t s = pl.lvl_large_sn[u];
            if (s >= pl.ns1) continue;
            const CopyStride &cs = pl.copy_stride[s];
            const unsigned nc = (unsigned)pl.ncopy;
            const int32_t r = (int32_t)(pl.sn_rptr[s + 1] - pl.sn_rptr[s]);
            const int32_t k = pl.sn_first[s + 1] - pl.sn_first[s];
            const T *F = front + pl.fr_off[s];
            bwd_init<T><<<dim3((k + 3) / 4, 1, nc), 256, 0, h->stream>>>(s, d.sn_first.p, d.sn_rptr.p, d.sn_rows.p,
                                                                         F, xp, d.vbuf.p, cs, pl.max_r);
            const int32_t nsb = (k + SB - 1) / SB;
            bwd_apply_all<T><<<dim3(SB / 64, (unsigned)nsb, nc), 256, 0, h->stream>>>(sinv + pl.sinv_off[s], k,
                                                                                 d.vbuf.p, d.ubuf.p, cs, pl.max_r);
            for (int32_t bi = nsb - 1; bi >= 0; --bi) {
                const int32_t K0 = bi * SB;
                const int32_t kb = std::min(SB, k - K0);
                const unsigned grid = (unsigned)std::max(1, (K0 + NB - 1) / NB);
                bwd_push<T><<<dim3(grid, 1, nc), 256, 0, h->stream>>>(wbuf + pl.w_off[s], r, K0, kb, d.ubuf.p,
                                                                     xp + pl.sn_first[s], cs, pl.max_r);
            }
        }
        if (L == pl.chain_L0 && nchain > 0)
            bwd_chain<T><<<(unsigned)nchain, 64 * SW, 0, h->stream>>>(
                d.chain_comp_ptr.p, d.chain_grp_ptr.p, d.chain_sn.p, d.sn_first.p, d.sn_rptr.p, d.sn_rows.p,
                d.fr_off.p, front, xp);
        int32_t s0 = pl.lvl_small_ptr[L];
        const int32_t s1 = pl.lvl_small_ptr[L + 1], nt = pl.lvl_tiny_cnt[L];
        if (nt > 0) {
            bwd_tiny<T><<<(nt + 15) / 16, 256, 0, h->stream>>>(nt, d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
                                                                d.sn_rows.p, d.fr_off.p, front, xp);
            s0 += nt;
        }
        if (s1 > s0)
            bwd_small<T><<<(s1 - s0 + SW - 1) / SW, 64 * SW, 0, h->stream>>>(s1 - s0, d.lvl_small_sn.p + s0, d.sn_first.p, d.sn_rptr.p,
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

static int enqueue_solve(qg_handle *h, void *arg) {
    return *static_cast<const int *>(arg) == QG_FP32_IR
               ? solve_perm<float>(h, h->d.front32.p, h->d.sinv32.p, h->d.w32.p)
               : solve_perm<double>(h, h->d.front64.p, h->d.sinv64.p, h->d.w64.p);
}

int launch_solve(qg_handle *h, const double *rhs, double *x, int precision) {
    const int32_t N = h->N;
    const unsigned g = (unsigned)((N + 255) / 256);
    gather_perm<<<g, 256, 0, h->stream>>>(rhs, h->d.perm.p, h->d.xp.p, N);
    // the sweeps work on the permuted vector xp and the handle's own buffers only, so one capture per
    // factor precision serves every right-hand side
    int prec = precision;
    int rc = h->st.graphs ? graph_replay(h, h->g_solve[precision == QG_FP32_IR ? 1 : 0], enqueue_solve, &prec)
                          : enqueue_solve(h, &prec);
    if (rc) return rc;
    scatter_perm<<<g, 256, 0, h->stream>>>(h->d.xp.p, h->d.perm.p, x, N);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

}  // namespace qg
