// Shared constants and small device helpers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qg {

// Fronts with r <= SMALL_R are factored and solved one workgroup per front
// entirely in LDS (r * r * 8 bytes <= 128 KiB of the 160 KiB per CU);
// larger fronts use the blocked multi-kernel path: panels of NB columns
// inside super-panels of SB columns, whose trailing update runs once per
// super-panel (rank SB).
constexpr int SMALL_R = 128;
constexpr int NB = 64;
constexpr int SB = 256;
// Outer blocks of large fronts: SB-column super-panels are factored four at a time; the columns
// beyond an outer block receive its updates as one rank-OB update (fewer passes over the trailing
// matrix than rank-SB updates).
constexpr int OB = 1024;
constexpr int32_t OB_WIDE_R = 16384;   // fronts of 1024 < r <= OB_WIDE_R use outer blocks of SB columns
// Rows of the largest front: the trailing-update kernels address a front's columns with 32-bit byte
// offsets (a larger front, 5.6e14 bytes in FP64, would not fit in any memory anyway).
constexpr int32_t MAX_FRONT_R = (1 << 23) - 1;
// Chains of small fronts on the narrow upper levels of deep elimination trees
// (one workgroup per component): levels with fewer than CHAIN_LEVEL_MIN
// fronts, fronts of at most CHAIN_R rows.
constexpr int CHAIN_LEVEL_MIN = 1024;
constexpr int CHAIN_R = 32;
constexpr int CHAIN_WIDTH_MAX = 8;   // a component's fronts per level, on average
// Tiny fronts (at most TINY_R rows) on levels that hold at least TINY_MIN of them: 16 lanes per
// front, 16 fronts per 256-thread workgroup, in the factorization and both solve sweeps.
constexpr int TINY_R = 16;
// Tiny fronts of at most TINY_R8 rows are factored in 8 x 8 LDS tiles (more workgroups per CU).
constexpr int32_t TINY_R8 = 8;
constexpr int TINY_MIN = 2048;
// Levels with fewer small fronts than this (all of at most CHAIN_R rows) solve them on the register
// path of the chains.
constexpr int REG_LEVEL_MAX = 4096;
// Lanes per matrix row in the sparse matrix-vector products (16 rows per
// 256-thread block) where a kernel has one fixed mapping; the residual
// reductions choose 4 or 16 from the rows' average length.
constexpr int RL = 16;
// Blocks per problem of the residual reductions (grid-stride over the rows).
constexpr int32_t RED_BLOCKS = 2048;
// Threads of the second reduction pass: one wavefront per scalar slot of the stopping test.
constexpr int FINISH_THREADS = 1024;
// Second-order cones with q >= QBIG entries are handled one wavefront per
// cone (lane-strided entries, butterfly sums); smaller cones one thread each.
constexpr int QBIG = 32;
// (3,3)-block entries of a big cone written per workgroup.
constexpr int BIG_CHUNK = 2048;

// Kind of a permuted KKT column: primal x, equality y, cone z.  Pivot signs
// of the quasi-definite matrix: + for x, - for y and z; static
// regularization +delta on x, -delta on y, none on z.
__host__ __device__ inline double pivot_sign(int8_t kind) { return kind == 0 ? 1.0 : -1.0; }
__host__ __device__ inline double static_reg(int8_t kind, double delta) {
    return kind == 0 ? delta : (kind == 1 ? -delta : 0.0);
}

// Maximum that propagates NaN (fmax drops it): a NaN anywhere in a max-norm
// must fail the tests built on it, never pass them.
__host__ __device__ inline double nan_max(double a, double b) { return (a != a || a > b) ? a : b; }

// p[i] if ok, else 0, with no branch: the address falls back to p[0] (which
// must be valid) when !ok.  A conditional load compiles to an exec-masked
// block that waits for its own result, so the loads of a loop would run one
// after another; this form keeps them all in flight.
template <typename T>
__device__ inline T ld_or0(const T *__restrict__ p, int64_t i, bool ok) {
    const T v = p[ok ? i : 0];
    return ok ? v : T(0);
}

// Offset of the block W_J of super-block J0 (a multiple of SB) within a large
// front's W storage: the earlier super-blocks are full, (r - J1') x SB each.
__host__ __device__ inline int64_t w_block_offset(int64_t r, int64_t J0) {
    const int64_t n = J0 / SB;
    return SB * (n * r - SB * n * (n + 1) / 2);
}

// Identical copies of a large front in a batch of problems on one pattern
// (qg_setup_batch) are factored and solved by one launch, copy z on
// blockIdx.z: the element distances between consecutive copies in each
// buffer (all zero for a single problem).
struct CopyStride {
    int64_t f = 0;       // front storage
    int64_t dinv = 0;    // inverses of the NB x NB diagonal blocks
    int64_t sinv = 0;    // inverses of the SB x SB diagonal blocks
    int64_t w = 0;       // W_J blocks
    int64_t task = 0;    // solve work vector (task slots)
    int32_t col = 0;     // permuted columns
    int32_t front = 0;   // front index
};

// Problem of cone unit t in a batch of kb problems (units: the l = kb l1 orthant
// entries, then the kb nsoc1 second-order cones, problem by problem in each
// part); units past the end count for the last problem.  kb = 1: always 0.
__host__ __device__ inline int32_t cone_problem(int32_t t, int32_t l, int32_t l1, int32_t nsoc1, int32_t kb) {
    const int32_t i = t < l ? t / l1 : (nsoc1 > 0 ? (t - l) / nsoc1 : 0);
    return i < kb ? i : kb - 1;
}

// Value of lane `src` (uniform over the wavefront) of v, for every lane.
__device__ inline float lane_bcast(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double lane_bcast(double v, int src) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

struct RegParams {
    double delta;     // static regularization
    double eps;       // dynamic threshold
    double dyn;       // dynamic replacement magnitude
};

}  // namespace qg
