// Shared constants and small device helpers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qg {

// Fronts with r <= SMALL_R are factored and solved one workgroup per front
// entirely in LDS (r * r * 8 bytes <= 32 KiB); larger fronts use the
// blocked multi-kernel path with panels of NB columns.
constexpr int SMALL_R = 64;
constexpr int NB = 64;

// Kind of a permuted KKT column: primal x, equality y, cone z.  Pivot signs
// of the quasi-definite matrix: + for x, - for y and z; static
// regularization +delta on x, -delta on y, none on z.
__host__ __device__ inline double pivot_sign(int8_t kind) { return kind == 0 ? 1.0 : -1.0; }
__host__ __device__ inline double static_reg(int8_t kind, double delta) {
    return kind == 0 ? delta : (kind == 1 ? -delta : 0.0);
}

struct RegParams {
    double delta;     // static regularization
    double eps;       // dynamic threshold
    double dyn;       // dynamic replacement magnitude
};

}  // namespace qg
