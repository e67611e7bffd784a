// Per-cone formulas shared by the cone kernels: one thread per cone, or one
// wavefront per cone (lane a handles entries a, a + 64, ...; every inner
// product is a butterfly sum, after which all lanes hold the same value).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qg {

// J-norm sqrt(u'Ju) of one second-order cone, as sqrt((u0 - |u1|)(u0 + |u1|)).
__device__ inline double jnorm(const double *u, int32_t q) {
    double n1 = 0.0;
    for (int32_t a = 1; a < q; ++a) n1 += u[a] * u[a];
    n1 = sqrt(n1);
    return sqrt((u[0] - n1) * (u[0] + n1));
}

// Maximum step of one second-order cone of q entries (u interior), one thread:
// 1/max(0, |rho1| - rho0) with the rho of the header, +inf when unbounded.
__device__ inline double soc_max_step(const double *uk, const double *dk, int32_t q) {
    const double uJ = jnorm(uk, q);
    double r0 = uk[0] / uJ * dk[0];
    for (int32_t c = 1; c < q; ++c) r0 -= uk[c] / uJ * dk[c];
    r0 /= uJ;
    const double coef = (r0 * uJ + dk[0]) / (1.0 + uk[0] / uJ);
    double n1 = 0.0;
    for (int32_t c = 1; c < q; ++c) {
        const double v = (dk[c] - coef * (uk[c] / uJ)) / uJ;
        n1 += v * v;
    }
    const double den = sqrt(n1) - r0;
    return den > 0.0 ? 1.0 / den : INFINITY;
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// sqrt(u'Ju) as sqrt((u0 - |u1|)(u0 + |u1|)), one wavefront
__device__ inline double wave_jnorm(const double *u, int32_t q, int lane) {
    double t = 0.0;
    for (int32_t a = 1 + lane; a < q; a += 64) t += u[a] * u[a];
    const double n1 = sqrt(wave_sum(t));
    return sqrt((u[0] - n1) * (u[0] + n1));
}

// Maximum step of one second-order cone, one wavefront (same formula as
// soc_max_step); every lane returns the same value, +inf when unbounded.
__device__ inline double wave_soc_max_step(const double *uk, const double *dk, int32_t q, int lane) {
    const double uJ = wave_jnorm(uk, q, lane);
    double r1 = 0.0;
    for (int32_t c = 1 + lane; c < q; c += 64) r1 += uk[c] / uJ * dk[c];
    const double r0 = (uk[0] / uJ * dk[0] - wave_sum(r1)) / uJ;
    const double coef = (r0 * uJ + dk[0]) / (1.0 + uk[0] / uJ);
    double n1 = 0.0;
    for (int32_t c = 1 + lane; c < q; c += 64) {
        const double v = (dk[c] - coef * (uk[c] / uJ)) / uJ;
        n1 += v * v;
    }
    const double den = sqrt(wave_sum(n1)) - r0;
    return den > 0.0 ? 1.0 / den : INFINITY;
}

}  // namespace qg
