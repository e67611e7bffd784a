// Maximum step over a product of cones without any device allocation
// (qg_max_step_noalloc in qg.h): the line search of the Newton step
// (alpha = sup{a >= 0 : u + a du in K}, per cone in closed form, then the
// minimum over the cones), for callers that cannot allocate device memory.
//
// Its only device memory beyond the caller's inputs is `scratch`, a
// file-scope array: one partial minimum per workgroup, then the final value.
// Host code never uses the array's name as an address: the address of each
// device's copy is looked up once per device with hipGetSymbolAddress and
// kept in scratch_ptr.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "cone_math.hpp"
#include "kernels.hpp"
#include "qg.h"

namespace qg {
namespace {

constexpr int32_t NA_THREADS = 256;
// One partial per workgroup of NA_THREADS cone units, plus one slot for the result.
constexpr int32_t NA_MAX_BLOCKS = QG_NOALLOC_MAX_UNITS / NA_THREADS;
static_assert(QG_NOALLOC_MAX_UNITS % NA_THREADS == 0, "whole workgroups");

__device__ __align__(256) double scratch[NA_MAX_BLOCKS + 1];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
double *scratch_ptr[MAX_DEVICES] = {};

// Address of this device's copy of `scratch` (looked up on first use per device).
hipError_t scratch_of(int dev, double **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

// Unit t < l: orthant entry t; unit l + k: second-order cone k.  A thread
// handles its unit when it is an orthant entry or a cone of fewer than QBIG
// entries; cones of QBIG entries or more in the wavefront's 64 units are
// handled one after another by the whole wavefront (the formula of the
// handle's one-wavefront-per-cone kernel).  Each workgroup writes the minimum
// of its units to partial[blockIdx.x]; nothing is accumulated across calls.
__global__ void __launch_bounds__(NA_THREADS) noalloc_step(int32_t l, int32_t nsoc,
                                                           const int32_t *__restrict__ soc_off,
                                                           const double *__restrict__ u,
                                                           const double *__restrict__ du,
                                                           double *__restrict__ partial) {
    const int32_t t = blockIdx.x * NA_THREADS + threadIdx.x;
    const int lane = threadIdx.x & 63;
    double a = INFINITY;
    bool big = false;
    if (t < l) {
        if (du[t] < 0.0) a = -u[t] / du[t];
    } else if (t - l < nsoc) {
        const int32_t k = t - l;
        const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
        if (q < QBIG) a = soc_max_step(u + off, du + off, q);
        else big = true;
    }
    uint64_t pending = __ballot(big);
    while (pending) {
        const int src = __ffsll((unsigned long long)pending) - 1;
        pending &= pending - 1;
        const int32_t k = blockIdx.x * NA_THREADS + (threadIdx.x & ~63) + src - l;
        const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
        const double ak = wave_soc_max_step(u + off, du + off, q, lane);
        if (lane == src) a = ak;
    }
    for (int o = 32; o > 0; o >>= 1) a = fmin(a, __shfl_xor(a, o));
    __shared__ double sh[NA_THREADS / 64];
    if (lane == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = sh[0];
        for (int w = 1; w < NA_THREADS / 64; ++w) v = fmin(v, sh[w]);
        partial[blockIdx.x] = v;
    }
}

// out = min(partial[0..nblk)), one workgroup
__global__ void __launch_bounds__(NA_THREADS) noalloc_finish(const double *__restrict__ partial, int32_t nblk,
                                                             double *__restrict__ out) {
    double v = INFINITY;
    for (int32_t b = threadIdx.x; b < nblk; b += NA_THREADS) v = fmin(v, partial[b]);
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    __shared__ double sh[NA_THREADS / 64];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < NA_THREADS / 64; ++w) v = fmin(v, sh[w]);
        *out = v;
    }
}

}  // namespace
}  // namespace qg

extern "C" int qg_max_step_noalloc(qg_int l, qg_int nsoc, const qg_int *soc_off, const double *u,
                                   const double *du, double *alpha, void *hip_stream) {
    using namespace qg;
    if (l < 0 || nsoc < 0 || !alpha || (nsoc > 0 && !soc_off)) return QG_ERR_ARG;
    const int64_t units = (int64_t)l + nsoc;
    if (units > QG_NOALLOC_MAX_UNITS) return QG_ERR_SIZE;
    if (units == 0) {
        *alpha = INFINITY;
        return QG_OK;
    }
    if (!u || !du) return QG_ERR_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return QG_ERR_DEVICE;
    double *buf = nullptr;
    if (scratch_of(dev, &buf) != hipSuccess) return QG_ERR_HIP;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int32_t nblk = (int32_t)((units + NA_THREADS - 1) / NA_THREADS);
    noalloc_step<<<nblk, NA_THREADS, 0, st>>>(l, nsoc, soc_off, u, du, buf);
    if (hipGetLastError() != hipSuccess) return QG_ERR_HIP;
    noalloc_finish<<<1, NA_THREADS, 0, st>>>(buf, nblk, buf + NA_MAX_BLOCKS);
    if (hipGetLastError() != hipSuccess) return QG_ERR_HIP;
    double a = 0.0;
    if (hipMemcpyAsync(&a, buf + NA_MAX_BLOCKS, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess)
        return QG_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess) return QG_ERR_HIP;
    *alpha = a;
    return QG_OK;
}
