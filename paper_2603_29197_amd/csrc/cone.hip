// Cone operations of the Newton step (paper Sec. 2.1: Jordan products and
// Nesterov-Todd scalings, implemented per cone and run in parallel, Sec. 2.3):
// one thread per orthant entry, one thread per second-order cone of fewer
// than QBIG entries, one wavefront per larger cone (the *_big kernels).
//
// Formulas (standard SOC Jordan algebra; NT scaling as in Vandenberghe's
// cone-QP method, which the paper's solver implements):
//   J = diag(1, -I); e = (1, 0, .., 0); u o v = (u'v, u0 v1 + v0 u1);
//   lam \ v: rho = lam0^2 - |lam1|^2, x0 = (lam0 v0 - lam1'v1)/rho,
//            x1 = (v1 - x0 lam1)/lam0;
//   NT: s_n = sqrt(s'Js), z_n = sqrt(z'Jz) (as sqrt((u0-|u1|)(u0+|u1|))),
//       sb = s/s_n, zb = z/z_n, gamma = sqrt((1 + zb'sb)/2),
//       wb = (sb + J zb)/(2 gamma), beta = sqrt(s_n/z_n), W = beta Wb,
//       Wb u = (wb'u, u1 + wb1 (u0 + wb1'u1/(1 + wb0))),
//       W^-1 = (1/beta) J Wb J,  W'W = beta^2 (2 wb wb' - J);
//   orthant: w = sqrt(s/z), lam = sqrt(s z), W'W = s/z.
//   Max step (u interior): orthant -u/du for du < 0; SOC with uJ = sqrt(u'Ju),
//   ub = u/uJ, rho0 = ub'J du/uJ, rho1 = (du1 - ((rho0 uJ + du0)/(1+ub0)) ub1)/uJ:
//   1/max(0, |rho1| - rho0).
#include "cone_math.hpp"
#include "vec.hpp"

#include <algorithm>

namespace qg {

// out = beta * Wb u  (inv = 0)   or   (1/beta) J Wb J u  (inv = 1)
__device__ inline void soc_w_apply(const double *wb, double beta, const double *u, double *out, int32_t q,
                                   int inv) {
    const double sg = inv ? -1.0 : 1.0;
    double w1u1 = 0.0;
    for (int32_t a = 1; a < q; ++a) w1u1 += wb[a] * (sg * u[a]);
    const double u0 = u[0];
    const double coef = u0 + w1u1 / (1.0 + wb[0]);
    const double scale = inv ? 1.0 / beta : beta;
    out[0] = scale * (wb[0] * u0 + w1u1);
    for (int32_t a = 1; a < q; ++a) out[a] = scale * sg * (sg * u[a] + wb[a] * coef);
}

// NT scaling and the (3,3) block of K.  block == 1 writes the derivative
// block -sym(Arw(z)^-1 Arw(s)) instead of -W'W (orthant: -s/z either way).
__global__ void scaling_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                               const int64_t *__restrict__ blk_off, const int64_t *__restrict__ blk33,
                               const double *__restrict__ s, const double *__restrict__ z,
                               double *__restrict__ w, double *__restrict__ wbar, double *__restrict__ beta,
                               double *__restrict__ lam, double *__restrict__ kval, int block) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t < l) {
        const double si = s[t], zi = z[t];
        w[t] = sqrt(si / zi);
        if (lam) lam[t] = sqrt(si * zi);
        kval[blk33[t]] = -(si / zi);
        return;
    }
    const int32_t k = t - l;
    if (k >= nsoc) return;
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    if (q >= QBIG) return;
    const double *sk = s + off, *zk = z + off;
    double *wb = wbar + (off - l);
    const int64_t base = l + blk_off[k];
    if (block == 1) {
        // H = Arw(z)^-1 Arw(s); Arw(z)^-1 = (1/d)[[z0, -z1'], [-z1, (d/z0) I + z1 z1'/z0]]
        const double z0 = zk[0];
        double z1z1 = 0.0;
        for (int32_t a = 1; a < q; ++a) z1z1 += zk[a] * zk[a];
        const double dz = z0 * z0 - z1z1;
        for (int32_t bcol = 0; bcol < q; ++bcol)
            for (int32_t arow = 0; arow <= bcol; ++arow) {
                // H(i, j) = sum_t Ainv(i, t) Arw(s)(t, j); symmetric part (H(a,b) + H(b,a)) / 2
                double hab = 0.0, hba = 0.0;
                for (int32_t pass = 0; pass < 2; ++pass) {
                    const int32_t i = pass ? bcol : arow, j = pass ? arow : bcol;
                    double acc = 0.0;
                    for (int32_t tt = 0; tt < q; ++tt) {
                        double ai;   // Ainv(i, tt) * d
                        if (i == 0 && tt == 0) ai = z0;
                        else if (i == 0) ai = -zk[tt];
                        else if (tt == 0) ai = -zk[i];
                        else ai = (i == tt ? dz / z0 : 0.0) + zk[i] * zk[tt] / z0;
                        double as;   // Arw(s)(tt, j)
                        if (tt == 0 && j == 0) as = sk[0];
                        else if (tt == 0) as = sk[j];
                        else if (j == 0) as = sk[tt];
                        else as = (tt == j) ? sk[0] : 0.0;
                        acc += ai * as;
                    }
                    if (pass) hba = acc / dz; else hab = acc / dz;
                }
                kval[blk33[base + (int64_t)bcol * (bcol + 1) / 2 + arow]] = -0.5 * (hab + hba);
            }
        return;
    }
    const double sn = jnorm(sk, q), zn = jnorm(zk, q);
    double dot = 0.0;
    for (int32_t a = 0; a < q; ++a) dot += (zk[a] / zn) * (sk[a] / sn);
    const double gamma = sqrt((1.0 + dot) * 0.5);
    for (int32_t a = 0; a < q; ++a) {
        const double zb = zk[a] / zn, sb = sk[a] / sn;
        wb[a] = (sb + (a == 0 ? zb : -zb)) / (2.0 * gamma);
    }
    const double bt = sqrt(sn / zn);
    beta[k] = bt;
    if (lam) soc_w_apply(wb, bt, zk, lam + off, q, 0);
    const double b2 = bt * bt;
    for (int32_t bcol = 0; bcol < q; ++bcol)
        for (int32_t arow = 0; arow <= bcol; ++arow) {
            const double jab = (arow == bcol) ? (arow == 0 ? 1.0 : -1.0) : 0.0;
            kval[blk33[base + (int64_t)bcol * (bcol + 1) / 2 + arow]] = -b2 * (2.0 * wb[arow] * wb[bcol] - jab);
        }
}

// op: 0 W u, 1 W^-1 u, 2 W'W u, 3 u o v, 4 u \ v
__global__ void cone_op_kernel(int op, int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                               const double *__restrict__ w, const double *__restrict__ wbar,
                               const double *__restrict__ beta, const double *__restrict__ u,
                               const double *__restrict__ v, double *__restrict__ out) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t < l) {
        const double ui = u[t];
        double r;
        switch (op) {
            case 0: r = w[t] * ui; break;
            case 1: r = ui / w[t]; break;
            case 2: r = w[t] * w[t] * ui; break;
            case 3: r = ui * v[t]; break;
            default: r = v[t] / ui; break;
        }
        out[t] = r;
        return;
    }
    const int32_t k = t - l;
    if (k >= nsoc) return;
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    if (q >= QBIG) return;
    const double *uk = u + off;
    double *ok = out + off;
    const double *wb = wbar + (off - l);
    if (op == 0 || op == 1) {
        soc_w_apply(wb, beta[k], uk, ok, q, op);
    } else if (op == 2) {
        // beta^2 (2 wb (wb'u) - J u)
        double wu = 0.0;
        for (int32_t a = 0; a < q; ++a) wu += wb[a] * uk[a];
        const double b2 = beta[k] * beta[k];
        for (int32_t a = 0; a < q; ++a) ok[a] = b2 * (2.0 * wb[a] * wu - (a == 0 ? uk[a] : -uk[a]));
    } else if (op == 3) {
        const double *vk = v + off;
        double dot = 0.0;
        for (int32_t a = 0; a < q; ++a) dot += uk[a] * vk[a];
        const double u0 = uk[0], v0 = vk[0];
        for (int32_t a = 1; a < q; ++a) ok[a] = u0 * vk[a] + v0 * uk[a];
        ok[0] = dot;
    } else {
        const double *vk = v + off;
        double l1l1 = 0.0, l1v1 = 0.0;
        for (int32_t a = 1; a < q; ++a) { l1l1 += uk[a] * uk[a]; l1v1 += uk[a] * vk[a]; }
        const double rho = uk[0] * uk[0] - l1l1;
        const double x0 = (uk[0] * vk[0] - l1v1) / rho;
        for (int32_t a = 1; a < q; ++a) ok[a] = (vk[a] - x0 * uk[a]) / uk[0];
        ok[0] = x0;
    }
}

// ds = tsign * tvec - W'W dz   (tvec may be s with tsign = -1: affine step)
__global__ void ds_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                          const double *__restrict__ w, const double *__restrict__ wbar,
                          const double *__restrict__ beta, const double *__restrict__ tvec, double tsign,
                          const double *__restrict__ dz, double *__restrict__ ds) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t < l) {
        ds[t] = tsign * tvec[t] - w[t] * w[t] * dz[t];
        return;
    }
    const int32_t k = t - l;
    if (k >= nsoc) return;
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    if (q >= QBIG) return;
    const double *wb = wbar + (off - l);
    double wu = 0.0;
    for (int32_t a = 0; a < q; ++a) wu += wb[a] * dz[off + a];
    const double b2 = beta[k] * beta[k];
    for (int32_t a = 0; a < q; ++a) {
        const double whw = b2 * (2.0 * wb[a] * wu - (a == 0 ? dz[off + a] : -dz[off + a]));
        ds[off + a] = tsign * tvec[off + a] - whw;
    }
}

// t = W'(lam \ d), d = -lam o lam - (W^-1 ds_a) o (W dz_a) + sigma mu e, with
// sigma = clip((1 - alpha_a)^3, 0, 1) and alpha_a = min(1, amin[0], amin[1]).
__global__ void corrector_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                                 const double *__restrict__ w, const double *__restrict__ wbar,
                                 const double *__restrict__ beta, const double *__restrict__ lam,
                                 const double *__restrict__ dsa, const double *__restrict__ dza,
                                 const unsigned long long *__restrict__ amin, const double *__restrict__ mu,
                                 double sigma_mu_fixed, double *__restrict__ tout, double *__restrict__ alpha_rec,
                                 int32_t l1, int32_t nsoc1, int32_t kb) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    const int32_t inst = cone_problem(t, l, l1, nsoc1, kb);
    double smu;
    if (sigma_mu_fixed >= 0.0) {
        smu = sigma_mu_fixed;
    } else {
        const unsigned long long *am = amin + 4 * inst;
        const double aa = fmin(1.0, fmin(__longlong_as_double((long long)am[0]),
                                         __longlong_as_double((long long)am[1])));
        const double om = 1.0 - aa;
        const double sigma = fmin(1.0, fmax(0.0, om * om * om));
        smu = sigma * mu[inst];
        if (t == 0 && alpha_rec) alpha_rec[0] = aa;
    }
    if (t < l) {
        const double li = lam[t], wi = w[t];
        const double d = -li * li - (dsa[t] / wi) * (wi * dza[t]) + smu;
        tout[t] = wi * (d / li);
        return;
    }
    const int32_t k = t - l;
    if (k >= nsoc) return;
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    if (q >= QBIG) return;
    const double *wb = wbar + (off - l);
    const double bt = beta[k];
    const double *lk = lam + off;
    const double *ua = dsa + off, *ub = dza + off;
    // A = W^-1 ds_a = (1/bt) J Wb J ds_a,  B = W dz_a = bt Wb dz_a, componentwise:
    //   A0 = (w0 u0 - w1'u1)/bt,  Aa = (u_a - w_a (u0 - w1'u1/(1+w0)))/bt
    //   B0 = bt (w0 v0 + w1'v1),   Ba = bt (v_a + w_a (v0 + w1'v1/(1+w0)))
    double wu = 0.0, wv = 0.0, ll = 0.0;
    for (int32_t a = 1; a < q; ++a) { wu += wb[a] * ua[a]; wv += wb[a] * ub[a]; }
    for (int32_t a = 0; a < q; ++a) ll += lk[a] * lk[a];
    const double ca = ua[0] - wu / (1.0 + wb[0]);
    const double cb = ub[0] + wv / (1.0 + wb[0]);
    const double A0 = (wb[0] * ua[0] - wu) / bt;
    const double B0 = bt * (wb[0] * ub[0] + wv);
    double ab = A0 * B0;
    for (int32_t a = 1; a < q; ++a) ab += ((ua[a] - wb[a] * ca) / bt) * (bt * (ub[a] + wb[a] * cb));
    // d = -lam o lam - A o B + smu e;  x = lam \ d;  t = W x
    const double d0 = -ll - ab + smu;
    double l1l1 = 0.0, l1d1 = 0.0;
    for (int32_t a = 1; a < q; ++a) {
        const double Aa = (ua[a] - wb[a] * ca) / bt, Ba = bt * (ub[a] + wb[a] * cb);
        const double da = -(2.0 * lk[0] * lk[a]) - (A0 * Ba + B0 * Aa);
        l1l1 += lk[a] * lk[a];
        l1d1 += lk[a] * da;
    }
    const double rho = lk[0] * lk[0] - l1l1;
    const double x0 = (lk[0] * d0 - l1d1) / rho;
    double wx = 0.0;
    for (int32_t a = 1; a < q; ++a) {
        const double Aa = (ua[a] - wb[a] * ca) / bt, Ba = bt * (ub[a] + wb[a] * cb);
        const double da = -(2.0 * lk[0] * lk[a]) - (A0 * Ba + B0 * Aa);
        wx += wb[a] * ((da - x0 * lk[a]) / lk[0]);
    }
    const double cx = x0 + wx / (1.0 + wb[0]);
    double *to = tout + off;
    for (int32_t a = 1; a < q; ++a) {
        const double Aa = (ua[a] - wb[a] * ca) / bt, Ba = bt * (ub[a] + wb[a] * cb);
        const double da = -(2.0 * lk[0] * lk[a]) - (A0 * Ba + B0 * Aa);
        const double xa = (da - x0 * lk[a]) / lk[0];
        to[a] = bt * (xa + wb[a] * cx);
    }
    to[0] = bt * (wb[0] * x0 + wx);
}

// per-cone maximum step, min-reduced into amin[slot] (ordered bits of a
// nonnegative double)
__device__ inline double cone_step(int32_t t, int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                                   const double *__restrict__ u, const double *__restrict__ du) {
    double a = INFINITY;
    if (t < l) {
        if (du[t] < 0.0) a = -u[t] / du[t];
    } else if (t - l < nsoc && soc_off[t - l + 1] - soc_off[t - l] < QBIG) {
        const int32_t k = t - l;
        const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
        a = soc_max_step(u + off, du + off, q);
    }
    return a;
}

// One problem: a grid-stride loop over the cone units, a block minimum and one atomic per block.
__global__ void __launch_bounds__(256) step_kernel_one(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                                                       const double *__restrict__ u, const double *__restrict__ du,
                                                       unsigned long long *__restrict__ amin) {
    double a = INFINITY;
    for (int32_t t = blockIdx.x * 256 + threadIdx.x; t < l + nsoc; t += gridDim.x * 256)
        a = fmin(a, cone_step(t, l, nsoc, soc_off, u, du));
    for (int off = 32; off > 0; off >>= 1) a = fmin(a, __shfl_xor(a, off));
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double b = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
        if (b < INFINITY) atomicMin(amin, (unsigned long long)__double_as_longlong(b));
    }
}

// A batch: one thread per cone unit, the minimum of each problem
__global__ void step_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                            const double *__restrict__ u, const double *__restrict__ du,
                            unsigned long long *__restrict__ amin, int32_t l1, int32_t nsoc1, int32_t kb) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    double a = cone_step(t, l, nsoc, soc_off, u, du);
    // the minimum of each problem: a wave min and one atomic per wave when the wave's cones belong to
    // one problem, else one atomic per cone
    const int32_t inst = cone_problem(t, l, l1, nsoc1, kb);
    if (__all(inst == __shfl(inst, 0))) {
        for (int off = 32; off > 0; off >>= 1) a = fmin(a, __shfl_xor(a, off));
        if ((threadIdx.x & 63) == 0) atomicMin(amin + 4 * inst, (unsigned long long)__double_as_longlong(a));
    } else if (a < INFINITY) {
        atomicMin(amin + 4 * inst, (unsigned long long)__double_as_longlong(a));
    }
}

__global__ void reset_steps_kernel(unsigned long long *amin, int32_t n) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) amin[i] = (unsigned long long)__double_as_longlong(INFINITY);
}

// lambda_min per cone (orthant u_i, SOC u0 - |u1|), reduced as max(-lambda_min)
__global__ void __launch_bounds__(256) lmin_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                                                   const double *__restrict__ u, double *__restrict__ partials) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    double v = -INFINITY;
    if (t < l) {
        v = -u[t];
    } else if (t - l < nsoc && soc_off[t - l + 1] - soc_off[t - l] < QBIG) {
        const int32_t k = t - l;
        const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
        double n1 = 0.0;
        for (int32_t a = 1; a < q; ++a) n1 += u[off + a] * u[off + a];
        v = -(u[off] - sqrt(n1));
    }
    for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o));
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = nan_max(nan_max(sh[0], sh[1]), nan_max(sh[2], sh[3]));
}

__global__ void __launch_bounds__(64) finish_max(const double *__restrict__ partials, int32_t nblk,
                                                  double *__restrict__ out) {
    double v = -INFINITY;
    for (int32_t b = threadIdx.x; b < nblk; b += 64) v = nan_max(v, partials[b]);
    for (int o = 32; o > 0; o >>= 1) v = nan_max(v, __shfl_xor(v, o));
    if (threadIdx.x == 0) *out = v;
}

// Batches: the shift of the initial point is each problem's own.  Key of a
// double whose unsigned integer order is the numeric order (a NaN above +inf),
// for one atomicMax per cone into the problem's slot.
__device__ inline unsigned long long ordered_key(double v) {
    if (v != v) v = __longlong_as_double(0x7ff8000000000000LL);
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ULL);
}
__device__ inline double ordered_value(unsigned long long k) {
    return __longlong_as_double((long long)((k >> 63) ? (k & 0x7fffffffffffffffULL) : ~k));
}

__global__ void init_keys_kernel(unsigned long long *__restrict__ keys, int32_t kb) {
    const int32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < kb) keys[4 * i] = ordered_key(-INFINITY);
}

// max over each problem's cones of -lambda_min (one thread per cone, any size: the initial point only)
__global__ void lmin_inst_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                                 const double *__restrict__ u, unsigned long long *__restrict__ keys, int32_t l1,
                                 int32_t nsoc1, int32_t kb) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= l + nsoc) return;
    double v;
    if (t < l) {
        v = -u[t];
    } else {
        const int32_t k = t - l;
        const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
        double n1 = 0.0;
        for (int32_t a = 1; a < q; ++a) n1 += u[off + a] * u[off + a];
        v = -(u[off] - sqrt(n1));
    }
    atomicMax(keys + 4 * cone_problem(t, l, l1, nsoc1, kb), ordered_key(v));
}

// u += (1 + a_i) e on the cones of every problem i with a_i = max(-lambda_min) >= 0
__global__ void add_e_inst_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off,
                                  const unsigned long long *__restrict__ keys, double *__restrict__ u, int32_t l1,
                                  int32_t nsoc1, int32_t kb) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t >= l + nsoc) return;
    const double a = ordered_value(keys[4 * cone_problem(t, l, l1, nsoc1, kb)]);
    if (a < 0.0) return;
    if (t < l) u[t] += 1.0 + a;
    else u[soc_off[t - l]] += 1.0 + a;
}

// u += c e
__global__ void add_e_kernel(int32_t l, int32_t nsoc, const int32_t *__restrict__ soc_off, double c,
                             double *__restrict__ u) {
    const int32_t t = blockIdx.x * 256 + threadIdx.x;
    if (t < l) u[t] += c;
    else if (t - l < nsoc) u[soc_off[t - l]] += c;
}

// ---------------------------------------------------------------------------
// Cones with q >= QBIG: one wavefront per cone.  Lane a handles entries a,
// a + 64, ...; every inner product is a butterfly sum, after which all lanes
// hold the same value.  Same formulas as the per-thread kernels above.
// ---------------------------------------------------------------------------
// wavefront index among the big cones (4 wavefronts per 256-thread block)
__device__ inline int32_t big_wave() { return (int32_t)(blockIdx.x * 4 + (threadIdx.x >> 6)); }

// NT scaling of a big cone (wb, beta, lam); its (3,3) block is written by block_big.
// block == 1 stores the two sums block_big needs for -sym(Arw(z)^-1 Arw(s)) instead.
__global__ void __launch_bounds__(256) scaling_big(int32_t l, int32_t nbig, const int32_t *__restrict__ big,
                                                   const int32_t *__restrict__ soc_off, const double *__restrict__ s,
                                                   const double *__restrict__ z, double *__restrict__ wbar,
                                                   double *__restrict__ beta, double *__restrict__ lam,
                                                   double *__restrict__ bigsc, int block) {
    const int32_t gw = big_wave();
    if (gw >= nbig) return;
    const int lane = threadIdx.x & 63;
    const int32_t k = big[gw];
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    const double *sk = s + off, *zk = z + off;
    if (block == 1) {
        double zz = 0.0, zs = 0.0;
        for (int32_t a = 1 + lane; a < q; a += 64) { zz += zk[a] * zk[a]; zs += zk[a] * sk[a]; }
        zz = wave_sum(zz);
        zs = wave_sum(zs);
        if (lane == 0) { bigsc[2 * gw] = zz; bigsc[2 * gw + 1] = zs; }
        return;
    }
    const double sn = wave_jnorm(sk, q, lane), zn = wave_jnorm(zk, q, lane);
    double dot = 0.0;
    for (int32_t a = lane; a < q; a += 64) dot += (zk[a] / zn) * (sk[a] / sn);
    dot = wave_sum(dot);
    const double gamma = sqrt((1.0 + dot) * 0.5);
    // wb[a] from (s, z): the lanes never read entries of wbar written by other lanes
    auto wbv = [&](int32_t a) {
        const double zb = zk[a] / zn, sb = sk[a] / sn;
        return (sb + (a == 0 ? zb : -zb)) / (2.0 * gamma);
    };
    double *wb = wbar + (off - l);
    for (int32_t a = lane; a < q; a += 64) wb[a] = wbv(a);
    const double bt = sqrt(sn / zn);
    if (lane == 0) beta[k] = bt;
    if (lam) {
        // lam = bt Wb z
        const double w0 = wbv(0);
        double w1z1 = 0.0;
        for (int32_t a = 1 + lane; a < q; a += 64) w1z1 += wbv(a) * zk[a];
        w1z1 = wave_sum(w1z1);
        const double coef = zk[0] + w1z1 / (1.0 + w0);
        double *lk = lam + off;
        if (lane == 0) lk[0] = bt * (w0 * zk[0] + w1z1);
        for (int32_t a = 1 + lane; a < q; a += 64) lk[a] = bt * (zk[a] + wbv(a) * coef);
    }
}

// (3,3) block entries of the big cones, BIG_CHUNK entries of one cone per
// workgroup (the host lists the chunks): entry t of a cone is (arow, bcol) of
// its upper triangle in column order, t = bcol (bcol + 1) / 2 + arow, so the
// reads of blk33 are contiguous.  block 0: -W'W = -beta^2 (2 wb wb' - J);
// block 1: -(H + H')/2 with d H = d Arw(z)^-1 Arw(s), d = z0^2 - |z1|^2:
//   (0,0) z0 s0 - z1's1; (0,j) z0 sj - s0 zj; (i,0) -zi s0 + (d/z0) si + zi z1's1/z0;
//   (i,j) -zi sj + [i=j] (d/z0) s0 + zi zj s0/z0.
__global__ void __launch_bounds__(256) block_big(int32_t l, const int32_t *__restrict__ big,
                                                 const int32_t *__restrict__ chunk_cone,
                                                 const int64_t *__restrict__ chunk_start,
                                                 const int32_t *__restrict__ soc_off,
                                                 const int64_t *__restrict__ blk_off,
                                                 const int64_t *__restrict__ blk33, const double *__restrict__ s,
                                                 const double *__restrict__ z, const double *__restrict__ wbar,
                                                 const double *__restrict__ beta, const double *__restrict__ bigsc,
                                                 double *__restrict__ kval, int block) {
    const int32_t j = chunk_cone[blockIdx.x];
    const int64_t st = chunk_start[blockIdx.x];
    const int32_t k = big[j];
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    const int64_t ne = (int64_t)q * (q + 1) / 2;
    const int64_t base = l + blk_off[k];
    const double *sk = s + off, *zk = z + off;
    const double *wb = wbar + (off - l);
    const double b2 = block == 1 ? 0.0 : beta[k] * beta[k];
    const double z0 = zk[0], s0 = sk[0];
    const double zz = block == 1 ? bigsc[2 * j] : 0.0, zs = block == 1 ? bigsc[2 * j + 1] : 0.0;
    const double dz = z0 * z0 - zz, dz0 = dz / z0;
    for (int i = threadIdx.x; i < BIG_CHUNK; i += 256) {
        const int64_t t = st + i;
        if (t >= ne) break;
        int32_t bcol = (int32_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((int64_t)(bcol + 1) * (bcol + 2) / 2 <= t) ++bcol;
        while ((int64_t)bcol * (bcol + 1) / 2 > t) --bcol;
        const int32_t arow = (int32_t)(t - (int64_t)bcol * (bcol + 1) / 2);
        double v;
        if (block == 1) {
            const double za = zk[arow], sa = sk[arow], zb = zk[bcol], sb = sk[bcol];
            double hsum;
            if (bcol == 0) hsum = 2.0 * (z0 * s0 - zs);
            else if (arow == 0) hsum = (z0 * sb - s0 * zb) + (-zb * s0 + dz0 * sb + zb * zs / z0);
            else hsum = -(za * sb + zb * sa) + (arow == bcol ? 2.0 * dz0 * s0 : 0.0) + 2.0 * za * zb * s0 / z0;
            v = -0.5 * hsum / dz;
        } else {
            const double jab = (arow == bcol) ? (arow == 0 ? 1.0 : -1.0) : 0.0;
            v = -b2 * (2.0 * wb[arow] * wb[bcol] - jab);
        }
        kval[blk33[base + t]] = v;
    }
}

// op: 0 W u, 1 W^-1 u, 2 W'W u, 3 u o v, 4 u \ v
__global__ void __launch_bounds__(256) cone_op_big(int op, int32_t l, int32_t nbig, const int32_t *__restrict__ big,
                                                   const int32_t *__restrict__ soc_off,
                                                   const double *__restrict__ wbar, const double *__restrict__ beta,
                                                   const double *__restrict__ u, const double *__restrict__ v,
                                                   double *__restrict__ out) {
    const int32_t gw = big_wave();
    if (gw >= nbig) return;
    const int lane = threadIdx.x & 63;
    const int32_t k = big[gw];
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    const double *uk = u + off;
    double *ok = out + off;
    const double *wb = wbar + (off - l);
    if (op == 0 || op == 1) {
        const double sg = op ? -1.0 : 1.0;
        double w1u1 = 0.0;
        for (int32_t a = 1 + lane; a < q; a += 64) w1u1 += wb[a] * (sg * uk[a]);
        w1u1 = wave_sum(w1u1);
        const double u0 = uk[0];
        const double coef = u0 + w1u1 / (1.0 + wb[0]);
        const double scale = op ? 1.0 / beta[k] : beta[k];
        if (lane == 0) ok[0] = scale * (wb[0] * u0 + w1u1);
        for (int32_t a = 1 + lane; a < q; a += 64) ok[a] = scale * sg * (sg * uk[a] + wb[a] * coef);
    } else if (op == 2) {
        double wu = 0.0;
        for (int32_t a = lane; a < q; a += 64) wu += wb[a] * uk[a];
        wu = wave_sum(wu);
        const double b2 = beta[k] * beta[k];
        for (int32_t a = lane; a < q; a += 64) ok[a] = b2 * (2.0 * wb[a] * wu - (a == 0 ? uk[a] : -uk[a]));
    } else if (op == 3) {
        const double *vk = v + off;
        double dot = 0.0;
        for (int32_t a = lane; a < q; a += 64) dot += uk[a] * vk[a];
        dot = wave_sum(dot);
        const double u0 = uk[0], v0 = vk[0];
        for (int32_t a = 1 + lane; a < q; a += 64) ok[a] = u0 * vk[a] + v0 * uk[a];
        if (lane == 0) ok[0] = dot;
    } else {
        const double *vk = v + off;
        double l1l1 = 0.0, l1v1 = 0.0;
        for (int32_t a = 1 + lane; a < q; a += 64) { l1l1 += uk[a] * uk[a]; l1v1 += uk[a] * vk[a]; }
        l1l1 = wave_sum(l1l1);
        l1v1 = wave_sum(l1v1);
        const double rho = uk[0] * uk[0] - l1l1;
        const double x0 = (uk[0] * vk[0] - l1v1) / rho;
        for (int32_t a = 1 + lane; a < q; a += 64) ok[a] = (vk[a] - x0 * uk[a]) / uk[0];
        if (lane == 0) ok[0] = x0;
    }
}

// ds = tsign * tvec - W'W dz
__global__ void __launch_bounds__(256) ds_big(int32_t l, int32_t nbig, const int32_t *__restrict__ big,
                                              const int32_t *__restrict__ soc_off, const double *__restrict__ wbar,
                                              const double *__restrict__ beta, const double *__restrict__ tvec,
                                              double tsign, const double *__restrict__ dz, double *__restrict__ ds) {
    const int32_t gw = big_wave();
    if (gw >= nbig) return;
    const int lane = threadIdx.x & 63;
    const int32_t k = big[gw];
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    const double *wb = wbar + (off - l);
    double wu = 0.0;
    for (int32_t a = lane; a < q; a += 64) wu += wb[a] * dz[off + a];
    wu = wave_sum(wu);
    const double b2 = beta[k] * beta[k];
    for (int32_t a = lane; a < q; a += 64) {
        const double whw = b2 * (2.0 * wb[a] * wu - (a == 0 ? dz[off + a] : -dz[off + a]));
        ds[off + a] = tsign * tvec[off + a] - whw;
    }
}

// t = W'(lam \ d), d = -lam o lam - (W^-1 ds_a) o (W dz_a) + sigma mu e (see corrector_kernel)
__global__ void __launch_bounds__(256) corrector_big(int32_t l, int32_t nbig, const int32_t *__restrict__ big,
                                                     const int32_t *__restrict__ soc_off,
                                                     const double *__restrict__ wbar,
                                                     const double *__restrict__ beta, const double *__restrict__ lam,
                                                     const double *__restrict__ dsa, const double *__restrict__ dza,
                                                     const unsigned long long *__restrict__ amin,
                                                     const double *__restrict__ mu, double sigma_mu_fixed,
                                                     double *__restrict__ tout, int32_t nsoc1) {
    const int32_t gw = big_wave();
    if (gw >= nbig) return;
    double smu;
    if (sigma_mu_fixed >= 0.0) {
        smu = sigma_mu_fixed;
    } else {
        const int32_t inst = big[gw] / nsoc1;
        const unsigned long long *am = amin + 4 * inst;
        const double aa = fmin(1.0, fmin(__longlong_as_double((long long)am[0]),
                                         __longlong_as_double((long long)am[1])));
        const double om = 1.0 - aa;
        smu = fmin(1.0, fmax(0.0, om * om * om)) * mu[inst];
    }
    const int lane = threadIdx.x & 63;
    const int32_t k = big[gw];
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    const double *wb = wbar + (off - l);
    const double bt = beta[k];
    const double *lk = lam + off;
    const double *ua = dsa + off, *ub = dza + off;
    double wu = 0.0, wv = 0.0, l1l1 = 0.0;
    for (int32_t a = 1 + lane; a < q; a += 64) {
        wu += wb[a] * ua[a];
        wv += wb[a] * ub[a];
        l1l1 += lk[a] * lk[a];
    }
    wu = wave_sum(wu);
    wv = wave_sum(wv);
    l1l1 = wave_sum(l1l1);
    const double w0 = wb[0], l0 = lk[0];
    const double ca = ua[0] - wu / (1.0 + w0);
    const double cb = ub[0] + wv / (1.0 + w0);
    const double A0 = (w0 * ua[0] - wu) / bt;
    const double B0 = bt * (w0 * ub[0] + wv);
    // tail entries of A = W^-1 ds_a, B = W dz_a and d
    auto da_of = [&](int32_t a) {
        const double Aa = (ua[a] - wb[a] * ca) / bt, Ba = bt * (ub[a] + wb[a] * cb);
        return -(2.0 * l0 * lk[a]) - (A0 * Ba + B0 * Aa);
    };
    double ab = 0.0, l1d1 = 0.0;
    for (int32_t a = 1 + lane; a < q; a += 64) {
        ab += ((ua[a] - wb[a] * ca) / bt) * (bt * (ub[a] + wb[a] * cb));
        l1d1 += lk[a] * da_of(a);
    }
    ab = A0 * B0 + wave_sum(ab);
    l1d1 = wave_sum(l1d1);
    const double d0 = -(l0 * l0 + l1l1) - ab + smu;
    const double rho = l0 * l0 - l1l1;
    const double x0 = (l0 * d0 - l1d1) / rho;
    double wx = 0.0;
    for (int32_t a = 1 + lane; a < q; a += 64) wx += wb[a] * ((da_of(a) - x0 * lk[a]) / l0);
    wx = wave_sum(wx);
    const double cx = x0 + wx / (1.0 + w0);
    double *to = tout + off;
    for (int32_t a = 1 + lane; a < q; a += 64) to[a] = bt * ((da_of(a) - x0 * lk[a]) / l0 + wb[a] * cx);
    if (lane == 0) to[0] = bt * (w0 * x0 + wx);
}

// per-cone maximum step, min-reduced into amin (see step_kernel)
__global__ void __launch_bounds__(256) step_big(int32_t nbig, const int32_t *__restrict__ big,
                                                const int32_t *__restrict__ soc_off, const double *__restrict__ u,
                                                const double *__restrict__ du, unsigned long long *__restrict__ amin,
                                                int32_t nsoc1) {
    const int32_t gw = big_wave();
    if (gw >= nbig) return;
    const int lane = threadIdx.x & 63;
    const int32_t k = big[gw];
    const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
    const double a = wave_soc_max_step(u + off, du + off, q, lane);
    if (lane == 0 && a < INFINITY) atomicMin(amin + 4 * (k / nsoc1), (unsigned long long)__double_as_longlong(a));
}

// -lambda_min = |u1| - u0 per big cone, max-reduced per block into partials[blockIdx.x]
__global__ void __launch_bounds__(256) lmin_big(int32_t nbig, const int32_t *__restrict__ big,
                                                const int32_t *__restrict__ soc_off, const double *__restrict__ u,
                                                double *__restrict__ partials) {
    const int32_t gw = big_wave();
    const int lane = threadIdx.x & 63;
    double v = -INFINITY;
    if (gw < nbig) {
        const int32_t k = big[gw];
        const int32_t off = soc_off[k], q = soc_off[k + 1] - off;
        double n1 = 0.0;
        for (int32_t a = 1 + lane; a < q; a += 64) n1 += u[off + a] * u[off + a];
        v = -(u[off] - sqrt(wave_sum(n1)));
    }
    __shared__ double sh[4];
    if (lane == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = nan_max(nan_max(sh[0], sh[1]), nan_max(sh[2], sh[3]));
}

static inline unsigned big_grid(qg_handle *h) { return (unsigned)((h->nbig + 3) / 4); }

static inline unsigned cone_grid(qg_handle *h) {
    const int64_t units = (int64_t)h->pp.l + h->pp.nsoc;
    return (unsigned)std::max<int64_t>(1, (units + 255) / 256);
}

// ---------------------------------------------------------------------------
// Lane groups: every second-order cone of the problem has the same q <= 16
// entries.  The orthant entries take one lane each in the first ceil(l / 64)
// wavefronts; then each cone takes G = 2^ceil(log2 q) consecutive lanes, lane
// e of its group holding entry e, so a wavefront's loads and stores are
// contiguous runs; a sum over a cone is a butterfly inside the group.  The
// formulas are those of the one-thread kernels (and of the wavefront-per-cone
// kernels, whose sums are butterflies too).  Measured on 1e5 cones of 4
// entries and 1e5 orthant entries: NT scaling with the (3,3) block 12.9 us
// against 20.7 us with one thread per cone.  (A lane-group line search took
// 25.3 us against 12.0 us: its blocks were 2.5 times as many, each with an
// atomic on the one minimum, and every lane repeats the divisions by the
// J-norm; the line search keeps one thread per cone.)
// ---------------------------------------------------------------------------
template <int G>
__device__ inline double grp_sum(double v) {
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <int G>
__global__ void __launch_bounds__(256) scaling_kernel_grp(int32_t l, int32_t nsoc, int32_t q,
                                                          const int64_t *__restrict__ blk_off,
                                                          const int64_t *__restrict__ blk33,
                                                          const double *__restrict__ s, const double *__restrict__ z,
                                                          double *__restrict__ w, double *__restrict__ wbar,
                                                          double *__restrict__ beta, double *__restrict__ lam,
                                                          double *__restrict__ kval) {
    const int64_t lpad = ((int64_t)l + 63) & ~(int64_t)63;
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < lpad) {                                   // whole wavefronts
        if (t < l) {
            const double si = s[t], zi = z[t];
            w[t] = sqrt(si / zi);
            if (lam) lam[t] = sqrt(si * zi);
            kval[blk33[t]] = -(si / zi);
        }
        return;
    }
    const int64_t tc = t - lpad, c = tc / G;
    const int e = (int)(tc % G);
    const int gb = (threadIdx.x & 63) & ~(G - 1);
    const bool cone = c < nsoc, live = cone && e < q;
    const int64_t off = l + c * q + e;
    const double sx = live ? s[off] : 0.0, zx = live ? z[off] : 0.0;
    const double s0 = __shfl(sx, gb), z0 = __shfl(zx, gb);
    const double ns1 = sqrt(grp_sum<G>(e >= 1 ? sx * sx : 0.0));
    const double nz1 = sqrt(grp_sum<G>(e >= 1 ? zx * zx : 0.0));
    const double sn = sqrt((s0 - ns1) * (s0 + ns1)), zn = sqrt((z0 - nz1) * (z0 + nz1));
    const double dot = grp_sum<G>(live ? (zx / zn) * (sx / sn) : 0.0);
    const double gamma = sqrt((1.0 + dot) * 0.5);
    const double zb = zx / zn, sb = sx / sn;
    const double wbv = (sb + (e == 0 ? zb : -zb)) / (2.0 * gamma);
    const double bt = sqrt(sn / zn);
    if (live) wbar[off - l] = wbv;
    if (cone && e == 0) beta[c] = bt;
    if (lam) {
        // lam = W z = bt (wb'z, z1 + wb1 (z0 + wb1'z1 / (1 + wb0)))
        const double w1u1 = grp_sum<G>(e >= 1 && live ? wbv * zx : 0.0);
        const double wb0 = __shfl(wbv, gb);
        const double coef = z0 + w1u1 / (1.0 + wb0);
        const double le = e == 0 ? bt * (wb0 * z0 + w1u1) : bt * (zx + wbv * coef);
        if (live) lam[off] = le;
    }
    // (3,3) block: -bt^2 (2 wb wb' - J), upper triangle, this lane's column e
    const double b2 = bt * bt;
    const int64_t base = cone ? l + blk_off[c] : 0;
#pragma unroll
    for (int ar = 0; ar < G; ++ar) {
        const double wa = __shfl(wbv, gb + ar);
        if (live && ar <= e) {
            const double jab = (ar == e) ? (ar == 0 ? 1.0 : -1.0) : 0.0;
            kval[blk33[base + (int64_t)e * (e + 1) / 2 + ar]] = -b2 * (2.0 * wa * wbv - jab);
        }
    }
}

static inline int grp_width(int32_t q) { return q <= 2 ? 2 : q <= 4 ? 4 : q <= 8 ? 8 : 16; }
static inline unsigned grp_grid(qg_handle *h, int G) {
    const int64_t lpad = ((int64_t)h->pp.l + 63) & ~(int64_t)63;
    return (unsigned)std::max<int64_t>(1, (lpad + (int64_t)h->pp.nsoc * G + 255) / 256);
}
static inline bool use_groups(qg_handle *h) { return h->grp_q > 0 && h->st.cone_lanes != 0 && h->ncopy == 1; }


int launch_scaling(qg_handle *h, const double *s, const double *z, double *lam, int block) {
    Device &d = h->d;
    if (block == 0 && use_groups(h)) {
        const int G = grp_width(h->grp_q);
        const unsigned g = grp_grid(h, G);
#define QG_SCALING_GRP(GG) scaling_kernel_grp<GG><<<g, 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, h->grp_q, \
        d.blk_off.p, d.blk33.p, s, z, d.w.p, d.wbar.p, d.beta.p, lam, d.kval.p)
        if (G == 2) QG_SCALING_GRP(2); else if (G == 4) QG_SCALING_GRP(4); else if (G == 8) QG_SCALING_GRP(8);
        else QG_SCALING_GRP(16);
#undef QG_SCALING_GRP
        QG_HIP(h, hipGetLastError());
        return QG_OK;
    }
    scaling_kernel<<<cone_grid(h), 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, d.blk_off.p,
                                                         d.blk33.p, s, z, d.w.p, d.wbar.p, d.beta.p, lam,
                                                         d.kval.p, block);
    QG_HIP(h, hipGetLastError());
    if (h->nbig) {
        scaling_big<<<big_grid(h), 256, 0, h->stream>>>(h->pp.l, h->nbig, d.big_cones.p, d.soc_off.p, s, z,
                                                         d.wbar.p, d.beta.p, lam, d.bigsc.p, block);
        QG_HIP(h, hipGetLastError());
        block_big<<<(unsigned)h->nbigchunk, 256, 0, h->stream>>>(h->pp.l, d.big_cones.p, d.big_chunk_cone.p,
                                                                  d.big_chunk_start.p, d.soc_off.p, d.blk_off.p,
                                                                  d.blk33.p, s, z, d.wbar.p, d.beta.p, d.bigsc.p,
                                                                  d.kval.p, block);
        QG_HIP(h, hipGetLastError());
    }
    return QG_OK;
}

int launch_cone_op(qg_handle *h, int op, const double *u, const double *v, double *out) {
    Device &d = h->d;
    cone_op_kernel<<<cone_grid(h), 256, 0, h->stream>>>(op, h->pp.l, h->pp.nsoc, d.soc_off.p, d.w.p, d.wbar.p,
                                                         d.beta.p, u, v, out);
    QG_HIP(h, hipGetLastError());
    if (h->nbig) {
        cone_op_big<<<big_grid(h), 256, 0, h->stream>>>(op, h->pp.l, h->nbig, d.big_cones.p, d.soc_off.p, d.wbar.p,
                                                         d.beta.p, u, v, out);
        QG_HIP(h, hipGetLastError());
    }
    return QG_OK;
}

int launch_ds_from_dz(qg_handle *h, const double *tvec, double tsign, const double *dz, double *ds) {
    Device &d = h->d;
    ds_kernel<<<cone_grid(h), 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, d.w.p, d.wbar.p, d.beta.p,
                                                    tvec, tsign, dz, ds);
    QG_HIP(h, hipGetLastError());
    if (h->nbig) {
        ds_big<<<big_grid(h), 256, 0, h->stream>>>(h->pp.l, h->nbig, d.big_cones.p, d.soc_off.p, d.wbar.p, d.beta.p,
                                                    tvec, tsign, dz, ds);
        QG_HIP(h, hipGetLastError());
    }
    return QG_OK;
}

int launch_corrector(qg_handle *h, const double *dsa, const double *dza, double sigma_mu,
                     const double *mu_dev, double *t) {
    Device &d = h->d;
    const int32_t kb = h->ncopy;
    corrector_kernel<<<cone_grid(h), 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, d.w.p, d.wbar.p,
                                                           d.beta.p, d.lam.p, dsa, dza, d.amin.p, mu_dev, sigma_mu,
                                                           t, d.alpha.p, h->pp.l / kb, h->pp.nsoc / kb, kb);
    QG_HIP(h, hipGetLastError());
    if (h->nbig) {
        corrector_big<<<big_grid(h), 256, 0, h->stream>>>(h->pp.l, h->nbig, d.big_cones.p, d.soc_off.p, d.wbar.p,
                                                           d.beta.p, d.lam.p, dsa, dza, d.amin.p, mu_dev, sigma_mu, t,
                                                           h->pp.nsoc / kb);
        QG_HIP(h, hipGetLastError());
    }
    return QG_OK;
}

// u <- u + (1 + a) e with a = -min_k lambda_min(u_k), when a >= 0
int launch_shift_interior(qg_handle *h, double *u) {
    Device &d = h->d;
    const unsigned g = cone_grid(h);
    const int32_t kb = h->ncopy;
    if (kb > 1) {
        // the amin slots serve as scratch here; the step kernels reset them before use
        init_keys_kernel<<<(kb + 255) / 256, 256, 0, h->stream>>>(d.amin.p, kb);
        lmin_inst_kernel<<<g, 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, u, d.amin.p, h->pp.l / kb,
                                                   h->pp.nsoc / kb, kb);
        add_e_inst_kernel<<<g, 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, d.amin.p, u, h->pp.l / kb,
                                                    h->pp.nsoc / kb, kb);
        QG_HIP(h, hipGetLastError());
        return QG_OK;
    }
    lmin_kernel<<<g, 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, u, d.partials.p);
    const unsigned gb = big_grid(h);
    if (gb) lmin_big<<<gb, 256, 0, h->stream>>>(h->nbig, d.big_cones.p, d.soc_off.p, u, d.partials.p + g);
    finish_max<<<1, 64, 0, h->stream>>>(d.partials.p, (int32_t)(g + gb), d.scal.p + NSCAL + 2);
    double a = 0.0;
    QG_HIP(h, hipMemcpyAsync(&a, d.scal.p + NSCAL + 2, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    QG_HIP(h, hipStreamSynchronize(h->stream));
    if (h->pp.l + h->pp.nsoc == 0 || a < 0.0) return QG_OK;
    add_e_kernel<<<g, 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, 1.0 + a, u);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int launch_identity_vec(qg_handle *h, double *u) {
    Device &d = h->d;
    int rc = launch_fill(h, h->m, 0.0, u);
    if (rc) return rc;
    add_e_kernel<<<cone_grid(h), 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, 1.0, u);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int launch_reset_steps(qg_handle *h) {
    const int32_t n = 4 * h->ncopy;
    reset_steps_kernel<<<(n + 255) / 256, 256, 0, h->stream>>>(h->d.amin.p, n);
    QG_HIP(h, hipGetLastError());
    return QG_OK;
}

int launch_step_min(qg_handle *h, const double *u, const double *du, int slot) {
    Device &d = h->d;
    const int32_t kb = h->ncopy;
    if (kb == 1)
        step_kernel_one<<<std::min(cone_grid(h), 1024u), 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, u,
                                                                               du, d.amin.p + slot);
    else
        step_kernel<<<cone_grid(h), 256, 0, h->stream>>>(h->pp.l, h->pp.nsoc, d.soc_off.p, u, du, d.amin.p + slot,
                                                          h->pp.l / kb, h->pp.nsoc / kb, kb);
    QG_HIP(h, hipGetLastError());
    if (h->nbig) {
        step_big<<<big_grid(h), 256, 0, h->stream>>>(h->nbig, d.big_cones.p, d.soc_off.p, u, du, d.amin.p + slot,
                                                      h->pp.nsoc / kb);
        QG_HIP(h, hipGetLastError());
    }
    return QG_OK;
}

int launch_max_step(qg_handle *h, const double *u, const double *du, int slot) {
    return launch_step_min(h, u, du, slot);
}

}  // namespace qg
