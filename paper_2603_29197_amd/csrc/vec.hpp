// Launchers shared by the device phases of the Newton step.
#pragma once

#include "kernels.hpp"
#include "solver.hpp"

namespace qg {

// slots of the residual reduction (sums or max-abs)
enum : int {
    S_PX = 0, S_ATY, S_GTZ, S_RX, S_XPX, S_CX, S_C, S_AX, S_RY, S_BY, S_B, S_GX, S_RZ, S_HZ, S_SZ, S_S,
    S_H, NSCAL
};
constexpr uint32_t SCAL_MAXMASK = (1u << S_PX) | (1u << S_ATY) | (1u << S_GTZ) | (1u << S_RX) | (1u << S_C) |
                                  (1u << S_AX) | (1u << S_RY) | (1u << S_B) | (1u << S_GX) | (1u << S_RZ) |
                                  (1u << S_S) | (1u << S_H);

int launch_residual(qg_handle *h, const double *x, const double *y, const double *z, const double *s,
                    double *scal_host);
int launch_build_rhs(qg_handle *h, const double *zpart, double zsign, double *rhs);
int launch_axpy(qg_handle *h, int32_t len, double a, const double *xv, double *yv);
int launch_update(qg_handle *h, const double *dvec, const double *ds, double frac, double *alpha_dev);

int launch_fill(qg_handle *h, int32_t len, double v, double *out);
int launch_scale_copy(qg_handle *h, int32_t len, double a, const double *xv, double *out);

// cone phases
int launch_shift_interior(qg_handle *h, double *u);
int launch_identity_vec(qg_handle *h, double *u);
int launch_ds_from_dz(qg_handle *h, const double *tvec, double tsign, const double *dz, double *ds);
int launch_reset_steps(qg_handle *h);
int launch_step_min(qg_handle *h, const double *u, const double *du, int slot);

}  // namespace qg
