// sabr_adjoint.hpp -- launch interface of the polish kernels: the adjoint and
// Levenberg-Marquardt kernels (sabr_adjoint.hip) and the Nelder-Mead kernel
// (sabr_nm.hip).  Not part of the public ABI.
#pragma once
#include "sabr_internal.hpp"

namespace sabr {

// Waves of the GLOBAL4 adjoint / LM grid (one wave per point, grid-stride).
constexpr int kAdjointMaxWaves = 2048;

int adjoint_waves(int n_pts);
size_t adjoint_lds_bytes(const DevMarket &m);
// Largest LDS allocation of one workgroup on the current device (bytes).
int lds_budget_bytes();

hipError_t launch_vjp(const DevMarket &m, int n_pts, const int *pt_inst, const double *params,
                      const double *g_cost, double *cost, double *g_params, double *jtwj,
                      double *jtwr, hipStream_t s);

hipError_t launch_lm(const DevMarket &m, int n_pts, const int *pt_inst, double *params,
                     const double *lb, const double *ub, int max_iter, double mu0, double tol,
                     double *cost_out, int *iters_out, hipStream_t s);

// Nelder-Mead: one wave per point, the simplex in LDS.
size_t nm_lds_bytes(const DevMarket &m);
hipError_t launch_nm(const DevMarket &m, int n_pts, const int *pt_inst, double *params,
                     const double *lb, const double *ub, int max_iter, double step, double tol,
                     double *cost_out, int *iters_out, hipStream_t s);

}  // namespace sabr
