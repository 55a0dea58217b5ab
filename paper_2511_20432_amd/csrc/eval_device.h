// Evaluation of the correction field T^ (Eq. 21) at parametric points given
// on the device: NURBS basis values and first derivatives per point
// (eval_device.hip), for the device-pointer variant of the temperature query.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sa {

// the patch's geometry on the device
struct GeoDev {
  const double *t[3];   // open knot vectors, n[d] + p[d] + 1 values
  int p[3], n[3];       // degree and control points per direction (p <= 6)
  const double *ctrl;   // [n2][n1][n0][4]: x, y, z, w
};

// At n parametric points xi [n][3]: x [n][3] = the physical point, Th [n] =
// sum_A R_A u_A and Gh [3][n] (component-major) = its physical gradient
// J^-T grad_xi.  A point outside [0,1]^3 gets NaN in x, Th and Gh.
void launch_eval_hat(hipStream_t st, int64_t n, const double *xi, const GeoDev &g, const double *u, double *x,
                     double *Th, double *Gh);

// T[i] = T0 + Th[i] + Tt[i]; gradT[3 i + c] = Gh[c n + i] + Gt[c n + i]
// (gradT may be NULL)
void launch_eval_combine(hipStream_t st, int64_t n, double T0, const double *Th, const double *Gh, const double *Tt,
                         const double *Gt, double *T, double *gradT);

}  // namespace sa
