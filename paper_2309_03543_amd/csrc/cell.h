// Internal: per-cell and per-side formulas shared by the assembly, adjoint and
// correction-step kernels (device code).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/pmcorr.h"

namespace pm {

// The caller's data of cell o: Kfrak = chi exp(-s) G (K11, K12, K22) and
// Xi = eps dt S^{-1} with S = I + nu eps dt Kfrak, which is eps M^{-1} for
// M = I/dt + nu eps Kfrak.  Flags err and returns false for non-finite or
// invalid data (eps <= 0, chi < 0, G not positive definite).
__device__ __forceinline__ bool cell_xi(int o, const double* __restrict__ eps,
                                        const double* __restrict__ logk,
                                        const double* __restrict__ chi,
                                        const double* __restrict__ g11,
                                        const double* __restrict__ g12,
                                        const double* __restrict__ g22, double nu, double dt,
                                        double& e, double& K11, double& K12, double& K22,
                                        double& X11, double& X12, double& X22, int32_t* err) {
  e = eps[o];
  const double s = logk[o];
  const double ch = chi ? chi[o] : 1.0;
  const double a11 = g11 ? g11[o] : 1.0, a12 = g12 ? g12[o] : 0.0, a22 = g22 ? g22[o] : 1.0;
  const bool finite_in = isfinite(e) && isfinite(s) && isfinite(ch) && isfinite(a11) &&
                         isfinite(a12) && isfinite(a22);
  if (!finite_in) {
    atomicExch(err, PM_NONFINITE);
    return false;
  }
  if (!(e > 0.0) || ch < 0.0 || !(a11 * a22 - a12 * a12 > 0.0) || !(a11 > 0.0)) {
    atomicExch(err, PM_INVALID_ARG);
    return false;
  }
  const double k = ch * exp(-s);
  K11 = k * a11;
  K22 = k * a22;
  K12 = k * a12;
  const double c = nu * e * dt;
  const double S11 = 1.0 + c * K11, S12 = c * K12, S22 = 1.0 + c * K22;
  const double det = S11 * S22 - S12 * S12;
  const double f = e * dt / det;
  X11 = f * S22;
  X12 = -f * S12;
  X22 = f * S11;
  return true;
}

// n.A.n for the outward unit normal of the CCW side vector t.
__device__ __forceinline__ double normal_quadratic(double tx, double ty, double a11, double a12,
                                                   double a22) {
  return (ty * ty * a11 - 2.0 * tx * ty * a12 + tx * tx * a22) / (tx * tx + ty * ty);
}

}  // namespace pm
