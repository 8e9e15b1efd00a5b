// Device helpers shared by the type-1 translation units: input loads and the
// fold of a coordinate onto the torus as a fixed-point grid coordinate.
#pragma once
#include "fk_internal.h"

namespace fk {

// Fold a coordinate onto [-pi, pi) and convert to a fixed-point grid
// coordinate U = round((x + pi) / h * 2^fb).  Returns false (and sets flags)
// for NaN or |x| outside [-2 pi, 2 pi).
__device__ __forceinline__ bool to_fixed(double x, double scale, uint32_t nf_fix, uint32_t* U,
                                         int* flags) {
  if (!(x == x) || isinf(x)) {
    atomicOr(&flags[kFlagNaN], 1);
    return false;
  }
  const double two_pi = 6.283185307179586476925;
  if (x < -two_pi || x >= two_pi) {
    atomicOr(&flags[kFlagRange], 1);
    return false;
  }
  if (x < -3.14159265358979323846) x += two_pi;
  if (x >= 3.14159265358979323846) x -= two_pi;
  double u = (x + 3.14159265358979323846) * scale;   // in [0, nf * 2^fb]
  uint64_t v = (uint64_t)__double2ll_rn(u);
  if (v >= nf_fix) v -= nf_fix;                       // x == pi - tiny rounding up to nf
  *U = (uint32_t)v;
  return true;
}

__device__ __forceinline__ double load_coord(const void* X, fk_dtype dt, int64_t idx) {
  return dt == FK_F64 ? static_cast<const double*>(X)[idx] : (double)static_cast<const float*>(X)[idx];
}
__device__ __forceinline__ float load_weight(const void* Y, fk_dtype dt, int64_t idx) {
  return dt == FK_F64 ? (float)static_cast<const double*>(Y)[idx] : static_cast<const float*>(Y)[idx];
}

}  // namespace fk
