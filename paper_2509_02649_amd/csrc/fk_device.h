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

// Bin coordinate of a point on one axis for the matrix-core spread.  The window of
// a point at grid coordinate u (U = u 2^fb) covers the w cells from i0 = ceil(u - w/2);
// its bin is (i0 mod nf) / 2^tshift, so the windows of a bin's points all start in the
// bin's 2^tshift cells.  wbias = 2^fb - 1 + 8 2^fb - w 2^(fb-1), computed on the host
// (the 8 cells of bias keep the 32-bit sum positive); nf is a power of two.
__device__ __forceinline__ int window_bin(uint32_t U, int fb, uint32_t wbias, int nf, int tshift) {
  const int i0 = (int)((U + wbias) >> fb) - 8;
  return (i0 & (nf - 1)) >> tshift;
}

__device__ __forceinline__ double load_coord(const void* X, fk_dtype dt, int64_t idx) {
  return dt == FK_F64 ? static_cast<const double*>(X)[idx] : (double)static_cast<const float*>(X)[idx];
}
__device__ __forceinline__ float load_weight(const void* Y, fk_dtype dt, int64_t idx) {
  return dt == FK_F64 ? (float)static_cast<const double*>(Y)[idx] : static_cast<const float*>(Y)[idx];
}

}  // namespace fk
