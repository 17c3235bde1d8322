// Orthonormal Noll Zernike polynomials j = 4..15 at integer frequency (ky, kx)
// of a pupil of radius r (rho = |k| / r, theta = atan2(ky, kx)), evaluated in
// Cartesian form: with X = kx / r, Y = ky / r the harmonics rho^m cos(m theta)
// and rho^m sin(m theta) are the real and imaginary parts of (X + jY)^m.
#pragma once

#include "common.hpp"

namespace apic {

__device__ __forceinline__ void zernike12(float kx, float ky, float inv_r, float z[12]) {
  const float X = kx * inv_r, Y = ky * inv_r;
  const float r2 = X * X + Y * Y;
  const float c2 = X * X - Y * Y, s2 = 2.f * X * Y;
  const float c3 = X * c2 - Y * s2, s3 = X * s2 + Y * c2;
  const float c4 = X * c3 - Y * s3, s4 = X * s3 + Y * c3;
  const float k3 = 1.7320508075688772f, k5 = 2.2360679774997896f, k6 = 2.449489742783178f,
              k8 = 2.8284271247461903f, k10 = 3.1622776601683795f;
  z[0] = k3 * (2.f * r2 - 1.f);                          // Z4  (2, 0)
  z[1] = k6 * s2;                                        // Z5  (2,-2)
  z[2] = k6 * c2;                                        // Z6  (2, 2)
  z[3] = k8 * (3.f * r2 - 2.f) * Y;                      // Z7  (3,-1)
  z[4] = k8 * (3.f * r2 - 2.f) * X;                      // Z8  (3, 1)
  z[5] = k8 * s3;                                        // Z9  (3,-3)
  z[6] = k8 * c3;                                        // Z10 (3, 3)
  z[7] = k5 * (6.f * r2 * r2 - 6.f * r2 + 1.f);          // Z11 (4, 0)
  z[8] = k10 * (4.f * r2 - 3.f) * c2;                    // Z12 (4, 2)
  z[9] = k10 * (4.f * r2 - 3.f) * s2;                    // Z13 (4,-2)
  z[10] = k10 * c4;                                      // Z14 (4, 4)
  z[11] = k10 * s4;                                      // Z15 (4,-4)
}

// phi(k) = sum_{j=4..15} c_j Z_j(k) with c[0..11] = c_4..c_15.
__device__ __forceinline__ float pupil_phase12(const float *c, float kx, float ky, float inv_r) {
  float z[12];
  zernike12(kx, ky, inv_r, z);
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 12; ++j) s = fmaf(c[j], z[j], s);
  return s;
}

}  // namespace apic
