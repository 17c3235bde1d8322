// Measurement probes for roofline reporting: a sustained FP64 FMA loop (eight
// independent chains per lane), the same on the FP64 matrix cores (16 x 16 x 4
// products, eight independent accumulators per wave) and a plain grid-stride
// 16-byte copy whose HBM traffic is known exactly (used to scale the
// FETCH_SIZE / WRITE_SIZE counters of the other kernels).
#pragma once

#include "common.hpp"

namespace apic {

__global__ __launch_bounds__(256) void k_calib_fma64(double *out, int iters, double a, double b) {
  double x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = threadIdx.x + k;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int r = 0; r < 16; ++r)
#pragma unroll
      for (int k = 0; k < 8; ++k) x[k] = fma(x[k], a, b);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

typedef double calib_d4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_calib_mfma64(double *out, int iters, double a, double b) {
  calib_d4 c[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) c[k] = calib_d4{0.0, 0.0, 0.0, (double)k};
  const double x = a + threadIdx.x, y = b - threadIdx.x;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c[k], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_calib_copy(const float4 *in, float4 *out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    out[i] = in[i];
}

}  // namespace apic
