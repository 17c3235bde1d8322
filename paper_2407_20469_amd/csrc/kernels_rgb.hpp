// Colour image of a stained slide from three single-wavelength
// reconstructions (Sec. 3.3: amplitudes of the R, G and B fields combined and
// white balanced).  Both passes stream the three complex fields once.
#pragma once

#include "common.hpp"

namespace apic {

constexpr int kRgbBlocks = 1024;

// Per-workgroup FP64 partial sums of |F_c| over all pixels, c = R, G, B.
__global__ __launch_bounds__(256) void k_rgb_mean(const c32 *fr, const c32 *fg, const c32 *fb,
                                                  int64_t count, double *partial) {
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const c32 a = fr[i], b = fg[i], c = fb[i];
    s[0] += hypotf(a.x, a.y);
    s[1] += hypotf(b.x, b.y);
    s[2] += hypotf(c.x, c.y);
  }
  __shared__ double red[3][4];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    for (int o = 32; o > 0; o >>= 1) s[k] += __shfl_xor(s[k], o);
    if ((threadIdx.x & 63) == 0) red[k][threadIdx.x >> 6] = s[k];
  }
  __syncthreads();
  if (threadIdx.x < 3)
    partial[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0] + red[threadIdx.x][1] +
                                            red[threadIdx.x][2] + red[threadIdx.x][3];
}

// rgb[t][c][q] = g_c |F_c[t][q]| (planar per tile, plane = pixels per tile).
__global__ __launch_bounds__(256) void k_rgb_combine(const c32 *fr, const c32 *fg, const c32 *fb,
                                                     int64_t plane, int64_t count, float gr,
                                                     float gg, float gb, float *rgb) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const int64_t t = i / plane, q = i - t * plane;
    float *o = rgb + 3 * t * plane + q;
    const c32 a = fr[i], b = fg[i], c = fb[i];
    o[0] = gr * hypotf(a.x, a.y);
    o[plane] = gg * hypotf(b.x, b.y);
    o[2 * plane] = gb * hypotf(c.x, c.y);
  }
}

}  // namespace apic
