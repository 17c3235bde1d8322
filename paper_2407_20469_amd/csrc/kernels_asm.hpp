// Patch assembly at known positions (Sec. 2.5: overlapping regions of
// adjacent tiles are blended to hide the seams).  Two HBM-bound passes over
// the tiles' complex fields: the overlap correlation of every overlapping
// pair (for the constant-phase alignment), and a gather blend in which each
// 32 x 32 block of the canvas reads the tiles that cover it and writes its
// pixels once.
#pragma once

#include "common.hpp"

namespace apic {

constexpr int kAsmBlock = 32;

// One overlapping pair: tiles t, u and the overlap [y0, y1) x [x0, x1) in
// canvas pixels.
struct AsmPair {
  int32_t t, u, y0, y1, x0, x1;
};

// C_tu = sum over the overlap of F_t conj(F_u), FP64 accumulation; one
// workgroup per pair.
__global__ __launch_bounds__(256) void k_overlap_corr(const c32 *fields, int n,
                                                      const int32_t *pos, const AsmPair *pairs,
                                                      c64 *out) {
  const AsmPair p = pairs[blockIdx.x];
  const c32 *ft = fields + (int64_t)p.t * n * n;
  const c32 *fu = fields + (int64_t)p.u * n * n;
  const int ty = pos[2 * p.t], tx = pos[2 * p.t + 1], uy = pos[2 * p.u], ux = pos[2 * p.u + 1];
  const int w = p.x1 - p.x0, cnt = (p.y1 - p.y0) * w;
  double sr = 0.0, si = 0.0;
  for (int q = threadIdx.x; q < cnt; q += 256) {
    const int y = p.y0 + q / w, x = p.x0 + q % w;
    const c32 a = ft[(y - ty) * n + (x - tx)], b = fu[(y - uy) * n + (x - ux)];
    sr += (double)a.x * b.x + (double)a.y * b.y;
    si += (double)a.y * b.x - (double)a.x * b.y;
  }
  __shared__ double rr[2][4];
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    si += __shfl_xor(si, o);
  }
  if ((threadIdx.x & 63) == 0) {
    rr[0][threadIdx.x >> 6] = sr;
    rr[1][threadIdx.x >> 6] = si;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    out[blockIdx.x] = make_double2(rr[0][0] + rr[0][1] + rr[0][2] + rr[0][3],
                                   rr[1][0] + rr[1][1] + rr[1][2] + rr[1][3]);
}

__device__ __forceinline__ float asm_ramp(int v, int n, float inv_w) {
  const float c = v + 0.5f;
  return fminf(1.f, fminf(c * inv_w, (n - c) * inv_w));
}

// canvas(p) = sum_t w_t(p) F_t(p) exp(-j theta_t) / sum_t w_t(p), 0 where no
// tile covers p.  Block b of the canvas (row-major, kAsmBlock square) lists
// its covering tiles in tiles[start[b] .. start[b + 1]); theta [T] (device,
// NULL = all 0).  The block's tile offsets and phase factors are staged in LDS
// once; each pixel is written once.
constexpr int kAsmMaxCover = 64;  // tiles staged per pass over a block's list
__global__ __launch_bounds__(256) void k_blend(const c32 *fields, int n, const int32_t *pos,
                                               const int32_t *start, const int32_t *tiles,
                                               const float *theta, float inv_w, c32 *canvas, int H,
                                               int W, int bw) {
  __shared__ int s_t[kAsmMaxCover], s_y[kAsmMaxCover], s_x[kAsmMaxCover];
  __shared__ c32 s_rot[kAsmMaxCover];
  const int b = blockIdx.x;
  const int by = (b / bw) * kAsmBlock, bx = (b % bw) * kAsmBlock;
  const int lx = threadIdx.x & 31, ly0 = threadIdx.x >> 5;  // 8 rows per pass
  const int x = bx + lx;
  const int k0 = start[b], k1 = start[b + 1];
  float ar[kAsmBlock / 8], ai[kAsmBlock / 8], den[kAsmBlock / 8];
#pragma unroll
  for (int i = 0; i < kAsmBlock / 8; ++i) ar[i] = ai[i] = den[i] = 0.f;
  for (int c0 = k0; c0 < k1; c0 += kAsmMaxCover) {
    const int cn = min(kAsmMaxCover, k1 - c0);
    __syncthreads();
    if (threadIdx.x < cn) {
      const int t = tiles[c0 + threadIdx.x];
      s_t[threadIdx.x] = t;
      s_y[threadIdx.x] = pos[2 * t];
      s_x[threadIdx.x] = pos[2 * t + 1];
      float sn = 0.f, cs = 1.f;
      if (theta) sincosf(theta[t], &sn, &cs);
      s_rot[threadIdx.x] = make_float2(cs, -sn);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kAsmBlock / 8; ++i) {
      const int y = by + ly0 + 8 * i;
      for (int k = 0; k < cn; ++k) {
        const int ty = y - s_y[k], tx = x - s_x[k];
        if (ty < 0 || ty >= n || tx < 0 || tx >= n) continue;
        const float w = asm_ramp(ty, n, inv_w) * asm_ramp(tx, n, inv_w);
        const c32 f = cmul(fields[(int64_t)s_t[k] * n * n + ty * n + tx], s_rot[k]);
        ar[i] = fmaf(w, f.x, ar[i]);
        ai[i] = fmaf(w, f.y, ai[i]);
        den[i] += w;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < kAsmBlock / 8; ++i) {
    const int y = by + ly0 + 8 * i;
    if (y < H && x < W)
      canvas[(int64_t)y * W + x] =
          den[i] > 0.f ? make_float2(ar[i] / den[i], ai[i] / den[i]) : make_float2(0.f, 0.f);
  }
}

}  // namespace apic
