// Pupil-aberration solve of Eq. 10 with one unknown per pupil pixel (the
// paper's own formulation): phi on the integer pupil disk, rows
// phi(K+K_i) - phi(K+K_l) - phi(K_i) + phi(K_l) = beta with weight w, solved
// for the minimum-norm weighted least-squares phi by conjugate gradients on
// the normal equations D^T W D phi = D^T W beta.  From phi = 0 every iterate
// stays in the range of D^T (no piston, tip or tilt), so the iteration ends
// at the minimum-norm solution; it stops when the normal-equation residual
// falls under tol times its first value.
#pragma once

#include "common.hpp"

namespace apic {

constexpr int kPixThreads = 1024;
constexpr int kPixWaves = kPixThreads / 64;
constexpr int kPixUnroll = 4;   // 64-row blocks whose loads a wavefront issues together

__device__ __forceinline__ int pix_pad_f(int n) { return (n + 63) & ~63; }  // 256-byte runs of floats
__device__ __forceinline__ int pix_pad_d(int n) { return (n + 31) & ~31; }  // of doubles

// Phase difference and weight of every pupil row (as the Zernike-basis rows):
// beta = arg(s_i(K) conj(s_l(K))), w = |s_i(K) s_l(K)|, FP32 products.
__global__ __launch_bounds__(256) void k_pix_rows(ClassArgs a) {
  const int t = blockIdx.x / a.n_chunks, chunk = blockIdx.x % a.n_chunks;
  const c32 *stack = a.at<c32>(t, a.lay.stack);
  float *wrow = a.at<float>(t, a.lay.gram);
  float *brow = wrow + pix_pad_f(a.n_rows);
  const int nn = a.n * a.n;
  const int end = min(a.n_rows, (chunk + 1) * kAbChunk);
  for (int row = chunk * kAbChunk + threadIdx.x; row < end; row += 256) {
    const uint32_t il = a.row_il[row], kw = a.row_k[row];
    const int i = il & 0xff, l = (il >> 8) & 0xff;
    const int pos = fft_pos(kunpack_y(kw), a.n) * a.n + fft_pos(kunpack_x(kw), a.n);
    const c32 z = cmulc(stack[(int64_t)i * nn + pos], stack[(int64_t)l * nn + pos]);
    brow[row] = atan2f(z.y, z.x);
    wrow[row] = hypotf(z.x, z.y);
  }
}

// Orthonormal Noll Z_1..Z_15 at (X, Y) = k / r (double).
__device__ __forceinline__ void zernike15_d(double X, double Y, double z[15]) {
  const double r2 = X * X + Y * Y;
  const double c2 = X * X - Y * Y, s2 = 2.0 * X * Y;
  const double c3 = X * c2 - Y * s2, s3 = X * s2 + Y * c2;
  const double c4 = X * c3 - Y * s3, s4 = X * s3 + Y * c3;
  const double k3 = 1.7320508075688772, k5 = 2.23606797749979, k6 = 2.449489742783178,
               k8 = 2.8284271247461903, k10 = 3.1622776601683795;
  z[0] = 1.0;
  z[1] = 2.0 * X;
  z[2] = 2.0 * Y;
  z[3] = k3 * (2.0 * r2 - 1.0);
  z[4] = k6 * s2;
  z[5] = k6 * c2;
  z[6] = k8 * (3.0 * r2 - 2.0) * Y;
  z[7] = k8 * (3.0 * r2 - 2.0) * X;
  z[8] = k8 * s3;
  z[9] = k8 * c3;
  z[10] = k5 * (6.0 * r2 * r2 - 6.0 * r2 + 1.0);
  z[11] = k10 * (4.0 * r2 - 3.0) * c2;
  z[12] = k10 * (4.0 * r2 - 3.0) * s2;
  z[13] = k10 * c4;
  z[14] = k10 * s4;
}

// One workgroup per tile.  The search direction and the operator's image
// live in LDS (two doubles per pixel); the iterate and the residual in the
// tile's workspace, each pixel owned by one thread.  The rows' pixel pairs and
// LED pixels come from the plan; per-row w and beta from k_pix_rows.
__global__ __launch_bounds__(kPixThreads) void k_pix_cg(ClassArgs a, double tol, int max_iter,
                                                        float *phi_out, float *zout,
                                                        int32_t *iters_out) {
  __shared__ double sp[kPixMax], sz[kPixMax];
  __shared__ double red[kPixThreads / 64];
  __shared__ double bc;
  __shared__ int sled[kMaxBf];
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
  const int np = a.n_pix, nr = a.n_rows;
  const uint32_t *pk = a.pix_tab, *rab = a.pix_tab + np;
  if (tid < a.n_bf) sled[tid] = (int)a.pix_tab[np + nr + tid];  // LED pixels
  const float *wrow = a.at<float>(t, a.lay.gram);
  const float *brow = wrow + pix_pad_f(nr);
  // the iterate and the residual follow the two float arrays of pix_pad_f(nr)
  // elements each, i.e. pix_pad_f(nr) doubles into the region
  double *x = reinterpret_cast<double *>(a.tile(t) + a.lay.gram) + pix_pad_f(nr);
  double *r = x + pix_pad_d(np);

  auto block_sum = [&](double v) -> double {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (lane == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kPixThreads / 64; ++w) s += red[w];
      bc = s;
    }
    __syncthreads();
    const double out = bc;
    __syncthreads();
    return out;
  };

  // sz = D^T W beta (rhs) or sz = D^T W D sp.  Wavefront v walks rows
  // [v * per, (v + 1) * per) 64 at a time (coalesced), issuing kPixUnroll
  // blocks' loads before their LDS work.  Rows are grouped by pair, so the
  // pair's two LED-pixel terms are summed in registers while the pair lasts
  // and flushed (one wavefront sum, two atomics) when it changes.
  auto wave_sum = [&](double v) -> double {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  };
  auto row_pass = [&](bool rhs) {
    for (int j = tid; j < np; j += kPixThreads) sz[j] = 0.0;
    __syncthreads();
    const int per = (nr + kPixWaves - 1) / kPixWaves;
    const int beg = (tid >> 6) * per, end = min(nr, beg + per);
    uint32_t cur = 0xffffffffu;  // pair being summed (wavefront-uniform)
    double dcur = 0.0;           // sp[LED i] - sp[LED l] of that pair
    double acc = 0.0;
    for (int s0 = beg; s0 < end; s0 += 64 * kPixUnroll) {
      uint32_t il[kPixUnroll], ab[kPixUnroll];
      float wv[kPixUnroll], bv[kPixUnroll];
#pragma unroll
      for (int u = 0; u < kPixUnroll; ++u) {
        const int row = s0 + u * 64 + lane;
        il[u] = 0xffffffffu;
        ab[u] = 0u;
        wv[u] = 0.f;
        bv[u] = 0.f;
        if (row < end) {
          il[u] = a.row_il[row] & 0xffffu;
          ab[u] = rab[row];
          wv[u] = wrow[row];
          if (rhs) bv[u] = brow[row];
        }
      }
#pragma unroll
      for (int u = 0; u < kPixUnroll; ++u) {
        if (s0 + u * 64 >= end) break;  // wavefront-uniform
        const bool live = il[u] != 0xffffffffu;
        const int pa = ab[u] & 0xffff, pb = ab[u] >> 16;
        if (__all(!live || il[u] == cur)) {
          if (live) {
            const double y = rhs ? (double)wv[u] * (double)bv[u]
                                 : (double)wv[u] * ((sp[pa] - sp[pb]) - dcur);
            atomicAdd(&sz[pa], y);
            atomicAdd(&sz[pb], -y);
            acc += y;
          }
          continue;
        }
        // the pair changes inside this block: flush the running sum, then
        // continue with the pair of the block's last live row
        double y = 0.0;
        if (live) {
          y = rhs ? (double)wv[u] * (double)bv[u]
                  : (double)wv[u] * ((sp[pa] - sp[pb]) - (sp[sled[il[u] & 0xff]] - sp[sled[il[u] >> 8]]));
          atomicAdd(&sz[pa], y);
          atomicAdd(&sz[pb], -y);
        }
        if (cur != 0xffffffffu) {
          const double sum = wave_sum(acc);
          if (lane == 0) {
            atomicAdd(&sz[sled[cur & 0xff]], -sum);
            atomicAdd(&sz[sled[cur >> 8]], sum);
          }
        }
        const int last = min(63, end - 1 - (s0 + u * 64));
        cur = __shfl(il[u], last);
        dcur = rhs ? 0.0 : sp[sled[cur & 0xff]] - sp[sled[cur >> 8]];
        acc = 0.0;
        if (live && il[u] == cur) {
          acc = y;
        } else if (live) {
          atomicAdd(&sz[sled[il[u] & 0xff]], -y);
          atomicAdd(&sz[sled[il[u] >> 8]], y);
        }
      }
    }
    if (cur != 0xffffffffu) {
      const double sum = wave_sum(acc);
      if (lane == 0) {
        atomicAdd(&sz[sled[cur & 0xff]], -sum);
        atomicAdd(&sz[sled[cur >> 8]], sum);
      }
    }
    __syncthreads();
  };

  row_pass(true);
  double g = 0.0;
  for (int j = tid; j < np; j += kPixThreads) {
    const double v = sz[j];
    r[j] = v;
    x[j] = 0.0;
    sp[j] = v;
    g += v * v;
  }
  double gamma = block_sum(g);
  const double stop = tol * tol * gamma;
  bool conv = !(gamma > 0.0);
  int it = 0;
  while (!conv && it < max_iter) {
    row_pass(false);
    double pz = 0.0;
    for (int j = tid; j < np; j += kPixThreads) pz += sp[j] * sz[j];
    pz = block_sum(pz);
    if (!(pz > 0.0)) break;
    const double alpha = gamma / pz;
    double rr = 0.0;
    for (int j = tid; j < np; j += kPixThreads) {
      x[j] += alpha * sp[j];
      const double rj = r[j] - alpha * sz[j];
      r[j] = rj;
      rr += rj * rj;
    }
    rr = block_sum(rr);
    ++it;
    if (rr <= stop) {
      conv = true;
      break;
    }
    const double beta = rr / gamma;
    gamma = rr;
    for (int j = tid; j < np; j += kPixThreads) sp[j] = r[j] + beta * sp[j];
    __syncthreads();
  }

  // phi on the N x N grid in FFT order, zero outside the pupil
  const int n = a.n, nn = n * n;
  const int gi = a.gidx(t);
  float *map = phi_out + (int64_t)gi * nn;
  for (int q = tid; q < nn; q += kPixThreads) {
    const int ky = signed_idx(q / n, n), kx = signed_idx(q % n, n);
    if (!a.circ(ky, kx)) map[q] = 0.f;
  }
  double h[15];
#pragma unroll
  for (int m = 0; m < 15; ++m) h[m] = 0.0;
  const double inv_r = 1.0 / a.r_d;
  for (int j = tid; j < np; j += kPixThreads) {
    const int ky = kunpack_y(pk[j]), kx = kunpack_x(pk[j]);
    const double v = x[j];
    map[fft_pos(ky, n) * n + fft_pos(kx, n)] = (float)v;
    double z[15];
    zernike15_d(kx * inv_r, ky * inv_r, z);
#pragma unroll
    for (int m = 0; m < 15; ++m) h[m] += z[m] * v;
  }
  // Zernike summary c = G^-1 Z^T phi (c_1..c_3 reported as 0)
  __shared__ double hs[15];
  for (int m = 0; m < 15; ++m) {
    const double v = block_sum(h[m]);
    if (tid == 0) hs[m] = v;
  }
  __syncthreads();
  if (tid < 15) {
    double c = 0.0;
    for (int m = 0; m < 15; ++m) c += a.pix_ginv[tid * 15 + m] * hs[m];
    zout[(int64_t)gi * 15 + tid] = tid < 3 ? 0.f : (float)c;
  }
  if (tid == 0) {
    if (iters_out) iters_out[gi] = it;
    if (!conv) status_or(a, t, APIC_TILE_PIXEL_NOT_CONVERGED);
  }
}

}  // namespace apic
