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

__host__ __device__ inline int pix_pad_f(int n) { return (n + 63) & ~63; }  // 256-byte runs of floats
__host__ __device__ inline int pix_pad_d(int n) { return (n + 31) & ~31; }  // of doubles

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

// phi of tile t (x over the pupil pixels) on the N x N grid in FFT order, zero
// outside the pupil, and its Zernike summary c = G^-1 Z^T phi (c_1..c_3
// reported as 0); iterations and the convergence status.  block_sum: a
// workgroup-wide sum (every thread of the workgroup calls this).
template <class BlockSum>
__device__ __forceinline__ void pix_finish(const ClassArgs &a, int t, const double *x, int it,
                                           bool conv, float *phi_out, float *zout,
                                           int32_t *iters_out, BlockSum &block_sum) {
  const int tid = threadIdx.x, np = a.n_pix;
  const uint32_t *pk = a.pix_tab;
  const int n = a.n, nn = n * n;
  const int gi = a.gidx(t);
  float *map = phi_out + (int64_t)gi * nn;
  for (int q = tid; q < nn; q += blockDim.x) {
    const int ky = signed_idx(q / n, n), kx = signed_idx(q % n, n);
    if (!a.circ(ky, kx)) map[q] = 0.f;
  }
  double h[15];
#pragma unroll
  for (int m = 0; m < 15; ++m) h[m] = 0.0;
  const double inv_r = 1.0 / a.r_d;
  for (int j = tid; j < np; j += blockDim.x) {
    const int ky = kunpack_y(pk[j]), kx = kunpack_x(pk[j]);
    const double v = x[j];
    map[fft_pos(ky, n) * n + fft_pos(kx, n)] = (float)v;
    double z[15];
    zernike15_d(kx * inv_r, ky * inv_r, z);
#pragma unroll
    for (int m = 0; m < 15; ++m) h[m] += z[m] * v;
  }
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
  const uint32_t *rab = a.pix_tab + np;
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

  pix_finish(a, t, x, it, conv, phi_out, zout, iters_out, block_sum);
}

// ---------------------------------------------------------------------------
// Beyond the LDS bound (512 px tiles): the same conjugate gradients with the
// four vectors in the tile's workspace.  Each iteration is two launches over
// the batch: k_pixg_apply spreads the row pass z = D^T W D p over many
// workgroups per tile (FP64 atomics into z, in L2), and k_pixg_step (one
// workgroup per tile) takes the CG step and clears z.  A tile that has
// converged (or hit max_iter) is marked done and skipped; the host polls the
// number of live tiles every few iterations.
//
// Workspace of a tile (the gram block): w and beta per row (float), then
// x, r, p, z (double, pix_pad_d(np) each), then PixState.
struct PixState {
  double gamma, stop;
  int it, done, conv, active;  // active: live tiles (tile 0's copy, for the host)
};
__host__ __device__ inline int64_t pixg_vec_off(int n_rows, int n_pix, int k) {
  return ((int64_t)pix_pad_f(n_rows) + (int64_t)k * pix_pad_d(n_pix)) * 8;
}
__device__ __forceinline__ double *pixg_vec(const ClassArgs &a, int t, int k) {
  return reinterpret_cast<double *>(a.tile(t) + a.lay.gram + pixg_vec_off(a.n_rows, a.n_pix, k));
}
__device__ __forceinline__ PixState *pixg_state(const ClassArgs &a, int t) {
  return reinterpret_cast<PixState *>(a.tile(t) + a.lay.gram + pixg_vec_off(a.n_rows, a.n_pix, 4));
}
constexpr int kPixgRowsPerWave = 4096;  // rows of a row pass per wavefront

// Workgroup-wide FP64 sum over kPixThreads threads (every thread calls it).
struct PixBlockSum {
  double *red, *bc;
  __device__ double operator()(double v) const {
    const int tid = threadIdx.x;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kPixThreads / 64; ++w) s += red[w];
      *bc = s;
    }
    __syncthreads();
    const double out = *bc;
    __syncthreads();
    return out;
  }
};

// z += D^T W beta (rhs) or z += D^T W D p over rows [beg, end) of the tile,
// wavefront by wavefront (the one-workgroup pass's pair grouping: a pair's
// two LED-pixel terms are summed in registers and flushed when it changes).
__global__ __launch_bounds__(256) void k_pixg_apply(ClassArgs a, int rhs, int wgs) {
  const int t = blockIdx.x / wgs, g = blockIdx.x % wgs;
  if (!rhs && pixg_state(a, t)->done) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int np = a.n_pix, nr = a.n_rows;
  const uint32_t *rab = a.pix_tab + np;
  __shared__ int sled[kMaxBf];
  if (tid < a.n_bf) sled[tid] = (int)a.pix_tab[np + nr + tid];
  __syncthreads();
  const float *wrow = a.at<float>(t, a.lay.gram);
  const float *brow = wrow + pix_pad_f(nr);
  const double *sp = pixg_vec(a, t, 2);
  double *sz = pixg_vec(a, t, 3);
  const int per = (nr + wgs * 4 - 1) / (wgs * 4);
  const int beg = (g * 4 + (tid >> 6)) * per, end = min(nr, beg + per);
  auto wave_sum = [&](double v) -> double {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
  };
  auto led_diff = [&](uint32_t il) { return sp[sled[il & 0xff]] - sp[sled[il >> 8]]; };
  uint32_t cur = 0xffffffffu;
  double dcur = 0.0, acc = 0.0;
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
          unsafeAtomicAdd(&sz[pa], y);
          unsafeAtomicAdd(&sz[pb], -y);
          acc += y;
        }
        continue;
      }
      double y = 0.0;
      if (live) {
        y = rhs ? (double)wv[u] * (double)bv[u]
                : (double)wv[u] * ((sp[pa] - sp[pb]) - led_diff(il[u]));
        unsafeAtomicAdd(&sz[pa], y);
        unsafeAtomicAdd(&sz[pb], -y);
      }
      if (cur != 0xffffffffu) {
        const double sum = wave_sum(acc);
        if (lane == 0) {
          unsafeAtomicAdd(&sz[sled[cur & 0xff]], -sum);
          unsafeAtomicAdd(&sz[sled[cur >> 8]], sum);
        }
      }
      const int last = min(63, end - 1 - (s0 + u * 64));
      cur = __shfl(il[u], last);
      dcur = rhs ? 0.0 : led_diff(cur);
      acc = 0.0;
      if (live && il[u] == cur) {
        acc = y;
      } else if (live) {
        unsafeAtomicAdd(&sz[sled[il[u] & 0xff]], -y);
        unsafeAtomicAdd(&sz[sled[il[u] >> 8]], y);
      }
    }
  }
  if (cur != 0xffffffffu) {
    const double sum = wave_sum(acc);
    if (lane == 0) {
      unsafeAtomicAdd(&sz[sled[cur & 0xff]], -sum);
      unsafeAtomicAdd(&sz[sled[cur >> 8]], sum);
    }
  }
}

// z = 0 before the right-hand side's row pass.
__global__ __launch_bounds__(256) void k_pixg_clear(ClassArgs a) {
  const int t = blockIdx.y;
  double *z = pixg_vec(a, t, 3);
  for (int j = blockIdx.x * 256 + threadIdx.x; j < a.n_pix; j += gridDim.x * 256) z[j] = 0.0;
}

// From z = D^T W beta: r = p = z, x = 0, z = 0, gamma = |r|^2, stop = tol^2 gamma.
__global__ __launch_bounds__(kPixThreads) void k_pixg_init(ClassArgs a, double tol) {
  __shared__ double red[kPixThreads / 64], bc;
  const PixBlockSum block_sum{red, &bc};
  const int t = blockIdx.x, tid = threadIdx.x, np = a.n_pix;
  double *x = pixg_vec(a, t, 0), *r = pixg_vec(a, t, 1), *p = pixg_vec(a, t, 2);
  double *z = pixg_vec(a, t, 3);
  double g = 0.0;
  for (int j = tid; j < np; j += kPixThreads) {
    const double v = z[j];
    r[j] = v;
    p[j] = v;
    x[j] = 0.0;
    z[j] = 0.0;
    g += v * v;
  }
  const double gamma = block_sum(g);
  if (tid == 0) {
    PixState *st = pixg_state(a, t);
    st->gamma = gamma;
    st->stop = tol * tol * gamma;
    st->it = 0;
    st->done = st->conv = !(gamma > 0.0);
  }
}

// One CG step from z = D^T W D p: x += alpha p, r -= alpha z, then either
// done (converged, max_iter, or a non-positive curvature) or p = r + beta p
// and z = 0 for the next row pass.
__global__ __launch_bounds__(kPixThreads) void k_pixg_step(ClassArgs a, int max_iter) {
  __shared__ double red[kPixThreads / 64], bc;
  const PixBlockSum block_sum{red, &bc};
  const int t = blockIdx.x, tid = threadIdx.x, np = a.n_pix;
  PixState *st = pixg_state(a, t);
  if (st->done) return;
  const double gamma = st->gamma, stop = st->stop;
  const int it = st->it + 1;
  double *x = pixg_vec(a, t, 0), *r = pixg_vec(a, t, 1), *p = pixg_vec(a, t, 2);
  double *z = pixg_vec(a, t, 3);
  double pz = 0.0;
  for (int j = tid; j < np; j += kPixThreads) pz += p[j] * z[j];
  pz = block_sum(pz);
  if (!(pz > 0.0)) {
    if (tid == 0) st->done = 1;
    return;
  }
  const double alpha = gamma / pz;
  double rr = 0.0;
  for (int j = tid; j < np; j += kPixThreads) {
    x[j] += alpha * p[j];
    const double rj = r[j] - alpha * z[j];
    r[j] = rj;
    rr += rj * rj;
  }
  rr = block_sum(rr);
  const bool conv = rr <= stop;
  const bool done = conv || it >= max_iter;
  if (!done) {
    const double beta = rr / gamma;
    for (int j = tid; j < np; j += kPixThreads) {
      p[j] = r[j] + beta * p[j];
      z[j] = 0.0;
    }
  }
  if (tid == 0) {
    st->it = it;
    st->gamma = rr;
    st->conv = conv;
    st->done = done;
  }
}

// Live tiles of the call, into tile 0's state (read by the host).
__global__ __launch_bounds__(256) void k_pixg_count(ClassArgs a) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int c = 0;
  for (int t = threadIdx.x; t < a.T; t += 256) c += pixg_state(a, t)->done ? 0 : 1;
  atomicAdd(&cnt, c);
  __syncthreads();
  if (threadIdx.x == 0) pixg_state(a, 0)->active = cnt;
}

// The result of each tile: phi map, Zernike summary, iterations, status.
__global__ __launch_bounds__(kPixThreads) void k_pixg_finish(ClassArgs a, float *phi_out,
                                                             float *zout, int32_t *iters_out) {
  __shared__ double red[kPixThreads / 64], bc;
  PixBlockSum block_sum{red, &bc};
  const int t = blockIdx.x;
  const PixState *st = pixg_state(a, t);
  const int it = st->it;
  const bool conv = st->conv != 0;
  pix_finish(a, t, pixg_vec(a, t, 0), it, conv, phi_out, zout, iters_out, block_sum);
}

}  // namespace apic
