// Batched FP64 Cholesky solve of the darkfield normal equations
//   (G + lambda tr(G)/n I) x = v,   one n x n Hermitian system per tile.
//
// The right-hand side rides along as row n of the (n+1)-row lower-triangular
// storage (row n holds conj(v)): factoring [[G, v], [v^H, *]] leaves
// conj(L^-1 v) in row n, so the forward substitution costs one extra row of
// the factorisation.  Right-looking, 64-wide panels; per panel three launches
// over all tiles of the class:
//   k_chol_potrf  : factor the 64 x 64 diagonal block in LDS and invert it
//                   (first panel: also add the ridge to the diagonal);
//   k_chol_trsm   : panel rows times the inverted block's conjugate transpose
//                   (64-row blocks, register-tiled like a GEMM);
//   k_chol_update : trailing lower 64 x 64 tiles minus panel times panel^H.
// k_chol_back then solves L^H x = y with one wavefront per tile and scatters
// x into the tile's spectrum.
#pragma once

#include "common.hpp"
#include "zern.hpp"

namespace apic {

constexpr int kCB = 64;   // panel width / tile size
constexpr int kCK = 16;   // k-chunk staged in LDS

struct CholArgs {
  int n;            // system size
  int kb;           // panel start column
  int64_t linv_off; // per-tile byte offset of the 64 x 64 inverse block
};

// Factor the diagonal block [kb, kb+bs) in place (lower), write it back, and
// write its lower-triangular inverse to the tile's inverse block.
__global__ __launch_bounds__(256) void k_chol_potrf(ClassArgs a, CholArgs c) {
  const int t = blockIdx.x, tid = threadIdx.x;
  const int n = c.n, kb = c.kb, ld = a.nu_pad;
  const int bs = min(kCB, n - kb);
  c64 *G = a.at<c64>(t, a.lay.gram);
  __shared__ c64 D[kCB][kCB + 1];
  __shared__ c64 tmp[kCB];
  __shared__ double red[256];
  __shared__ int fail;
  if (tid == 0) fail = 0;
  if (kb == 0) {
    double tr = 0.0;
    for (int i = tid; i < n; i += 256) tr += G[(int64_t)i * ld + i].x;
    red[tid] = tr;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    const double ridge = a.ridge_df * red[0] / n;
    for (int i = tid; i < n; i += 256) G[(int64_t)i * ld + i].x += ridge;
    __syncthreads();
  }
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int r = e / kCB, q = e % kCB;
    D[r][q] = (r < bs && q <= r) ? G[(int64_t)(kb + r) * ld + kb + q] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  const double tiny = 1e-300;
  for (int q = 0; q < bs; ++q) {
    if (tid == 0) {
      double d = D[q][q].x;
      if (!(d > 0.0)) {
        fail = 1;
        d = fmax(fabs(d), tiny);
      }
      D[q][q] = make_double2(sqrt(d), 0.0);
    }
    __syncthreads();
    if (tid > q && tid < bs) D[tid][q] = cscale(D[tid][q], 1.0 / D[q][q].x);
    __syncthreads();
    for (int e = tid; e < bs * bs; e += 256) {
      const int r = e / bs, cc = e % bs;
      if (cc > q && r >= cc) D[r][cc] = csub(D[r][cc], cmulc(D[r][q], D[cc][q]));
    }
    __syncthreads();
  }
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int r = e / kCB, q = e % kCB;
    if (r < bs && q <= r) G[(int64_t)(kb + r) * ld + kb + q] = D[r][q];
  }
  // in-place inverse of the lower-triangular block, last column first
  for (int j = bs - 1; j >= 0; --j) {
    if (tid < bs) tmp[tid] = D[tid][j];
    __syncthreads();
    const double djj = 1.0 / tmp[j].x;
    if (tid > j && tid < bs) {
      c64 s = make_double2(0.0, 0.0);
      for (int p = j + 1; p <= tid; ++p) s = cadd(s, cmul(D[tid][p], tmp[p]));
      D[tid][j] = cscale(s, -djj);
    }
    if (tid == j) D[j][j] = make_double2(djj, 0.0);
    __syncthreads();
  }
  c64 *linv = a.at<c64>(t, c.linv_off);
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int r = e / kCB, q = e % kCB;
    linv[e] = (r < bs && q <= r) ? D[r][q] : make_double2(0.0, 0.0);
  }
  if (tid == 0 && fail) status_or(a, t, APIC_TILE_DF_CHOL_FAIL);
}

// 64 x 64 register-tiled complex FP64 product over a K range staged in LDS:
// acc[i][j] += sum_p A(row i, p) conj(B(row j, p)), with the operands given by
// loader callbacks.  16 x 16 threads, 4 x 4 outputs each.
template <class LA, class LB>
__device__ __forceinline__ void tile_gemm_nc(c64 (&acc)[4][4], int K, LA la, LB lb,
                                             c64 (&sA)[kCK][kCB], c64 (&sB)[kCK][kCB]) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  for (int k0 = 0; k0 < K; k0 += kCK) {
#pragma unroll
    for (int m = 0; m < (kCK * kCB) / 256; ++m) {
      const int e = tid + m * 256;
      const int kk = e / kCB, rr = e % kCB;
      const bool ok = k0 + kk < K;
      sA[kk][rr] = ok ? la(rr, k0 + kk) : make_double2(0.0, 0.0);
      sB[kk][rr] = ok ? lb(rr, k0 + kk) : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kCK; ++kk) {
      c64 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].x = fma(av[i].x, bv[j].x, fma(av[i].y, bv[j].y, acc[i][j].x));
          acc[i][j].y = fma(av[i].y, bv[j].x, fma(-av[i].x, bv[j].y, acc[i][j].y));
        }
    }
    __syncthreads();
  }
}

// Panel rows [kb+bs, n] (row n = right-hand side): X = A_panel Linv^H.
__global__ __launch_bounds__(256) void k_chol_trsm(ClassArgs a, CholArgs c) {
  const int n = c.n, kb = c.kb, ld = a.nu_pad;
  const int bs = min(kCB, n - kb);
  const int r0 = kb + bs;
  const int nrb = (n + 1 - r0 + kCB - 1) / kCB;
  const int t = blockIdx.x / nrb, rb = blockIdx.x % nrb;
  const int rbase = r0 + rb * kCB;
  c64 *G = a.at<c64>(t, a.lay.gram);
  const c64 *linv = a.at<c64>(t, c.linv_off);
  __shared__ c64 sA[kCK][kCB], sB[kCK][kCB];
  c64 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  auto la = [&](int rr, int p) {
    const int r = rbase + rr;
    return (r <= n) ? G[(int64_t)r * ld + kb + p] : make_double2(0.0, 0.0);
  };
  auto lb = [&](int q, int p) { return linv[q * kCB + p]; };
  tile_gemm_nc(acc, bs, la, lb, sA, sB);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = rbase + ty * 4 + i;
    if (r > n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tx * 4 + j;
      if (q < bs) G[(int64_t)r * ld + kb + q] = acc[i][j];
    }
  }
}

// Trailing update of the lower tiles of rows [kb+bs, n] x cols [kb+bs, n).
__global__ __launch_bounds__(256) void k_chol_update(ClassArgs a, CholArgs c) {
  const int n = c.n, kb = c.kb, ld = a.nu_pad;
  const int bs = min(kCB, n - kb);
  const int c0 = kb + bs;
  const int nrb = (n + 1 - c0 + kCB - 1) / kCB;
  const int ntri = nrb * (nrb + 1) / 2;
  const int t = blockIdx.x / ntri;
  int rem = blockIdx.x % ntri, I = 0;
  while (rem > I) {
    rem -= I + 1;
    ++I;
  }
  const int J = rem;
  const int ib = c0 + I * kCB, jb = c0 + J * kCB;
  if (jb >= n) return;
  c64 *G = a.at<c64>(t, a.lay.gram);
  __shared__ c64 sA[kCK][kCB], sB[kCK][kCB];
  c64 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  auto la = [&](int rr, int p) {
    const int r = ib + rr;
    return (r <= n) ? G[(int64_t)r * ld + kb + p] : make_double2(0.0, 0.0);
  };
  auto lb = [&](int rr, int p) {
    const int r = jb + rr;
    return (r < n) ? G[(int64_t)r * ld + kb + p] : make_double2(0.0, 0.0);
  };
  tile_gemm_nc(acc, bs, la, lb, sA, sB);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ib + ty * 4 + i;
    if (r > n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = jb + tx * 4 + j;
      if (q < n && q <= r) {
        c64 *gp = G + (int64_t)r * ld + q;
        *gp = csub(*gp, acc[i][j]);
      }
    }
  }
}

// L^H x = y with y = conj(row n), one wavefront per tile; then
// O_hat(u) = x(u) exp(-j phi_c(u + k_j)) on U.
__global__ __launch_bounds__(64) void k_chol_back(ClassArgs a, StepArgs s, int n) {
  const int t = blockIdx.x, lane = threadIdx.x, ld = a.nu_pad;
  const c64 *G = a.at<c64>(t, a.lay.gram);
  c64 *x = a.at<c64>(t, a.lay.vec);
  __shared__ c64 acc[64], xs[64];
  const int nblk = (n + 63) / 64;
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * 64, b1 = min(n, b0 + 64);
    const int i = b0 + lane;
    c64 v = make_double2(0.0, 0.0);
    if (i < b1) {
      v = cconj(G[(int64_t)n * ld + i]);
      for (int p = b1; p < n; ++p) v = csub(v, cmul(cconj(G[(int64_t)p * ld + i]), x[p]));
    }
    acc[lane] = v;
    __syncthreads();
    for (int q = b1 - 1; q >= b0; --q) {
      if (lane == q - b0) xs[lane] = cscale(acc[lane], 1.0 / G[(int64_t)q * ld + q].x);
      __syncthreads();
      if (lane < q - b0) acc[lane] = csub(acc[lane], cmul(cconj(G[(int64_t)q * ld + b0 + lane]),
                                                          xs[q - b0]));
      __syncthreads();
    }
    if (i < b1) x[i] = xs[lane];
    __syncthreads();
  }
  const float *co = a.at<float>(t, a.lay.coef);
  float cz[12];
#pragma unroll
  for (int j = 0; j < 12; ++j) cz[j] = co[j];
  for (int u = lane; u < n; u += 64) {
    const uint32_t w = s.u[u];
    const int ky = kunpack_y(w), kx = kunpack_x(w);
    const float ph = pupil_phase12(cz, (float)(kx + s.kx), (float)(ky + s.ky), a.inv_r);
    float sn, cs;
    sincosf(ph, &sn, &cs);
    const c64 xv = x[u];
    const int pos = fft_pos(ky, a.n) * a.n + fft_pos(kx, a.n);
    a.at<c32>(t, a.lay.ohat)[pos] =
        make_float2((float)(xv.x * cs + xv.y * sn), (float)(xv.y * cs - xv.x * sn));
  }
}

}  // namespace apic
