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

// Factor the diagonal block [kb, kb+bs) (lower) and write it back; write its
// lower-triangular inverse to the tile's inverse block kb / 64.  The factor
// uses the unscaled update D[r][c] -= D[r][q] conj(D[c][q]) / D[q][q] (one
// barrier per column: column q is only read in step q) and scales the columns
// by 1/sqrt(pivot) at the end.  The inverse M = L^-1 is built one column per
// thread by forward substitution, stored transposed in the unused upper
// triangle of the same LDS block.
__global__ __launch_bounds__(256) void k_chol_potrf(ClassArgs a, CholArgs c) {
  const int t = blockIdx.x, tid = threadIdx.x;
  const int n = c.n, kb = c.kb, ld = a.nu_pad;
  const int bs = min(kCB, n - kb);
  c64 *G = a.at<c64>(t, a.lay.gram);
  __shared__ c64 D[kCB][kCB + 1];
  __shared__ double piv[kCB], mdiag[kCB];
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
  for (int q = 0; q < bs; ++q) {
    double d = D[q][q].x;
    if (!(d > 0.0)) d = 1e-300;  // flagged below
    const double inv = 1.0 / d;
    const int m = bs - q - 1;    // trailing block size
    for (int e = tid; e < m * m; e += 256) {
      const int r = q + 1 + e / m, cc = q + 1 + e % m;
      if (cc <= r) D[r][cc] = csub(D[r][cc], cscale(cmulc(D[r][q], D[cc][q]), inv));
    }
    __syncthreads();
  }
  if (tid < bs) {
    double d = D[tid][tid].x;
    if (!(d > 0.0)) {
      fail = 1;
      d = 1e-300;
    }
    piv[tid] = sqrt(d);
  }
  __syncthreads();
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int r = e / kCB, q = e % kCB;
    if (r < bs && q < r) D[r][q] = cscale(D[r][q], 1.0 / piv[q]);
  }
  if (tid < bs) D[tid][tid] = make_double2(piv[tid], 0.0);
  __syncthreads();
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int r = e / kCB, q = e % kCB;
    if (r < bs && q <= r) G[(int64_t)(kb + r) * ld + kb + q] = D[r][q];
  }
  // column q of M = L^-1 by thread q: M[i][q] = -(sum_{p=q}^{i-1} L[i][p] M[p][q]) / L[i][i],
  // kept at D[q][i] (upper triangle); M[q][q] = 1 / L[q][q].
  if (tid < bs) {
    const int q = tid;
    mdiag[q] = 1.0 / piv[q];
    for (int i = q + 1; i < bs; ++i) {
      c64 s = cscale(D[i][q], mdiag[q]);
      for (int p = q + 1; p < i; ++p) s = cadd(s, cmul(D[i][p], D[q][p]));
      D[q][i] = cscale(s, -1.0 / piv[i]);
    }
  }
  __syncthreads();
  c64 *linv = a.at<c64>(t, c.linv_off) + (int64_t)(kb / kCB) * kCB * kCB;
  for (int e = tid; e < kCB * kCB; e += 256) {
    const int r = e / kCB, q = e % kCB;
    c64 v = make_double2(0.0, 0.0);
    if (r < bs && q < r) v = D[q][r];
    else if (r < bs && q == r) v = make_double2(mdiag[r], 0.0);
    linv[e] = v;
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
  const c64 *linv = a.at<c64>(t, c.linv_off) + (int64_t)(kb / kCB) * kCB * kCB;
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

// L^H x = y with y = conj(row n), block by block from the last: four
// wavefronts form r = y_b - sum_{p beyond the block} conj(L[p][b]) x_p over
// strided rows, then x_b = M_b^H r with the stored inverse M_b of the block's
// diagonal factor.  Finally O_hat(u) = x(u) exp(-j phi_c(u + k_j)) on U.
__global__ __launch_bounds__(256) void k_chol_back(ClassArgs a, StepArgs s, int n,
                                                   int64_t linv_off) {
  const int t = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wq = tid >> 6;
  const int ld = a.nu_pad;
  const c64 *G = a.at<c64>(t, a.lay.gram);
  const c64 *linv = a.at<c64>(t, linv_off);
  c64 *x = a.at<c64>(t, a.lay.vec);
  __shared__ c64 part[4][64], rr[64];
  const int nblk = (n + 63) / 64;
  for (int b = nblk - 1; b >= 0; --b) {
    const int b0 = b * 64, b1 = min(n, b0 + 64), bs = b1 - b0;
    const int i = b0 + lane;
    c64 v = make_double2(0.0, 0.0);
    if (i < b1)
      for (int p = b1 + wq; p < n; p += 4) v = cadd(v, cmul(cconj(G[(int64_t)p * ld + i]), x[p]));
    part[wq][lane] = v;
    __syncthreads();
    if (wq == 0) {
      c64 r = make_double2(0.0, 0.0);
      if (lane < bs) {
        r = cconj(G[(int64_t)n * ld + i]);
        r = csub(r, cadd(cadd(part[0][lane], part[1][lane]), cadd(part[2][lane], part[3][lane])));
      }
      rr[lane] = r;
    }
    __syncthreads();
    if (wq == 0 && lane < bs) {
      const c64 *m = linv + (int64_t)b * 64 * 64;
      c64 xv = make_double2(0.0, 0.0);
      for (int q = lane; q < bs; ++q) xv = cadd(xv, cmul(cconj(m[q * 64 + lane]), rr[q]));
      x[i] = xv;
    }
    __syncthreads();
  }
  const float *co = a.at<float>(t, a.lay.coef);
  float cz[12];
#pragma unroll
  for (int j = 0; j < 12; ++j) cz[j] = co[j];
  for (int u = tid; u < n; u += 256) {
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
