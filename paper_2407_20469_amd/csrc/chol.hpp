// Batched FP64 Cholesky solve of the darkfield normal equations
//   (G + lambda tr(G)/n I) x = v,   one n x n Hermitian system per tile.
//
// The right-hand side rides along as row n of the (n+1)-row lower-triangular
// storage (row n holds conj(v)): factoring [[G, v], [v^H, *]] leaves
// conj(L^-1 v) in row n, so the forward substitution costs one extra row of
// the factorisation.  Right-looking with two levels of panels: the trailing
// matrix is updated once per kCW columns (each update streams the whole
// trailing triangle, so wider panels move fewer bytes), and inside a wide
// panel its 64-column sub-panels are factored one after another with
// launches over all tiles of the class:
//   k_chol_potrf  : factor the 64 x 64 diagonal block in registers and
//                   invert it in LDS (first panel: also add the ridge);
//   k_chol_trsm   : panel rows times the inverted block's conjugate transpose
//                   (64-row blocks, register-tiled like a GEMM);
//   k_chol_update : lower 64 x 64 tiles minus panel times panel^H (the rest
//                   of the wide panel's columns, then the trailing matrix).
// k_chol_back then solves L^H x = y with one wavefront per tile and scatters
// x into the tile's spectrum.
#pragma once

#include "common.hpp"
#include "zern.hpp"

namespace apic {

constexpr int kCB = 64;   // sub-panel width / tile size
constexpr int kCW = 128;  // wide-panel width (trailing update interval)
constexpr int kCK = 16;   // k-chunk staged in LDS

struct CholArgs {
  int n;            // system size
  int kb;           // panel start column (update: first column of its K range)
  int64_t linv_off; // per-tile byte offset of the 64 x 64 inverse block
  int kw;           // update: K width (columns kb .. kb + kw - 1)
  int c0;           // update: first output row and column
  int cend;         // update: output columns end here (exclusive)
};

// Output tiles of an update: row blocks from c0 through row n (the right-hand
// side row), column blocks from c0 up to cend, lower triangle only.
__host__ __device__ inline int upd_row_blocks(const CholArgs &c) {
  return (c.n + 1 - c.c0 + kCB - 1) / kCB;
}
__host__ __device__ inline int upd_col_blocks(const CholArgs &c) {
  return ((c.cend < c.n ? c.cend : c.n) - c.c0 + kCB - 1) / kCB;
}
__host__ __device__ inline int upd_tiles(const CholArgs &c) {
  const int nr = upd_row_blocks(c), nc = upd_col_blocks(c);
  return nc * nr - nc * (nc - 1) / 2;
}

// Factor the diagonal block [kb, kb+bs) (lower) and write it back; write its
// lower-triangular inverse to the tile's inverse block kb / 64.
//
// Factor: thread (r = tid / 4, s = tid % 4) keeps row r's columns s, s+4, ...
// in registers.  Step q publishes column q through LDS (double-buffered, one
// barrier per step) and every owner of a trailing element applies the
// unscaled update D[r][c] -= D[r][q] conj(D[c][q]) / D[q][q]; the columns are
// scaled by 1/sqrt(pivot) at the end, into a packed lower triangle in LDS.
// Inverse M = L^-1, column by column in parallel: four lanes per column q
// split the sum M[i][q] = -(sum_{q<=p<i} L[i][p] M[p][q]) / L[i][i] by
// p mod 4, each lane keeping the entries M[p][q] with p = its s mod 4 in
// registers (the only terms it needs), and combine it with lane shuffles.
// LDS holds only the packed factor (33 KB) and registers stay under 128 per
// lane, so four workgroups share a compute unit: a 1024-tile launch runs in
// one round.
constexpr int kTri = kCB * (kCB + 1) / 2;  // packed lower triangle, row i at i (i + 1) / 2
__global__ __launch_bounds__(256) void k_chol_potrf(ClassArgs a, CholArgs c) {
  const int t = blockIdx.x, tid = threadIdx.x;
  const int n = c.n, kb = c.kb, ld = a.nu_pad;
  const int bs = min(kCB, n - kb);
  c64 *G = a.at<c64>(t, a.lay.gram);
  __shared__ c64 Lp[kTri];
  __shared__ c64 col[2][kCB];
  __shared__ double piv[kCB], mdiag[kCB], pinv[2];
  __shared__ double red[256];
  __shared__ int fail;
  if (tid == 0) fail = 0;
  // the column buffers start at zero: the masked update reads entries that
  // no step has written (they are multiplied by 0, which needs them finite)
  for (int e = tid; e < 2 * kCB; e += 256) col[e / kCB][e % kCB] = make_double2(0.0, 0.0);
  __syncthreads();
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
  const int r = tid >> 2, s4 = tid & 3;
  c64 v[kCB / 4];
  const c64 *grow = G + (int64_t)(kb + min(r, bs - 1)) * ld + kb;
#pragma unroll
  for (int j = 0; j < kCB / 4; ++j) {
    const int cc = s4 + 4 * j;
    const c64 g = grow[min(cc, bs - 1)];
    v[j] = (r < bs && cc <= r) ? g : make_double2(0.0, 0.0);
  }
  for (int q = 0; q < bs; ++q) {
    c64 *cq = col[q & 1];
    if ((q & 3) == s4 && r >= q && r < bs) {
      // v[q / 4] with a wave-uniform index: a scalar branch, not a select chain
      c64 x;
      switch (q >> 2) {
#define APIC_POTRF_CASE(j) \
  case j:                  \
    x = v[j];              \
    break;
        APIC_POTRF_CASE(0) APIC_POTRF_CASE(1) APIC_POTRF_CASE(2) APIC_POTRF_CASE(3)
        APIC_POTRF_CASE(4) APIC_POTRF_CASE(5) APIC_POTRF_CASE(6) APIC_POTRF_CASE(7)
        APIC_POTRF_CASE(8) APIC_POTRF_CASE(9) APIC_POTRF_CASE(10) APIC_POTRF_CASE(11)
        APIC_POTRF_CASE(12) APIC_POTRF_CASE(13) APIC_POTRF_CASE(14)
        default:
          x = v[15];
#undef APIC_POTRF_CASE
      }
      cq[r] = x;
      if (r == q) {  // the pivot's reciprocal, once for everyone
        const double d = x.x;
        piv[q] = d;
        pinv[q & 1] = d > 0.0 ? 1.0 / d : 1e300;  // a failed pivot is flagged below
      }
    }
    __syncthreads();
    const double inv = pinv[q & 1];
    if (r > q && r < bs) {
      // v[j] -= m dr conj(col[c]) with m = 1 on the trailing part of the row
      // (q < c <= r) and 0 elsewhere (an exact no-op there: every operand is
      // finite), so no select keeps old and new values alive together; the
      // groups of four columns entirely at or left of q are skipped (q is
      // uniform, so the test is a scalar branch)
      const c64 dr = cscale(cq[r], inv);
#pragma unroll
      for (int j = 0; j < kCB / 4; ++j) {
        if (4 * j + 3 > q) {
          const int cc = s4 + 4 * j;
          const double msk = (cc > q && cc <= r) ? 1.0 : 0.0;
          const c64 cv = cq[cc];
          const double tx = fma(dr.x, cv.x, dr.y * cv.y), ty = fma(dr.y, cv.x, -dr.x * cv.y);
          v[j].x = fma(-msk, tx, v[j].x);
          v[j].y = fma(-msk, ty, v[j].y);
        }
      }
    }
  }
  __syncthreads();
  if (tid < bs) {
    double d = piv[tid];
    if (!(d > 0.0)) {
      fail = 1;
      d = 1e-300;
    }
    piv[tid] = sqrt(d);
    mdiag[tid] = 1.0 / piv[tid];
  }
  __syncthreads();
  // scaled factor to the packed triangle in LDS and back to the gram
  if (r < bs) {
#pragma unroll
    for (int j = 0; j < kCB / 4; ++j) {
      const int cc = s4 + 4 * j;
      if (cc < r) {
        const c64 l = cscale(v[j], mdiag[cc]);
        Lp[r * (r + 1) / 2 + cc] = l;
        G[(int64_t)(kb + r) * ld + kb + cc] = l;
      } else if (cc == r) {
        Lp[r * (r + 1) / 2 + r] = make_double2(piv[r], 0.0);
        G[(int64_t)(kb + r) * ld + kb + r] = make_double2(piv[r], 0.0);
      }
    }
  }
  __syncthreads();
  // inverse, column q = tid / 4 split over the four lanes s4 = tid % 4; lane
  // s4 keeps m[j] = M[4 j + s4][q] (zero above the diagonal, where p < q)
  const int q = r;
  c64 m[kCB / 4];
#pragma unroll
  for (int j = 0; j < kCB / 4; ++j)
    m[j] = (4 * j + s4 == q && q < bs) ? make_double2(mdiag[q], 0.0) : make_double2(0.0, 0.0);
  for (int i = 1; i < bs; ++i) {
    // terms p = 4 j + s4 < i (M[p][q] = 0 for p < q); the row's reads stay
    // inside the packed triangle (i (i + 1) / 2 + p <= kTri - 1)
    const c64 *Li = Lp + i * (i + 1) / 2;
    const int jend = (i + 3) >> 2;  // uniform
    c64 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < kCB / 4; ++j) {
      if (j < jend) {
        const int p = 4 * j + s4;
        const c64 tv = cmul(Li[p], m[j]);
        if (p < i) sum = cadd(sum, tv);
      }
      if ((j & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // loads four at a time
    }
    sum.x += __shfl_xor(sum.x, 1);
    sum.y += __shfl_xor(sum.y, 1);
    sum.x += __shfl_xor(sum.x, 2);
    sum.y += __shfl_xor(sum.y, 2);
    if (q < i && (i & 3) == s4) {
      const c64 mi = cscale(sum, -mdiag[i]);
      switch (i >> 2) {  // m[i / 4] with a wave-uniform index
#define APIC_INV_CASE(j) \
  case j:                \
    m[j] = mi;           \
    break;
        APIC_INV_CASE(0) APIC_INV_CASE(1) APIC_INV_CASE(2) APIC_INV_CASE(3)
        APIC_INV_CASE(4) APIC_INV_CASE(5) APIC_INV_CASE(6) APIC_INV_CASE(7)
        APIC_INV_CASE(8) APIC_INV_CASE(9) APIC_INV_CASE(10) APIC_INV_CASE(11)
        APIC_INV_CASE(12) APIC_INV_CASE(13) APIC_INV_CASE(14)
        default:
          m[15] = mi;
#undef APIC_INV_CASE
      }
    }
  }
  // linv[row][col] = M[row][col] (zero above the diagonal and outside bs)
  c64 *linv = a.at<c64>(t, c.linv_off) + (int64_t)(kb / kCB) * kCB * kCB;
#pragma unroll
  for (int j = 0; j < kCB / 4; ++j) {
    const int p = 4 * j + s4;
    linv[p * kCB + q] = (p < bs && q < bs) ? m[j] : make_double2(0.0, 0.0);
  }
  if (tid == 0 && fail) status_or(a, t, APIC_TILE_DF_CHOL_FAIL);
}

// 64 x 64 register-tiled complex FP64 product over a K range staged in LDS:
// acc[i][j] += sum_p A(row ty + 16 i, p) conj(B(row tx + 16 j, p)), with the
// operands given by loader callbacks.  16 x 16 threads, 4 x 4 outputs each,
// 16 apart, so that the lanes reading one LDS row read consecutive elements
// (no bank conflicts) and write consecutive columns.  The loaders run
// along p (kCK consecutive elements of a row per kCK lanes, one K chunk ahead
// in registers); the LDS rows are padded by one element so that the
// transposing store does not serialise on one bank group.
template <class LA, class LB>
__device__ __forceinline__ void tile_gemm_nc(c64 (&acc)[4][4], int K, LA la, LB lb,
                                             c64 (&sA)[kCK][kCB + 1], c64 (&sB)[kCK][kCB + 1]) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  // loader: element lk of rows lr + RS m (RS rows per pass, kCB / RS passes)
  constexpr int RS = 256 / kCK, NP = kCB / RS;
  static_assert(RS * kCK == 256 && NP * RS == kCB, "loader covers the tile exactly");
  const int lk = tid % kCK, lr = tid / kCK;
  c64 pa[NP], pb[NP];
  auto fetch = [&](int k0) {
    const bool ok = k0 + lk < K;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      pa[m] = ok ? la(lr + RS * m, k0 + lk) : make_double2(0.0, 0.0);
      pb[m] = ok ? lb(lr + RS * m, k0 + lk) : make_double2(0.0, 0.0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += kCK) {
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      sA[lk][lr + RS * m] = pa[m];
      sB[lk][lr + RS * m] = pb[m];
    }
    __syncthreads();
    if (k0 + kCK < K) fetch(k0 + kCK);
#pragma unroll 4
    for (int kk = 0; kk < kCK; ++kk) {
      c64 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tx + 16 * j];
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
  const int bid = xcd_remap(blockIdx.x, gridDim.x);
  const int t = bid / nrb, rb = bid % nrb;
  const int rbase = r0 + rb * kCB;
  c64 *G = a.at<c64>(t, a.lay.gram);
  const c64 *linv = a.at<c64>(t, c.linv_off) + (int64_t)(kb / kCB) * kCB * kCB;
  __shared__ c64 sA[kCK][kCB + 1], sB[kCK][kCB + 1];
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
    const int r = rbase + ty + 16 * i;
    if (r > n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = tx + 16 * j;
      if (q < bs) G[(int64_t)r * ld + kb + q] = acc[i][j];
    }
  }
}

// Update A[r][q] -= sum_{p in [kb, kb + kw)} L[r][p] conj(L[q][p]) of the lower
// tiles of rows [c0, n] x columns [c0, min(cend, n)): the trailing matrix
// after a wide panel, or the rest of the panel's own columns after one of its
// 64-column sub-panels.  Tiles are enumerated column block by column block.
__global__ __launch_bounds__(256) void k_chol_update(ClassArgs a, CholArgs c) {
  const int n = c.n, kb = c.kb, ld = a.nu_pad;
  const int nrb = upd_row_blocks(c);
  const int per_tile = upd_tiles(c);
  const int bid = xcd_remap(blockIdx.x, gridDim.x);  // a tile's blocks on one XCD
  const int t = bid / per_tile;
  int rem = bid % per_tile, J = 0;
  while (rem >= nrb - J) {
    rem -= nrb - J;
    ++J;
  }
  const int I = J + rem;
  const int ib = c.c0 + I * kCB, jb = c.c0 + J * kCB;
  const int qend = min(c.cend, n);
  c64 *G = a.at<c64>(t, a.lay.gram);
  __shared__ c64 sA[kCK][kCB + 1], sB[kCK][kCB + 1];
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
    return (r < qend) ? G[(int64_t)r * ld + kb + p] : make_double2(0.0, 0.0);
  };
  tile_gemm_nc(acc, c.kw, la, lb, sA, sB);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ib + ty + 16 * i;
    if (r > n) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = jb + tx + 16 * j;
      if (q < qend && q <= r) {
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
