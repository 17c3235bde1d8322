// Brightfield half of the reconstruction (Fig. 2 upper part): image
// statistics, Kramers-Kronig recovery (Eq. 4-7), pupil normal equations and
// solve (Eq. 8-10), and correction + stitching (text after Eq. 10).
#pragma once

#include "fft.hpp"
#include "zern.hpp"

namespace apic {

// ---------------------------------------------------------------- statistics
// Mean of every NA-matched image -> log floor eps = log_floor_rel * mean(I);
// flags non-finite input and floor hits.
__global__ __launch_bounds__(256) void k_image_stats(ClassArgs a) {
  const int t = blockIdx.x / a.n_bf, i = blockIdx.x % a.n_bf;
  const float *img = a.image(t, i);
  const int nn = a.n * a.n;
  double s = 0.0;
  float mn = 3.0e38f;
  int bad = 0;
  for (int p = threadIdx.x; p < nn; p += 256) {
    const float v = img[p];
    if (!isfinite(v)) bad = 1;
    else {
      s += v;
      mn = fminf(mn, v);
    }
  }
  __shared__ double ss[256];
  __shared__ float sm[256];
  __shared__ int sb;
  if (threadIdx.x == 0) sb = 0;
  ss[threadIdx.x] = s;
  sm[threadIdx.x] = mn;
  __syncthreads();
  if (bad) atomicOr(&sb, 1);
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      ss[threadIdx.x] += ss[threadIdx.x + w];
      sm[threadIdx.x] = fminf(sm[threadIdx.x], sm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float eps = (float)(a.log_floor_rel * (ss[0] / nn));
    a.at<float>(t, a.lay.eps)[i] = eps;
    uint32_t bits = 0;
    if (sb) bits |= APIC_TILE_NONFINITE_INPUT;
    if (sm[0] < eps) bits |= APIC_TILE_LOG_FLOOR;
    if (bits) status_or(a, t, bits);
  }
}

// Background statistic of each tile (Sec. 3.2: patches whose low-resolution
// images barely vary are empty glass and are not reconstructed): the mean over
// the NA-matched images of var(I_i) / mean(I_i)^2, population variance over the
// N x N pixels, accumulated in FP64 around the image's first pixel.  One
// workgroup per tile streams its NA-matched images once with 16-byte loads.
constexpr int kBgThreads = 512;
__global__ __launch_bounds__(kBgThreads) void k_bg_stat(ClassArgs a, float *stat_out) {
  const int t = blockIdx.x;
  const int nn = a.n * a.n;
  __shared__ double red[2][kBgThreads / 64];
  double acc = 0.0;
  for (int i = 0; i < a.n_bf; ++i) {
    const float *img = a.image(t, i);
    const double x0 = img[0];
    const float4 *v4 = reinterpret_cast<const float4 *>(img);
    double s = 0.0, q = 0.0;
    for (int p = threadIdx.x; p < nn / 4; p += kBgThreads) {
      const float4 v = v4[p];
      const double d0 = v.x - x0, d1 = v.y - x0, d2 = v.z - x0, d3 = v.w - x0;
      s += (d0 + d1) + (d2 + d3);
      q += (d0 * d0 + d1 * d1) + (d2 * d2 + d3 * d3);
    }
    for (int o = 32; o > 0; o >>= 1) {
      s += __shfl_xor(s, o);
      q += __shfl_xor(q, o);
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = s;
      red[1][threadIdx.x >> 6] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double ts = 0.0, tq = 0.0;
      for (int w = 0; w < kBgThreads / 64; ++w) {
        ts += red[0][w];
        tq += red[1][w];
      }
      const double md = ts / nn, mean = x0 + md;
      acc += (tq / nn - md * md) / (mean * mean);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) stat_out[a.gidx(t)] = (float)(acc / a.n_bf);
}

// ---------------------------------------------------------------- KK passes
// Pass 1 (rows): L = log(max(I, eps)), row FFT.
template <int N> struct OpKK1 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  __device__ int rows() const { return N; }
  __device__ int row_of(int r) const { return r; }
  __device__ c32 load(int arr, int y, int x) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    const float v = a.image(t, i)[y * N + x];
    const float eps = a.at<float>(t, a.lay.eps)[i];
    return make_float2(logf(fmaxf(v, eps)), 0.f);
  }
  __device__ void mid(int, int, int, c32 &) const {}
  __device__ void store(int arr, int y, int x, c32 v) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    a.at<c32>(t, a.lay.stack)[((int64_t)i * N + y) * N + x] = v;
  }
};

// Pass 2 (columns): column FFT completes Lambda = fft2(L); multiply by Eq. 5's
// half-plane weights (1, 1/2, 0 by the sign of the integer k.k_i); column IFFT.
template <int N> struct OpKK2 {
  static constexpr bool INV1 = false, TWO = true, INV2 = true;
  ClassArgs a;
  __device__ c32 load(int arr, int y, int x) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    return a.at<c32>(t, a.lay.stack)[((int64_t)i * N + y) * N + x];
  }
  __device__ void mid(int arr, int y, int x, c32 &v) const {
    const int i = arr % a.n_bf;
    const int dot = signed_idx(x, N) * a.kx[i] + signed_idx(y, N) * a.ky[i];
    const float m = dot < 0 ? 1.f : (dot == 0 ? 0.5f : 0.f);
    v = cscale(v, m);
  }
  __device__ void store(int arr, int y, int x, c32 v) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    a.at<c32>(t, a.lay.stack)[((int64_t)i * N + y) * N + x] = v;
  }
};

// Pass 3 (rows): row IFFT completes ifft2(G) (times N^2); s = exp(. / N^2)
// (Eq. 6); row FFT.
template <int N> struct OpKK3 {
  static constexpr bool INV1 = true, TWO = true, INV2 = false;
  ClassArgs a;
  __device__ int rows() const { return N; }
  __device__ int row_of(int r) const { return r; }
  __device__ c32 load(int arr, int y, int x) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    return a.at<c32>(t, a.lay.stack)[((int64_t)i * N + y) * N + x];
  }
  __device__ void mid(int, int, int, c32 &v) const {
    constexpr float inv = 1.0f / (float(N) * float(N));
    const float mag = expf(v.x * inv);
    float sn, cs;
    sincosf(v.y * inv, &sn, &cs);
    v = make_float2(mag * cs, mag * sn);
  }
  __device__ void store(int arr, int y, int x, c32 v) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    a.at<c32>(t, a.lay.stack)[((int64_t)i * N + y) * N + x] = v;
  }
};

// Pass 4 (columns): column FFT completes fft2(s); keep the pupil support
// Circ(k + k_i) (Eq. 7) -> KK stack.  `out` (optional) receives a copy.
template <int N> struct OpKK4 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  c32 *out;  // [T][n_bf][N][N] or nullptr
  __device__ c32 load(int arr, int y, int x) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    return a.at<c32>(t, a.lay.stack)[((int64_t)i * N + y) * N + x];
  }
  __device__ void mid(int, int, int, c32 &) const {}
  __device__ void store(int arr, int y, int x, c32 v) const {
    const int t = arr / a.n_bf, i = arr % a.n_bf;
    const int ky = signed_idx(y, N), kx = signed_idx(x, N);
    if (!a.circ(ky + a.ky[i], kx + a.kx[i])) v = make_float2(0.f, 0.f);
    a.at<c32>(t, a.lay.stack)[((int64_t)i * N + y) * N + x] = v;
    if (out) out[(((int64_t)t * a.n_bf + i) * N + y) * N + x] = v;
  }
};

// ---------------------------------------------------------------- pupil solve
// Where a re-wrapped pupil pass takes its seed c0 (Noll 4..15) from: nowhere
// (plain pass), the caller's [T][15] array, the tile's seed block (the
// previous band of the coarse-to-fine continuation) or the tile's surrogate
// prediction.
enum SeedSrc : int { kSeedNone = 0, kSeedCaller = 1, kSeedBand = 2, kSeedSur = 3 };

__device__ __forceinline__ const float *seed_of(const ClassArgs &a, int t, const float *caller,
                                                int src) {
  if (src == kSeedCaller) return caller + (int64_t)a.gidx(t) * 15 + 3;
  if (src == kSeedBand) return a.at<float>(t, a.lay.seed);
  if (src == kSeedSur) return a.at<float>(t, a.lay.sur);
  return nullptr;
}

// One row of Eq. 10 per (pair, K): beta = arg(s_i conj(s_l)), w = |s_i s_l|,
// a_j = Z_j(K+k_i) - Z_j(K+k_l) - Z_j(k_i) + Z_j(k_l).  A workgroup takes a
// chunk of rows of one tile, stages (w a, a, beta, w, cell) of 256 rows in
// LDS, and 124 threads accumulate one normal-equation entry each in FP64:
// 78 entries of A's upper triangle, 12 of b, sum w beta^2, sum w, 32 cells.
// The rows are sorted by |K| band, so a pass over the first a.n_rows rows is
// a pass over the rows with |K| <= f r of one band of the continuation.
__global__ __launch_bounds__(256) void k_pupil_partial(ClassArgs a, const float *caller_seed,
                                                       int seed_src) {
  const int t = blockIdx.x / a.n_chunks, chunk = blockIdx.x % a.n_chunks;
  __shared__ float s_wa[256][13];
  __shared__ float s_a[256][13];
  __shared__ float s_beta[256], s_w[256];
  __shared__ int s_cell[256];
  const int tid = threadIdx.x;
  // entry owned by this thread: two threads per entry (ent = tid % 128), one
  // for each half of a batch of 256 rows, so all four wavefronts accumulate
  const int ent = tid & 127, half = tid >> 7;
  int p = 0, q = 0;
  if (ent < 78) {  // upper-triangle index -> (p, q), p <= q
    int rem = ent;
    p = 0;
    while (rem >= 12 - p) {
      rem -= 12 - p;
      ++p;
    }
    q = p + rem;
  }
  float c0[12];
  const float *seed = seed_of(a, t, caller_seed, seed_src);
  const bool seeded = seed != nullptr;
  if (seeded) {
#pragma unroll
    for (int j = 0; j < 12; ++j) c0[j] = seed[j];
  }
  const c32 *stack = a.at<c32>(t, a.lay.stack);
  const int nn = a.n * a.n;
  double acc = 0.0;
  const int row_end = min(a.n_rows, (chunk + 1) * kAbChunk);
  for (int rb = chunk * kAbChunk; rb < row_end; rb += 256) {
    const int row = rb + tid;
    float w = 0.f, beta = 0.f, av[12];
    int cell = -1;
#pragma unroll
    for (int j = 0; j < 12; ++j) av[j] = 0.f;
    if (row < row_end) {
      const uint32_t il = a.row_il[row], kw = a.row_k[row];
      const int i = il & 0xff, l = (il >> 8) & 0xff;
      cell = (int)(il >> 16);
      const int Ky = kunpack_y(kw), Kx = kunpack_x(kw);
      const int pos = fft_pos(Ky, a.n) * a.n + fft_pos(Kx, a.n);
      const c32 si = stack[(int64_t)i * nn + pos], sl = stack[(int64_t)l * nn + pos];
      const c32 z = cmulc(si, sl);
      beta = atan2f(z.y, z.x);
      w = hypotf(z.x, z.y);
      float zi[12], zl[12], zi0[12], zl0[12];
      zernike12((float)(Kx + a.kx[i]), (float)(Ky + a.ky[i]), a.inv_r, zi);
      zernike12((float)(Kx + a.kx[l]), (float)(Ky + a.ky[l]), a.inv_r, zl);
      zernike12((float)a.kx[i], (float)a.ky[i], a.inv_r, zi0);
      zernike12((float)a.kx[l], (float)a.ky[l], a.inv_r, zl0);
#pragma unroll
      for (int j = 0; j < 12; ++j) av[j] = (zi[j] - zi0[j]) - (zl[j] - zl0[j]);
      if (seeded) {
        float pred = 0.f;
#pragma unroll
        for (int j = 0; j < 12; ++j) pred = fmaf(av[j], c0[j], pred);
        const float d = beta - pred;
        beta = d - 6.283185307179586f * rintf(d * 0.15915494309189535f);
      }
    }
#pragma unroll
    for (int j = 0; j < 12; ++j) {
      s_wa[tid][j] = w * av[j];
      s_a[tid][j] = av[j];
    }
    s_beta[tid] = beta;
    s_w[tid] = w;
    s_cell[tid] = cell;
    __syncthreads();
    // rows [128 half, 128 half + 128) of the batch, four independent partial
    // sums (rows r .. r + 3) so the FP64 adds do not form one long chain
    double ac[4] = {0.0, 0.0, 0.0, 0.0};
    const int r0 = half * 128, r1 = r0 + 128;
    if (ent < 78) {
      for (int r = r0; r < r1; r += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) ac[u] += (double)(s_wa[r + u][p] * s_a[r + u][q]);
    } else if (ent < 90) {
      const int pp = ent - 78;
      for (int r = r0; r < r1; r += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) ac[u] += (double)(s_wa[r + u][pp] * s_beta[r + u]);
    } else if (ent == 90) {
      for (int r = r0; r < r1; r += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          ac[u] += (double)(s_w[r + u] * s_beta[r + u] * s_beta[r + u]);
    } else if (ent == 91) {
      for (int r = r0; r < r1; r += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) ac[u] += (double)s_w[r + u];
    } else if (ent < kAbEntries) {
      const int cc = ent - 92;
      for (int r = r0; r < r1; r += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) ac[u] += (s_cell[r + u] == cc) ? (double)s_w[r + u] : 0.0;
    }
    acc += (ac[0] + ac[1]) + (ac[2] + ac[3]);
    __syncthreads();
  }
  // the two halves of each entry, combined in a fixed order
  __shared__ double s_half[128];
  if (half == 1) s_half[ent] = acc;
  __syncthreads();
  if (half == 0 && ent < kAbEntries)
    a.at<double>(t, a.lay.part)[(int64_t)chunk * kAbEntries + ent] = acc + s_half[ent];
}

// Sum the chunk partials of each tile in a fixed order (deterministic).
__global__ __launch_bounds__(128) void k_pupil_reduce(ClassArgs a) {
  const int t = blockIdx.x, e = threadIdx.x;
  if (e >= kAbEntries) return;
  const double *part = a.at<double>(t, a.lay.part);
  double s = 0.0;
  for (int c = 0; c < a.n_chunks; ++c) s += part[(int64_t)c * kAbEntries + e];
  a.at<double>(t, a.lay.sums)[e] = s;
}

// Eigenvalues of a symmetric 12x12 matrix by cyclic Jacobi (kappa = max/min).
__device__ inline void jacobi_eig12(double m[12][12], double ev[12]) {
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < 12; ++i)
      for (int j = 0; j < 12; ++j) {
        tot += m[i][j] * m[i][j];
        if (i != j) off += m[i][j] * m[i][j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < 11; ++p)
      for (int q = p + 1; q < 12; ++q) {
        if (m[p][q] == 0.0) continue;
        const double th = (m[q][q] - m[p][p]) / (2.0 * m[p][q]);
        const double tt = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
        for (int k = 0; k < 12; ++k) {
          const double mkp = m[k][p], mkq = m[k][q];
          m[k][p] = c * mkp - s * mkq;
          m[k][q] = s * mkp + c * mkq;
        }
        for (int k = 0; k < 12; ++k) {
          const double mpk = m[p][k], mqk = m[q][k];
          m[p][k] = c * mpk - s * mqk;
          m[q][k] = s * mpk + c * mqk;
        }
      }
  }
  for (int i = 0; i < 12; ++i) ev[i] = m[i][i];
}

// One thread per tile: c_J = (A + mu tr(A)/12 I)^-1 b by FP64 Cholesky;
// diagnostics R(c) = (sum w beta^2 - 2 c.b + c.A.c)/sum w, kappa(A), sum w,
// smallest pivot; surrogate features log1p(cell / N^4).  With a seed the
// solution is the increment and c = c0 + x.  A band pass of the continuation
// (final = 0) writes c to the tile's seed block and nothing else; the final
// pass writes the coefficient block, outputs, diagnostics and status.
__global__ __launch_bounds__(64) void k_pupil_solve(ClassArgs a, const float *caller_seed,
                                                    int seed_src, int final_pass, float *zout,
                                                    float *diag, float *feat) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= a.T) return;
  const float *seed = seed_of(a, t, caller_seed, seed_src);
  const double *s = a.at<double>(t, a.lay.sums);
  double A[12][12], L[12][12], b[12], x[12];
  int e = 0;
  for (int p = 0; p < 12; ++p)
    for (int q = p; q < 12; ++q, ++e) A[p][q] = A[q][p] = s[e];
  for (int p = 0; p < 12; ++p) b[p] = s[78 + p];
  const double sbb = s[90], sw = s[91];
  double tr = 0.0;
  for (int p = 0; p < 12; ++p) tr += A[p][p];
  const double mu = a.ridge_pupil * tr / 12.0;
  double minpiv = 1e300;
  uint32_t bits = seed_src == kSeedCaller ? APIC_TILE_SEEDED : 0u;
  for (int j = 0; j < 12; ++j) {
    double d = A[j][j] + mu;
    for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
    minpiv = fmin(minpiv, d);
    if (!(d > 0.0)) {
      bits |= APIC_TILE_PUPIL_CHOL_FAIL;
      d = fmax(fabs(tr), 1e-300) * 1e-12;
    }
    L[j][j] = sqrt(d);
    for (int i = j + 1; i < 12; ++i) {
      double v = A[i][j];
      for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
      L[i][j] = v / L[j][j];
    }
  }
  for (int i = 0; i < 12; ++i) {
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[i][k] * x[k];
    x[i] = v / L[i][i];
  }
  for (int i = 11; i >= 0; --i) {
    double v = x[i];
    for (int k = i + 1; k < 12; ++k) v -= L[k][i] * x[k];
    x[i] = v / L[i][i];
  }
  if (!final_pass) {
    // the band's solution seeds the next band (read in full before writing:
    // the seed may be this same block)
    float nxt[12];
    for (int j = 0; j < 12; ++j) nxt[j] = (float)(x[j] + (seed ? (double)seed[j] : 0.0));
    float *sb = a.at<float>(t, a.lay.seed);
    for (int j = 0; j < 12; ++j) sb[j] = nxt[j];
    return;
  }
  double cb = 0.0, cac = 0.0;
  for (int p = 0; p < 12; ++p) {
    cb += x[p] * b[p];
    double r = 0.0;
    for (int q = 0; q < 12; ++q) r += A[p][q] * x[q];
    cac += x[p] * r;
  }
  const double resid = (sbb - 2.0 * cb + cac) / sw;
  double ev[12];
  jacobi_eig12(A, ev);
  double emax = ev[0], emin = ev[0];
  for (int i = 1; i < 12; ++i) {
    emax = fmax(emax, ev[i]);
    emin = fmin(emin, ev[i]);
  }
  const double kappa = emin > 0 ? emax / emin : 1e300;
  if (kappa > 1e6) bits |= APIC_TILE_PUPIL_ILLCOND;
  const int g = a.gidx(t);
  float *co = a.at<float>(t, a.lay.coef);
  for (int j = 0; j < 12; ++j) {
    double cj = x[j];
    if (seed) cj += (double)seed[j];
    if (!isfinite(cj)) bits |= APIC_TILE_NONFINITE_OUT;
    co[j] = (float)cj;
    if (zout) zout[(int64_t)g * 15 + 3 + j] = (float)cj;
  }
  co[14] = (float)fmin(kappa, 3.0e38);
  if (zout)
    for (int j = 0; j < 3; ++j) zout[(int64_t)g * 15 + j] = 0.f;
  if (diag) {
    diag[(int64_t)g * 4 + 0] = (float)resid;
    diag[(int64_t)g * 4 + 1] = (float)kappa;
    diag[(int64_t)g * 4 + 2] = (float)sw;
    diag[(int64_t)g * 4 + 3] = (float)minpiv;
  }
  if (feat) {
    const double n4 = (double)a.n * a.n * (double)a.n * a.n;
    for (int c = 0; c < kNumFeat; ++c) feat[(int64_t)g * kNumFeat + c] = (float)log1p(s[92 + c] / n4);
  }
  if (bits) status_or(a, t, bits);
}

// Copy caller-given coefficients into the tile's coefficient block.
__global__ __launch_bounds__(64) void k_coef_load(ClassArgs a, const float *zin) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= a.T) return;
  float *co = a.at<float>(t, a.lay.coef);
  for (int j = 0; j < 12; ++j) co[j] = zin[(int64_t)a.gidx(t) * 15 + 3 + j];
}

// phi_c(k_i) of every illumination vector (the constant offsets theta_i).
__global__ __launch_bounds__(64) void k_coef_led_phase(ClassArgs a) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= a.T) return;
  float *co = a.at<float>(t, a.lay.coef);
  float c[12];
  for (int j = 0; j < 12; ++j) c[j] = co[j];
  for (int i = 0; i < a.n_img; ++i)
    co[16 + i] = pupil_phase12(c, (float)a.kx[i], (float)a.ky[i], a.inv_r);
}

// ---------------------------------------------------------------- stitch
// O_hat(k) = mean over covering i of s_i(k) exp(-j[phi_c(k+k_i) - phi_c(k_i)]).
// The phasor exp(-j phi_c(q)) depends on the pupil point q = k + k_i only:
// k_pupil_phasor evaluates it once per point of the pupil disk, into the
// tile's ptil block (free until the darkfield stage, which overwrites it),
// and k_stitch gathers it for each covering image, times exp(j phi_c(k_i)).
__global__ __launch_bounds__(256) void k_pupil_phasor(ClassArgs a) {
  const int nn = a.n * a.n;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)a.T * nn) return;
  const int t = (int)(gid / nn), pix = (int)(gid % nn);
  const int qy = signed_idx(pix / a.n, a.n), qx = signed_idx(pix % a.n, a.n);
  if (!a.circ(qy, qx)) return;
  const float *co = a.at<float>(t, a.lay.coef);
  float c[12];
#pragma unroll
  for (int j = 0; j < 12; ++j) c[j] = co[j];
  float sn, cs;
  sincosf(pupil_phase12(c, (float)qx, (float)qy, a.inv_r), &sn, &cs);
  a.at<c32>(t, a.lay.ptil)[pix] = make_float2(cs, -sn);
}

__global__ __launch_bounds__(256) void k_stitch(ClassArgs a, float *spec_out) {
  const int nn = a.n * a.n;  // a multiple of 256: a workgroup stays in one tile
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int t = (int)min((int64_t)a.T - 1, ((int64_t)blockIdx.x * 256) / nn);
  __shared__ c32 led[kMaxBf];  // exp(j phi_c(k_i))
  if (threadIdx.x < a.n_bf) {
    float sn, cs;
    sincosf(a.at<float>(t, a.lay.coef)[16 + threadIdx.x], &sn, &cs);
    led[threadIdx.x] = make_float2(cs, sn);
  }
  __syncthreads();
  if (gid >= (int64_t)a.T * nn) return;
  const int pix = (int)(gid % nn);
  const int ky = signed_idx(pix / a.n, a.n), kx = signed_idx(pix % a.n, a.n);
  const c32 *stack = a.at<c32>(t, a.lay.stack);
  const c32 *tab = a.at<c32>(t, a.lay.ptil);
  // eight images at a time: their loads first (independent, in flight
  // together), then their sums
  constexpr int G = 8;
  float ax = 0.f, ay = 0.f;
  int cnt = 0;
  for (int i0 = 0; i0 < a.n_bf; i0 += G) {
    c32 v[G], e[G];
    bool in[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int i = i0 + g;
      v[g] = e[g] = make_float2(0.f, 0.f);
      in[g] = false;
      if (i < a.n_bf) {
        const int qy = ky + a.ky[i], qx = kx + a.kx[i];
        in[g] = a.circ(qy, qx);
        if (in[g]) {
          e[g] = tab[fft_pos(qy, a.n) * a.n + fft_pos(qx, a.n)];
          v[g] = stack[(int64_t)i * nn + pix];
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (!in[g]) continue;
      const c32 w = cmul(e[g], led[i0 + g]);
      ax += v[g].x * w.x - v[g].y * w.y;  // v * exp(-j [phi_c(q) - phi_c(k_i)])
      ay += v[g].x * w.y + v[g].y * w.x;
      ++cnt;
    }
  }
  const float inv = cnt ? 1.f / (float)cnt : 0.f;
  const c32 o = make_float2(ax * inv, ay * inv);
  a.at<c32>(t, a.lay.ohat)[pix] = o;
  if (spec_out) reinterpret_cast<c32 *>(spec_out)[a.out_off(t) + pix] = o;
}

}  // namespace apic
