// Learned Zernike surrogate: a 34 -> 128 -> 128 -> 12 ReLU perceptron from
// (tile x, tile y, 32 spectral-overlap features) to c_4..c_15, with bfloat16
// operands on the matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulate),
// FP32 master weights and Adam.  Not part of the paper's method: it seeds or
// replaces the pupil solve on tiles where the closed form is weak, and the
// closed form stays its fallback and the arbiter of its error (residual
// rule below).
//
// MFMA 16x16x16 operand layout (wave64): lane l holds A[l % 16][4 (l / 16) + q]
// and B[4 (l / 16) + q][l % 16] for q = 0..3, and receives
// D[4 (l / 16) + q][l % 16].
#pragma once

#include "common.hpp"

namespace apic {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 34, kMlpInPad = 64, kMlpHid = 128, kMlpOut = 12, kMlpOutPad = 16;
constexpr int kMlpTile = 64;  // samples per tile
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHid * kMlpInPad;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpOutPad * kMlpHid;
constexpr int kMlpParams = kOffB3 + kMlpOutPad;

// float -> bfloat16, round to nearest, ties to even (NaN kept quiet).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// Workgroup GEMM over bfloat16 operands in LDS:
//   C(i, j) = sum_k A(i, k) B(k, j),  A(i, k) = A[i sai + k sak], B(k, j) = B[k sbk + j sbj]
// M, N, K multiples of 16; 16 x 16 output tiles round-robin over the 4 waves;
// st(i, j, value) receives every output once.
template <class Store>
__device__ __forceinline__ void wg_gemm(int M, int N, int K, const uint16_t *A, int sai, int sak,
                                        const uint16_t *B, int sbk, int sbj, Store st) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 15, kq = (lane >> 4) * 4;
  const int nt = N / 16, tiles = (M / 16) * nt;
  for (int tile = wave; tile < tiles; tile += 4) {
    const int i0 = (tile / nt) * 16, j0 = (tile % nt) * 16;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x4_t av, bv;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        av[q] = (short)A[(i0 + r) * sai + (k0 + kq + q) * sak];
        bv[q] = (short)B[(k0 + kq + q) * sbk + (j0 + r) * sbj];
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) st(i0 + kq + q, j0 + r, acc[q]);
  }
}

// Library utility (layout check): C[M][N] = A[M][K] B[K][N], bfloat16 row-major
// inputs, FP32 output, M, N, K <= 64 and multiples of 16, one workgroup.
__global__ __launch_bounds__(256) void k_bf16_gemm(int M, int N, int K, const uint16_t *A,
                                                   const uint16_t *B, float *C) {
  __shared__ uint16_t sa[64 * 64], sb[64 * 64];
  for (int e = threadIdx.x; e < M * K; e += 256) sa[e] = A[e];
  for (int e = threadIdx.x; e < K * N; e += 256) sb[e] = B[e];
  __syncthreads();
  wg_gemm(M, N, K, sa, K, 1, sb, N, 1, [&](int i, int j, float v) { C[i * N + j] = v; });
}

// Weights and biases of the model in LDS (bfloat16 weights, FP32 biases).
struct MlpLds {
  uint16_t w1[kMlpHid * kMlpInPad];
  uint16_t w2[kMlpHid * kMlpHid];
  uint16_t w3[kMlpOutPad * kMlpHid];
  float b1[kMlpHid], b2[kMlpHid], b3[kMlpOutPad];
};

__device__ __forceinline__ void mlp_load_weights(MlpLds &w, const float *theta) {
  for (int e = threadIdx.x; e < kMlpHid * kMlpInPad; e += 256) w.w1[e] = f2bf(theta[kOffW1 + e]);
  for (int e = threadIdx.x; e < kMlpHid * kMlpHid; e += 256) w.w2[e] = f2bf(theta[kOffW2 + e]);
  for (int e = threadIdx.x; e < kMlpOutPad * kMlpHid; e += 256) w.w3[e] = f2bf(theta[kOffW3 + e]);
  for (int e = threadIdx.x; e < kMlpHid; e += 256) {
    w.b1[e] = theta[kOffB1 + e];
    w.b2[e] = theta[kOffB2 + e];
  }
  if (threadIdx.x < kMlpOutPad) w.b3[threadIdx.x] = theta[kOffB3 + threadIdx.x];
}

// Forward pass of one 64-sample tile held in sx (bfloat16, 64 x 64):
// h1, h2 (bfloat16 64 x 128), y (FP32 64 x 16).
__device__ __forceinline__ void mlp_forward_tile(const MlpLds &w, const uint16_t *sx, uint16_t *h1,
                                                 uint16_t *h2, float *y) {
  wg_gemm(kMlpTile, kMlpHid, kMlpInPad, sx, kMlpInPad, 1, w.w1, 1, kMlpInPad,
          [&](int i, int j, float v) { h1[i * kMlpHid + j] = f2bf(fmaxf(v + w.b1[j], 0.f)); });
  __syncthreads();
  wg_gemm(kMlpTile, kMlpHid, kMlpHid, h1, kMlpHid, 1, w.w2, 1, kMlpHid,
          [&](int i, int j, float v) { h2[i * kMlpHid + j] = f2bf(fmaxf(v + w.b2[j], 0.f)); });
  __syncthreads();
  wg_gemm(kMlpTile, kMlpOutPad, kMlpHid, h2, kMlpHid, 1, w.w3, 1, kMlpHid,
          [&](int i, int j, float v) { y[i * kMlpOutPad + j] = v + w.b3[j]; });
  __syncthreads();
}

// Normalised, bfloat16 input row: (x - mean) / std over 34 values, 0 beyond.
__device__ __forceinline__ void mlp_load_inputs(uint16_t *sx, int n, const int *rows,
                                                const float *inputs, const float *mean,
                                                const float *stdv) {
  for (int e = threadIdx.x; e < kMlpTile * kMlpInPad; e += 256) {
    const int i = e / kMlpInPad, c = e % kMlpInPad;
    float v = 0.f;
    if (rows[i] >= 0 && c < kMlpIn) v = (inputs[(int64_t)rows[i] * kMlpIn + c] - mean[c]) / stdv[c];
    sx[e] = f2bf(v);
  }
}

struct MlpTrainArgs {
  float *theta, *m, *v, *grad;         // kMlpParams each (device)
  const float *inputs, *targets;       // [n][34], [n][12]
  const float *mean, *stdv;            // [34]
  const int32_t *order;                // [steps * batch] sample indices (-1 = none)
  int n, steps, batch, t0;             // t0: Adam steps already taken
  float lr, beta1, beta2, eps;
  float *loss_out;                     // [steps]
  int grad_only;                       // 1: one gradient pass over order[0..batch), no update
};

// Training in one workgroup: for every step, forward + backward over the
// step's samples in 64-sample tiles (weight gradients accumulated in FP32 in
// `grad`), then an Adam update of the FP32 master weights and a refresh of
// the bfloat16 working copy.
__global__ __launch_bounds__(256) void k_mlp_train(MlpTrainArgs a) {
  __shared__ MlpLds w;
  __shared__ uint16_t sx[kMlpTile * kMlpInPad];
  __shared__ uint16_t h1[kMlpTile * kMlpHid], h2[kMlpTile * kMlpHid];
  __shared__ float y[kMlpTile * kMlpOutPad];
  __shared__ uint16_t dy[kMlpTile * kMlpOutPad];
  __shared__ int rows[kMlpTile];
  __shared__ float red[256];
  const int tid = threadIdx.x;
  mlp_load_weights(w, a.theta);
  __syncthreads();
  for (int step = 0; step < a.steps; ++step) {
    for (int e = tid; e < kMlpParams; e += 256) a.grad[e] = 0.f;
    int valid = 0;
    for (int i = 0; i < a.batch; ++i) valid += a.order[(int64_t)step * a.batch + i] >= 0;
    const float scale = 2.f / (float)(max(valid, 1) * kMlpOut);
    float lsum = 0.f;
    __syncthreads();
    for (int t0 = 0; t0 < a.batch; t0 += kMlpTile) {
      if (tid < kMlpTile) {
        const int idx = t0 + tid;
        rows[tid] = idx < a.batch ? a.order[(int64_t)step * a.batch + idx] : -1;
      }
      __syncthreads();
      mlp_load_inputs(sx, a.n, rows, a.inputs, a.mean, a.stdv);
      __syncthreads();
      mlp_forward_tile(w, sx, h1, h2, y);
      for (int e = tid; e < kMlpTile * kMlpOutPad; e += 256) {
        const int i = e / kMlpOutPad, j = e % kMlpOutPad;
        float d = 0.f;
        if (rows[i] >= 0 && j < kMlpOut) {
          const float diff = y[e] - a.targets[(int64_t)rows[i] * kMlpOut + j];
          lsum += diff * diff;
          d = scale * diff;
        }
        dy[e] = f2bf(d);
      }
      __syncthreads();
      // dW3 += dY^T H2, db3 += sum dY
      wg_gemm(kMlpOutPad, kMlpHid, kMlpTile, dy, 1, kMlpOutPad, h2, kMlpHid, 1,
              [&](int o, int i, float v) { a.grad[kOffW3 + o * kMlpHid + i] += v; });
      if (tid < kMlpOutPad) {
        float s = 0.f;
        for (int i = 0; i < kMlpTile; ++i) s += bf2f(dy[i * kMlpOutPad + tid]);
        a.grad[kOffB3 + tid] += s;
      }
      __syncthreads();
      // dZ2 = bf16((dY W3) * [H2 > 0]), written over H2
      wg_gemm(kMlpTile, kMlpHid, kMlpOutPad, dy, kMlpOutPad, 1, w.w3, kMlpHid, 1,
              [&](int i, int j, float v) {
                const int e = i * kMlpHid + j;
                h2[e] = f2bf(bf2f(h2[e]) > 0.f ? v : 0.f);
              });
      __syncthreads();
      // dW2 += dZ2^T H1, db2 += sum dZ2
      wg_gemm(kMlpHid, kMlpHid, kMlpTile, h2, 1, kMlpHid, h1, kMlpHid, 1,
              [&](int o, int i, float v) { a.grad[kOffW2 + o * kMlpHid + i] += v; });
      if (tid < kMlpHid) {
        float s = 0.f;
        for (int i = 0; i < kMlpTile; ++i) s += bf2f(h2[i * kMlpHid + tid]);
        a.grad[kOffB2 + tid] += s;
      }
      __syncthreads();
      // dZ1 = bf16((dZ2 W2) * [H1 > 0]), written over H1
      wg_gemm(kMlpTile, kMlpHid, kMlpHid, h2, kMlpHid, 1, w.w2, kMlpHid, 1,
              [&](int i, int j, float v) {
                const int e = i * kMlpHid + j;
                h1[e] = f2bf(bf2f(h1[e]) > 0.f ? v : 0.f);
              });
      __syncthreads();
      // dW1 += dZ1^T X, db1 += sum dZ1
      wg_gemm(kMlpHid, kMlpInPad, kMlpTile, h1, 1, kMlpHid, sx, kMlpInPad, 1,
              [&](int o, int i, float v) { a.grad[kOffW1 + o * kMlpInPad + i] += v; });
      if (tid < kMlpHid) {
        float s = 0.f;
        for (int i = 0; i < kMlpTile; ++i) s += bf2f(h1[i * kMlpHid + tid]);
        a.grad[kOffB1 + tid] += s;
      }
      __syncthreads();
    }
    red[tid] = lsum;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) red[tid] += red[tid + s];
      __syncthreads();
    }
    if (tid == 0 && a.loss_out) a.loss_out[step] = red[0] / (float)(max(valid, 1) * kMlpOut);
    if (a.grad_only) break;
    const int t = a.t0 + step + 1;
    const float c1 = 1.f - powf(a.beta1, (float)t), c2 = 1.f - powf(a.beta2, (float)t);
    for (int e = tid; e < kMlpParams; e += 256) {
      const float g = a.grad[e];
      const float mm = a.beta1 * a.m[e] + (1.f - a.beta1) * g;
      const float vv = a.beta2 * a.v[e] + (1.f - a.beta2) * g * g;
      a.m[e] = mm;
      a.v[e] = vv;
      a.theta[e] -= a.lr * (mm / c1) / (sqrtf(vv / c2) + a.eps);
    }
    __syncthreads();
    mlp_load_weights(w, a.theta);
    __syncthreads();
  }
}

// Inference: y[n][12] for n samples, one 64-sample tile per workgroup.
__global__ __launch_bounds__(256) void k_mlp_forward(const float *theta, const float *mean,
                                                     const float *stdv, int n, const float *inputs,
                                                     float *out) {
  __shared__ MlpLds w;
  __shared__ uint16_t sx[kMlpTile * kMlpInPad];
  __shared__ uint16_t h1[kMlpTile * kMlpHid], h2[kMlpTile * kMlpHid];
  __shared__ float y[kMlpTile * kMlpOutPad];
  __shared__ int rows[kMlpTile];
  mlp_load_weights(w, theta);
  if (threadIdx.x < kMlpTile) {
    const int i = blockIdx.x * kMlpTile + threadIdx.x;
    rows[threadIdx.x] = i < n ? i : -1;
  }
  __syncthreads();
  mlp_load_inputs(sx, n, rows, inputs, mean, stdv);
  __syncthreads();
  mlp_forward_tile(w, sx, h1, h2, y);
  for (int e = threadIdx.x; e < kMlpTile * kMlpOut; e += 256) {
    const int i = e / kMlpOut, j = e % kMlpOut;
    if (rows[i] >= 0) out[(int64_t)rows[i] * kMlpOut + j] = y[i * kMlpOutPad + j];
  }
}

}  // namespace apic

namespace apic {

// Surrogate inside the reconstruction.
struct SurrogateArgs {
  const float *theta, *mean, *stdv;  // model (device)
  const float *positions;            // [batch][2] normalised (x, y), indexed by batch index
  float rho_max;                     // residual excess allowed before falling back (rad)
  float kappa_max;                   // tiles with kappa(A) above this keep the surrogate
  float resid_max;                   // tiles whose closed form fits worse keep the surrogate
  int seed_mode;                     // 0: the surrogate replaces the closed form when the
                                     // rule allows; 1: it also seeds the re-wrapped solve
};

// c_sur of every tile of the class: inputs are the tile position and the 32
// features log1p(cell weight / N^4) reduced by the pupil pass.
__global__ __launch_bounds__(256) void k_surrogate_predict(ClassArgs a, SurrogateArgs s) {
  __shared__ MlpLds w;
  __shared__ uint16_t sx[kMlpTile * kMlpInPad];
  __shared__ uint16_t h1[kMlpTile * kMlpHid], h2[kMlpTile * kMlpHid];
  __shared__ float y[kMlpTile * kMlpOutPad];
  mlp_load_weights(w, s.theta);
  const double n4 = (double)a.n * a.n * (double)a.n * a.n;
  for (int e = threadIdx.x; e < kMlpTile * kMlpInPad; e += 256) {
    const int i = e / kMlpInPad, c = e % kMlpInPad, t = blockIdx.x * kMlpTile + i;
    float v = 0.f;
    if (t < a.T && c < kMlpIn) {
      float raw;
      if (c < 2) raw = s.positions[(int64_t)a.gidx(t) * 2 + c];
      else raw = (float)log1p(a.at<double>(t, a.lay.sums)[92 + (c - 2)] / n4);
      v = (raw - s.mean[c]) / s.stdv[c];
    }
    sx[e] = f2bf(v);
  }
  __syncthreads();
  mlp_forward_tile(w, sx, h1, h2, y);
  for (int e = threadIdx.x; e < kMlpTile * kMlpOut; e += 256) {
    const int i = e / kMlpOut, j = e % kMlpOut, t = blockIdx.x * kMlpTile + i;
    if (t < a.T) a.at<float>(t, a.lay.sur)[j] = y[i * kMlpOutPad + j];
  }
}

// Fallback rule, one thread per tile.  R(c) = (sum w beta^2 - 2 c.b + c.A.c) / sum w
// is the weighted linearised residual of Eq. 10 for coefficients c; with
// rho = sqrt(max(0, R(c_sur) - R(c_cf))) the closed form is kept when
// rho > rho_max on a tile where the closed form is trustworthy (kappa(A) <=
// kappa_max and R(c_cf) <= resid_max: noise-only tiles have random wrapped
// phase differences, R near pi^2 / 3), the surrogate otherwise.  When the
// final pupil pass was re-wrapped about a seed c0 (the caller's, the last
// continuation band's or the surrogate's own prediction) its sums describe
// the increment, so both candidates are judged as R(c - c0).
__global__ __launch_bounds__(64) void k_surrogate_decide(ClassArgs a, SurrogateArgs s,
                                                         const float *caller_seed, int seed_src,
                                                         float *zout, float *zcf, float *zsur) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t >= a.T) return;
  const double *sm = a.at<double>(t, a.lay.sums);
  float *co = a.at<float>(t, a.lay.coef);
  const float *cs = a.at<float>(t, a.lay.sur);
  const float *c0 = seed_of(a, t, caller_seed, seed_src);
  double A[12][12], b[12];
  int e = 0;
  for (int p = 0; p < 12; ++p)
    for (int q = p; q < 12; ++q, ++e) A[p][q] = A[q][p] = sm[e];
  for (int p = 0; p < 12; ++p) b[p] = sm[78 + p];
  auto resid = [&](const float *c) {
    double d[12];
    for (int p = 0; p < 12; ++p) d[p] = (double)c[p] - (c0 ? (double)c0[p] : 0.0);
    double cb = 0.0, cac = 0.0;
    for (int p = 0; p < 12; ++p) {
      cb += d[p] * b[p];
      double r = 0.0;
      for (int q = 0; q < 12; ++q) r += A[p][q] * d[q];
      cac += d[p] * r;
    }
    return (sm[90] - 2.0 * cb + cac) / sm[91];
  };
  const double r_cf = resid(co);
  const double rho = sqrt(fmax(0.0, resid(cs) - r_cf));
  const bool keep_cf = rho > (double)s.rho_max && co[14] <= s.kappa_max && r_cf <= s.resid_max;
  const int g = a.gidx(t);
  for (int j = 0; j < 12; ++j) {
    if (zcf) zcf[(int64_t)g * 15 + 3 + j] = co[j];
    if (zsur) zsur[(int64_t)g * 15 + 3 + j] = cs[j];
    if (!keep_cf) co[j] = cs[j];
    if (zout) zout[(int64_t)g * 15 + 3 + j] = co[j];
  }
  for (int j = 0; j < 3; ++j) {
    if (zcf) zcf[(int64_t)g * 15 + j] = 0.f;
    if (zsur) zsur[(int64_t)g * 15 + j] = 0.f;
    if (zout) zout[(int64_t)g * 15 + j] = 0.f;
  }
  status_or(a, t, keep_cf ? APIC_TILE_FALLBACK_USED : APIC_TILE_SURROGATE_USED);
}

}  // namespace apic
