// Device-side shared definitions: complex helpers, the per-class launch
// argument block, twiddle tables and small utilities.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan.hpp"

namespace apic {

using c32 = float2;
using c64 = double2;

template <class C> struct real_of;
template <> struct real_of<c32> { using type = float; };
template <> struct real_of<c64> { using type = double; };

__device__ __forceinline__ c32 cmul(c32 a, c32 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ c64 cmul(c64 a, c64 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ c32 cmulc(c32 a, c32 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ c64 cmulc(c64 a, c64 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ c32 cadd(c32 a, c32 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c64 cadd(c64 a, c64 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ c32 csub(c32 a, c32 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ c64 csub(c64 a, c64 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ c32 cscale(c32 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ c64 cscale(c64 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ c32 cconj(c32 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ c64 cconj(c64 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ c64 to64(c32 a) { return make_double2(a.x, a.y); }
__device__ __forceinline__ c32 to32(c64 a) { return make_float2((float)a.x, (float)a.y); }
template <class C> __device__ __forceinline__ C czero();
template <> __device__ __forceinline__ c32 czero<c32>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ c64 czero<c64>() { return make_double2(0.0, 0.0); }
template <class C> __device__ __forceinline__ C cmake(double re, double im);
template <> __device__ __forceinline__ c32 cmake<c32>(double re, double im) {
  return make_float2((float)re, (float)im);
}
template <> __device__ __forceinline__ c64 cmake<c64>(double re, double im) {
  return make_double2(re, im);
}

__device__ __forceinline__ int signed_idx(int i, int n) { return i < (n >> 1) ? i : i - n; }
__device__ __forceinline__ int fft_pos(int k, int n) { return k & (n - 1); }
__device__ __forceinline__ bool in_grid(int ky, int kx, int n) {
  const int h = n >> 1;
  return ky >= -h && ky < h && kx >= -h && kx < h;
}
__device__ __forceinline__ int kunpack_y(uint32_t w) { return (int)(int16_t)(uint16_t)(w & 0xffffu); }
__device__ __forceinline__ int kunpack_x(uint32_t w) { return (int)(int16_t)(uint16_t)(w >> 16); }

// Twiddle tables exp(-2 pi j t / L) for L = 64 .. 1024, stored at offset L - 64.
constexpr int kTwTotal = 64 + 128 + 256 + 512 + 1024;
__device__ c32 g_tw32[kTwTotal];
__device__ c64 g_tw64[kTwTotal];

template <class C> __device__ __forceinline__ const C *tw_table(int L);
template <> __device__ __forceinline__ const c32 *tw_table<c32>(int L) { return g_tw32 + (L - 64); }
template <> __device__ __forceinline__ const c64 *tw_table<c64>(int L) { return g_tw64 + (L - 64); }

// Launch arguments of one geometry class (passed by value to every kernel).
struct ClassArgs {
  int n, nf, n_bf, n_df, n_img, T;
  int r2;                 // Circ(k) <=> kx^2 + ky^2 <= r2
  float r, inv_r;
  double r_d;             // pupil radius in double precision
  float log_floor_rel;
  int n_rows, n_chunks, nu_pad;
  int fft_var;                    // column-pass panel: 0 ColShape, 1 ColShapeAlt
  int n_band;                     // band passes of the pupil continuation (0: single pass)
  int band_rows[kPupilBands];     // rows of each band pass (a prefix of the sorted rows)
  double ridge_pupil, ridge_df;
  int kx[kMaxImg], ky[kMaxImg];  // NA-matched first, then darkfield
  const float *images;
  // Per-tile descriptors: affine in t (tile t of the class at base + t * step)
  // when `affine` is set, else device arrays copied from the caller's list.
  int affine;
  int64_t img0, img_step, out0, out_step;
  int g0, g_step;
  const int64_t *d_img_off;       // [T] float offset of each tile's image stack
  const int64_t *d_out_off;       // [T] complex offset of each tile's output
  const int32_t *d_gidx;          // [T] index of the tile in the caller's batch
  char *ws;                       // workspace base of tile 0 of this class
  int64_t stride;                 // bytes between tiles
  TileLayout lay;
  uint32_t *status;               // caller's status array (indexed by gidx)
  const uint32_t *row_il, *row_k; // pupil rows
  const int16_t *known_at;        // N*N
  const uint32_t *coords;         // darkfield coordinate lists
  const uint64_t *masks;          // darkfield block-sparsity masks
  int n_pix;                      // pupil pixels of the pixel-domain solve (0: unsupported)
  const uint32_t *pix_tab;        // pixel k, per-row pixel pairs, LED pixels
  const double *pix_ginv;         // inverse Gram matrix of Z_1..Z_15 over the pixels

  __device__ __forceinline__ char *tile(int t) const { return ws + (int64_t)t * stride; }
  template <class T> __device__ __forceinline__ T *at(int t, int64_t off) const {
    return reinterpret_cast<T *>(tile(t) + off);
  }
  __device__ __forceinline__ int64_t img_off(int t) const {
    return affine ? img0 + (int64_t)t * img_step : d_img_off[t];
  }
  __device__ __forceinline__ int64_t out_off(int t) const {
    return affine ? out0 + (int64_t)t * out_step : d_out_off[t];
  }
  __device__ __forceinline__ int gidx(int t) const { return affine ? g0 + t * g_step : d_gidx[t]; }
  __device__ __forceinline__ const float *image(int t, int i) const {
    return images + img_off(t) + (int64_t)i * n * n;
  }
  __device__ __forceinline__ bool circ(int ky_, int kx_) const {
    return kx_ * kx_ + ky_ * ky_ <= r2;
  }
};

// Per-darkfield-step arguments.
struct StepArgs {
  int j;              // darkfield index (0-based)
  int img;            // image index in the tile stack (n_bf + j)
  int kx, ky;
  int nu, np, m, ne;
  const uint32_t *u, *p, *q, *e;
  const uint64_t *gmask;          // block-sparsity masks of E chunks
  int nwe;                        // mask words per block of 64 unknowns
  const uint64_t *qbits;          // Q membership over the grid (bit y N + x)
  // rows of D (P_hat and the unknowns), of Q (b), where z is read, and
  // where P_hat is written (D and the previous image's D, which it clears):
  // FFT-order first row and row count, rounded up to whole row-pass
  // workgroups
  int dy0, dn, qy0, qn, zy0, zn, py0, pn;
};

// Row y (FFT order) lies in the cyclic range of cnt rows from y0.
__device__ __forceinline__ bool row_in(int y, int y0, int cnt, int n) {
  return ((y - y0) & (n - 1)) < cnt;
}

// Workgroups are dispatched to the 8 XCDs round robin (workgroup b on XCD
// b mod 8), each XCD with its own L2.  Maps the b-th of n workgroups to a work
// index so that each XCD takes one contiguous range of work items.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  constexpr int kXcd = 8;
  const int per = n / kXcd;
  if (b >= per * kXcd) return b;
  return (b % kXcd) * per + b / kXcd;
}

__device__ __forceinline__ void status_or(const ClassArgs &a, int t, uint32_t bits) {
  atomicOr(a.status + a.gidx(t), bits);
}

}  // namespace apic
