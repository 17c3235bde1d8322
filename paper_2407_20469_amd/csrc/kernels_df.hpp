// Darkfield half of the reconstruction (Fig. 2 lower part, Eq. 11-13) and the
// upsampled output.  For darkfield image j (known set P, unknown set U, linear
// region Q, excluded set E = (P - U) - Q, all plan tables):
//
//   P_hat(k) = O_hat(k) exp(j phi_c(k + k_j)) on P, 0 elsewhere  (OpP1 load)
//   z        = fft2(|ifft2 P_hat|^2 + i I_j)  FP64 passes        (OpP*)
//   fpp(k)   = (z(k) + conj z(-k)) / 2 = fft2(|P|^2)(k)
//   fimg(k)  = (z(k) - conj z(-k)) / 2i = fft2(I_j)(k)
//   b(k)     = conj(fimg(k) - fpp(k)),  k in Q                   (OpR1)
//   G[u,u']  = sum_{k in Q} P_hat(u+k) conj(P_hat(u'+k)) / N^4   (k_df_gram)
//            = fpp(u - u') / N^2 - sum_{k in E} P_hat(u+k) conj(P_hat(u'+k)) / N^4
//   v[u]     = sum_{k in Q} P_hat(u+k) b(k) / N^2                (OpR*, k_df_rhs_gather)
//            = fft2(p . fft2(b))(u) / N^2,  p = ifft2(P_hat) (normalised)
//   x        = (G + lambda tr(G)/N_u I)^-1 v   FP64 Cholesky     (chol.hpp)
//   O_hat(u) = x(u) exp(-j phi_c(u + k_j)),  u in U              (k_chol_back)
//
// |P|^2 and I_j are both real, so their spectra are Hermitian and one complex
// transform of |P|^2 + i I_j carries both: the pair z(k), z(-k) separates them.
// The gram identity: the sum over every k of P_hat(u+k) conj(P_hat(u'+k)) is
// the autocorrelation of P_hat at u' - u, which is N^2 fpp(u - u'); Q and E
// partition P - U, so the Q-sum is that minus the (smaller) E-sum.
// The right-hand side: with P_hat = fft2(p), sum_k b(k) P_hat(u + k) =
// sum_x p(x) fft2(b)(x) exp(-2 pi i u.x / N), a forward transform of
// p . fft2(b); the circular sums equal the linear ones because 4r < N (plan).
#pragma once

#include "fft.hpp"
#include "zern.hpp"

namespace apic {

// P_hat at grid index pix of tile t (zero off the shifted pupil and on
// points not yet known before image j).
__device__ __forceinline__ c64 phat_at(const ClassArgs &a, const StepArgs &s, int t, int pix) {
  const int ky = signed_idx(pix / a.n, a.n), kx = signed_idx(pix % a.n, a.n);
  c64 v = make_double2(0.0, 0.0);
  const int qy = ky + s.ky, qx = kx + s.kx;
  if (a.circ(qy, qx) && a.known_at[pix] < s.j) {
    const float *co = a.at<float>(t, a.lay.coef);
    float c[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) c[j] = co[j];
    const float ph = pupil_phase12(c, (float)qx, (float)qy, a.inv_r);
    float sn, cs;
    sincosf(ph, &sn, &cs);
    const c32 o = a.at<c32>(t, a.lay.ohat)[pix];
    v = make_double2((double)o.x * cs - (double)o.y * sn, (double)o.x * sn + (double)o.y * cs);
  }
  return v;
}

// P chain, pass 1 (rows): form P_hat (kept for the gram's gathers) and
// row-IFFT it.  P_hat is zero outside the rows of D, so the pass runs over
// D's rows and those of the previous image's D (which it clears); every row
// outside the two already holds zeros (the first image of a call covers all
// rows).
template <int N> struct OpP1 {
  static constexpr bool INV1 = true, TWO = false, INV2 = false;
  ClassArgs a;
  StepArgs s;
  __device__ int rows() const { return s.pn; }
  __device__ int row_of(int r) const { return (s.py0 + r) & (N - 1); }
  __device__ c64 load(int t, int y, int x) const {
    const c64 v = phat_at(a, s, t, y * N + x);
    a.at<c64>(t, a.lay.phat)[y * N + x] = v;
    return v;
  }
  __device__ void mid(int, int, int, c64 &) const {}
  // rows outside D are zero rows: not stored, and read as zero by pass 2
  __device__ void store(int t, int y, int x, c64 v) const {
    if (row_in(y, s.dy0, s.dn, N)) a.at<c64>(t, a.lay.dtmp)[y * N + x] = v;
  }
};
// Pass 2 (columns): column IFFT gives N^2 P; keep P (normalised) for the
// right-hand side; |P|^2 = |.|^2 / N^4 as the real part and the darkfield
// image as the imaginary part; column FFT.
template <int N> struct OpP2 {
  static constexpr bool INV1 = true, TWO = true, INV2 = false, SIDE = true;
  ClassArgs a;
  StepArgs s;
  __device__ c64 load(int t, int y, int x) const {
    if (!row_in(y, s.dy0, s.dn, N)) return make_double2(0.0, 0.0);
    return a.at<c64>(t, a.lay.dtmp)[y * N + x];
  }
  // the image pixel, read with the loads
  __device__ float side(int t, int y, int x) const { return a.image(t, s.img)[y * N + x]; }
  __device__ void mid_side(int t, int y, int x, c64 &v, float img) const {
    constexpr double inv2 = 1.0 / ((double)N * N), inv4 = inv2 * inv2;
    a.at<c64>(t, a.lay.ptil)[y * N + x] = make_double2(v.x * inv2, v.y * inv2);
    v = make_double2((v.x * v.x + v.y * v.y) * inv4, (double)img);
  }
  // only the rows where z is read go on to pass 3
  __device__ void store(int t, int y, int x, c64 v) const {
    if (row_in(y, s.zy0, s.zn, N)) a.at<c64>(t, a.lay.dtmp)[y * N + x] = v;
  }
};
// Pass 3 (the rows where z is read): row FFT completes z = fft2(|P|^2 + i I_j).
template <int N> struct OpP3 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  StepArgs s;
  __device__ int rows() const { return s.zn; }
  __device__ int row_of(int r) const { return (s.zy0 + r) & (N - 1); }
  __device__ c64 load(int t, int y, int x) const { return a.at<c64>(t, a.lay.dtmp)[y * N + x]; }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.fpp)[y * N + x] = v; }
};
// Grid index of -k for the grid index of k.
template <int N> __device__ __forceinline__ int neg_pix(int y, int x) {
  return ((N - y) & (N - 1)) * N + ((N - x) & (N - 1));
}

// Right-hand side pass 1 (rows): b(k) = conj(fft2(I_j)(k) - fft2(|P|^2)(k))
// on Q (Eq. 13, conjugated), zero elsewhere, both spectra separated from z;
// row FFT.
template <int N> struct OpR1 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  StepArgs s;
  __device__ int rows() const { return s.qn; }  // the rows of Q; pass 2 reads the rest as zero
  __device__ int row_of(int r) const { return (s.qy0 + r) & (N - 1); }
  __device__ c64 load(int t, int y, int x) const {
    const int pix = y * N + x;
    if (!((s.qbits[pix >> 6] >> (pix & 63)) & 1u)) return make_double2(0.0, 0.0);
    // conj(fimg - fpp) from z(k) and z(-k)
    const c64 *z = a.at<c64>(t, a.lay.fpp);
    const c64 z1 = z[pix], z2 = z[neg_pix<N>(y, x)];
    return make_double2(0.5 * ((z1.y + z2.y) - (z1.x + z2.x)), 0.5 * ((z1.x - z2.x) + (z1.y - z2.y)));
  }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.dtmp)[y * N + x] = v; }
};
// Pass 2 (columns): column FFT completes fft2(b); times p; column FFT.
template <int N> struct OpR2 {
  static constexpr bool INV1 = false, TWO = true, INV2 = false;
  ClassArgs a;
  StepArgs s;
  __device__ c64 load(int t, int y, int x) const {
    if (!row_in(y, s.qy0, s.qn, N)) return make_double2(0.0, 0.0);
    return a.at<c64>(t, a.lay.dtmp)[y * N + x];
  }
  __device__ void mid(int t, int y, int x, c64 &v) const {
    v = cmul(v, a.at<c64>(t, a.lay.ptil)[y * N + x]);
  }
  // only the rows of D (which hold U) go on to pass 3
  __device__ void store(int t, int y, int x, c64 v) const {
    if (row_in(y, s.dy0, s.dn, N)) a.at<c64>(t, a.lay.dtmp)[y * N + x] = v;
  }
};
// Pass 3 (rows of D): row FFT completes N^2 v on the rows that hold U.
template <int N> struct OpR3 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  StepArgs s;
  __device__ int rows() const { return s.dn; }
  __device__ int row_of(int r) const { return (s.dy0 + r) & (N - 1); }
  __device__ c64 load(int t, int y, int x) const { return a.at<c64>(t, a.lay.dtmp)[y * N + x]; }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.dtmp)[y * N + x] = v; }
};
// conj(v[u]) into row n of the gram storage (the Cholesky's right-hand-side row).
__global__ __launch_bounds__(256) void k_df_rhs_gather(ClassArgs a, StepArgs s) {
  const int t = blockIdx.y;
  const int u = blockIdx.x * 256 + threadIdx.x;
  if (u >= s.nu) return;
  const uint32_t w = s.u[u];
  const int pos = fft_pos(kunpack_y(w), a.n) * a.n + fft_pos(kunpack_x(w), a.n);
  const c64 c = a.at<c64>(t, a.lay.dtmp)[pos];
  const double inv2 = 1.0 / ((double)a.n * a.n);
  a.at<c64>(t, a.lay.gram)[(int64_t)s.nu * a.nu_pad + u] = make_double2(c.x * inv2, -c.y * inv2);
}

// The gram reads P_hat(u + k) for u in U, k in E with periodic indexing.
// u + k lies within 3r of the darkfield support's centre and P within r of
// it, so a wrapped position (off by a multiple of N > 4r) never falls in P,
// where P_hat is nonzero: the periodic read equals the bounded one.

// Gram of the darkfield system in 32 x 32 blocks (I >= J) of the N_u x N_u
// Hermitian matrix, one wavefront per block: lane (ty, tx) = (lane / 8,
// lane % 8) holds rows ty + 8 i and columns tx + 8 j, so the lanes reading one
// LDS row read consecutive elements (no bank conflicts).
//
// A product P_hat(u + k) conj(P_hat(u' + k)) is nonzero only when both u + k
// and u' + k fall in P, so the E-sum is sparse.  A plan mask per half-block
// (16 unknowns) marks the excluded k for which some unknown of the half lands
// in P; a block pair visits the k marked in a half of each block, in
// ascending order, walking the mask words with wave-uniform state, two k per
// iteration (four k).  Every lane holds part of each 16 x 16 quadrant (rows ty + 8 i
// lie in half i / 2, columns tx + 8 j in half j / 2), so for each k the wave
// skips, with a uniform branch, the quadrants whose two halves do not both
// mark it: a quarter of the multiply-adds per quadrant.  Each
// lane gathers two operand elements per iteration (its unknown u of each
// block, for two of the four k); a lane without an element reads a grid
// position that is never in P (the point opposite the support's centre),
// where P_hat is zero, so every lane loads unconditionally.  Software
// pipeline: while the current four k are multiplied from LDS, the operands of
// the next four are in flight and the four after those are being looked up in
// E.  Four k per iteration (not two) give each wave twice the multiply-adds
// per gather latency, which the four waves per SIMD did not hide.  A diagonal block
// has one operand and is formed whole (its upper half is not read by the
// Cholesky).
constexpr int kGramRows = 4;                          // excluded k per iteration
constexpr int kGramSlots = kGramRows * kGramUB / 64;  // gathers per lane and iteration
static_assert(kGramSlots * 64 == kGramRows * kGramUB, "the lanes cover the gathers exactly");
constexpr uint32_t kNoK = 0x7fff7fffu;  // padding: outside every support
__global__ __launch_bounds__(64) void k_df_gram(ClassArgs a, StepArgs s) {
  const int nb = (s.nu + kGramUB - 1) / kGramUB;
  const int ntri = nb * (nb + 1) / 2;
  const int bid = xcd_remap(blockIdx.x, gridDim.x);  // a tile's blocks on one XCD
  const int t = bid / ntri;
  int rem = bid % ntri, I = 0;
  while (rem > I) {
    rem -= I + 1;
    ++I;
  }
  const int J = rem;
  const bool diag = I == J;
  const c64 *phat = a.at<c64>(t, a.lay.phat);
  // a grid position outside the darkfield support (centre -k_j, radius
  // r < N / 4): the centre shifted by (N/2, N/2), at distance N / sqrt 2
  const int zpos = fft_pos(-s.ky + a.n / 2, a.n) * a.n + fft_pos(-s.kx + a.n / 2, a.n);
  __shared__ c64 sA[kGramRows][kGramUB];
  __shared__ c64 sB[kGramRows][kGramUB];
  __shared__ uint32_t su[2][kGramUB];
  const int lane = threadIdx.x;
  const int ty = lane >> 3, tx = lane & 7;
  const int uu = lane & (kGramUB - 1), kk = lane / kGramUB;  // slot sl: k row kk + 2 sl
  const int ui = I * kGramUB + uu, uj = J * kGramUB + uu;
  const uint32_t wa = ui < s.nu ? s.u[ui] : kNoK;
  const uint32_t wb = uj < s.nu ? s.u[uj] : kNoK;
  if (lane < kGramUB) {
    su[0][lane] = wa;
    su[1][lane] = wb;
  }
  const int ay = kunpack_y(wa), ax = kunpack_x(wa), by = kunpack_y(wb), bx = kunpack_x(wb);
  // marked k in ascending order, walked with wave-uniform state: each step
  // returns the E row in the low 24 bits and the live quadrants (bit 2 hi +
  // hj: row half hi, column half hj) above them
  const uint64_t *ma0 = s.gmask + (int64_t)(2 * I) * s.nwe, *ma1 = ma0 + s.nwe;
  const uint64_t *mb0 = s.gmask + (int64_t)(2 * J) * s.nwe, *mb1 = mb0 + s.nwe;
  int mw = 0;
  uint64_t w00 = 0, w01 = 0, w10 = 0, w11 = 0, bits = 0;
  auto load_word = [&]() {
    const uint64_t a0 = ma0[mw], a1 = ma1[mw], b0 = mb0[mw], b1 = mb1[mw];
    w00 = a0 & b0;
    w01 = a0 & b1;
    w10 = a1 & b0;
    w11 = a1 & b1;
    bits = w00 | w01 | w10 | w11;
  };
  if (s.nwe > 0) load_word();
  auto next_k = [&]() -> int {
    while (bits == 0) {
      if (++mw >= s.nwe) return -1;
      load_word();
    }
    const int p = __builtin_ctzll(bits);
    bits &= bits - 1;
    const int q = (int)((w00 >> p) & 1) | (int)(((w01 >> p) & 1) << 1) |
                  (int)(((w10 >> p) & 1) << 2) | (int)(((w11 >> p) & 1) << 3);
    return (mw * 64 + p) | (q << 24);
  };
  constexpr int kRowMask = (1 << 24) - 1;
  // this lane's excluded k of slot sl among four E rows (kNoK for a missing
  // row).  The rows are wave-uniform: both candidate words are read through
  // the constant address space (scalar loads; the table is read-only here)
  // and each lane selects its own.
  typedef const uint32_t __attribute__((address_space(4))) *cword_ptr;
  const cword_ptr ew = (cword_ptr)s.e;
  auto k_of = [&](const int (&rr)[kGramRows], int sl) -> uint32_t {
    const int r0 = rr[2 * sl], r1 = rr[2 * sl + 1];
    const uint32_t e0 = r0 >= 0 ? ew[r0 & kRowMask] : kNoK;
    const uint32_t e1 = r1 >= 0 ? ew[r1 & kRowMask] : kNoK;
    return kk ? e1 : e0;
  };
  // this lane's operand elements of one k: P_hat(u_a + k), P_hat(u_b + k)
  // (the second only off the diagonal)
  struct Ops {
    c64 a, b;
  };
  // grid position of u + k with shifts and masks (N is a power of two),
  // always in range; a select replaces it by zpos for a missing u or k
  const uint32_t nmask = (uint32_t)a.n - 1u, nshift = (uint32_t)__builtin_ctz(a.n);
  const bool va = wa != kNoK, vb = wb != kNoK;
  auto pos_of = [&](int uy, int ux, int ky, int kx) -> uint32_t {
    return ((((uint32_t)(uy + ky)) & nmask) << nshift) | (((uint32_t)(ux + kx)) & nmask);
  };
  auto gather = [&](uint32_t kw) -> Ops {
    const bool kv = kw != kNoK;
    const int ky = kunpack_y(kw), kx = kunpack_x(kw);
    const uint32_t ia = (kv && va) ? pos_of(ay, ax, ky, kx) : (uint32_t)zpos;
    Ops o;
    o.a = phat[ia];
    o.b = make_double2(0.0, 0.0);
    if (!diag) {
      const uint32_t ib = (kv && vb) ? pos_of(by, bx, ky, kx) : (uint32_t)zpos;
      o.b = phat[ib];
    }
    return o;
  };
  c64 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  __syncthreads();
  int cur[kGramRows], nxt[kGramRows];
#pragma unroll
  for (int r = 0; r < kGramRows; ++r) cur[r] = next_k();
#pragma unroll
  for (int r = 0; r < kGramRows; ++r) nxt[r] = next_k();
  static_assert(kGramSlots == 2, "two gathers per lane and iteration");
  Ops g0 = gather(k_of(cur, 0)), g1 = gather(k_of(cur, 1));
  uint32_t kw_nxt0 = k_of(nxt, 0), kw_nxt1 = k_of(nxt, 1);
  const c64(*sBd)[kGramUB] = diag ? sA : sB;  // the column operand
  while (cur[0] >= 0) {
    sA[kk][uu] = g0.a;
    sA[kk + 2][uu] = g1.a;
    if (!diag) {
      sB[kk][uu] = g0.b;
      sB[kk + 2][uu] = g1.b;
    }
    __syncthreads();
    int nn[kGramRows];
#pragma unroll
    for (int r = 0; r < kGramRows; ++r) nn[r] = next_k();  // -1 once the walk has ended
    const uint32_t kw_nn0 = k_of(nn, 0), kw_nn1 = k_of(nn, 1);
    g0 = gather(kw_nxt0);
    g1 = gather(kw_nxt1);
#pragma unroll
    for (int r = 0; r < kGramRows; ++r) {
      if (cur[r] < 0) break;  // wave-uniform; the rows in use are a prefix
      const int quad = cur[r] >> 24;
      c64 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[r][ty + 8 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sBd[r][tx + 8 * j];
#pragma unroll
      for (int hi = 0; hi < 2; ++hi)
#pragma unroll
        for (int hj = 0; hj < 2; ++hj) {
          if (!(quad & (1 << (2 * hi + hj)))) continue;  // wave-uniform
#pragma unroll
          for (int i = 2 * hi; i < 2 * hi + 2; ++i)
#pragma unroll
            for (int j = 2 * hj; j < 2 * hj + 2; ++j) {  // acc += a * conj(b)
              acc[i][j].x = fma(av[i].x, bv[j].x, fma(av[i].y, bv[j].y, acc[i][j].x));
              acc[i][j].y = fma(av[i].y, bv[j].x, fma(-av[i].x, bv[j].y, acc[i][j].y));
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kGramRows; ++r) {
      cur[r] = nxt[r];
      nxt[r] = nn[r];
    }
    kw_nxt0 = kw_nn0;
    kw_nxt1 = kw_nn1;
  }
  // G[r][c] = fft2(|P|^2)(d) / N^2 - acc / N^4 with d = u_r - u_c, where
  // fft2(|P|^2)(d) = (z(d) + conj z(-d)) / 2; per row the Toeplitz values are
  // read first (padding entries read a harmless value), then the valid
  // entries stored, so those loads are in flight together
  const double n2 = (double)a.n * a.n, inv2 = 1.0 / n2, inv4 = inv2 * inv2, hinv2 = 0.5 * inv2;
  const c64 *z = a.at<c64>(t, a.lay.fpp);
  c64 *G = a.at<c64>(t, a.lay.gram);
  const int ld = a.nu_pad;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t wr = su[0][ty + 8 * i];
    const int ry = kunpack_y(wr), rx = kunpack_x(wr);
    const int r = I * kGramUB + ty + 8 * i;
    c64 tv[4], tw[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const uint32_t wc = su[1][tx + 8 * j];
      const int dy = ry - kunpack_y(wc), dx = rx - kunpack_x(wc);
      tv[j] = z[fft_pos(dy, a.n) * a.n + fft_pos(dx, a.n)];
      tw[j] = z[fft_pos(-dy, a.n) * a.n + fft_pos(-dx, a.n)];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = J * kGramUB + tx + 8 * j;
      if (r < s.nu && c < s.nu)
        G[(int64_t)r * ld + c] = make_double2((tv[j].x + tw[j].x) * hinv2 - acc[i][j].x * inv4,
                                              (tv[j].y - tw[j].y) * hinv2 - acc[i][j].y * inv4);
    }
  }
}

// Output pass 1 (rows of the fN grid that carry spectrum, i.e. |ky| < N/2):
// zero-embed the N x N spectrum and row-IFFT.
template <int NF> struct OpOut1 {
  static constexpr bool INV1 = true, TWO = false, INV2 = false;
  ClassArgs a;
  const c32 *src;     // if set: spectra at src + t * N * N, else the tile's O_hat
  __device__ int rows() const { return a.n; }
  __device__ int row_of(int r) const { return fft_pos(signed_idx(r, a.n), NF); }
  __device__ c32 load(int t, int y, int x) const {
    const int ky = signed_idx(y, NF), kx = signed_idx(x, NF);
    const int h = a.n >> 1;
    if (kx < -h || kx >= h) return make_float2(0.f, 0.f);
    const int pos = fft_pos(ky, a.n) * a.n + fft_pos(kx, a.n);
    return src ? src[(int64_t)t * a.n * a.n + pos] : a.at<c32>(t, a.lay.ohat)[pos];
  }
  __device__ void mid(int, int, int, c32 &) const {}
  __device__ void store(int t, int y, int x, c32 v) const {
    a.at<c32>(t, a.lay.stack)[(int64_t)y * NF + x] = v;
  }
};
// Output pass 2 (columns): rows without spectrum are zero; column IFFT,
// scale f^2 / (fN)^2 = 1 / N^2, store the field.
template <int NF> struct OpOut2 {
  static constexpr bool INV1 = true, TWO = false, INV2 = false;
  ClassArgs a;
  c32 *field;
  __device__ c32 load(int t, int y, int x) const {
    const int ky = signed_idx(y, NF), h = a.n >> 1;
    if (ky < -h || ky >= h) return make_float2(0.f, 0.f);
    return a.at<c32>(t, a.lay.stack)[(int64_t)y * NF + x];
  }
  __device__ void mid(int, int, int, c32 &) const {}
  __device__ void store(int t, int y, int x, c32 v) const {
    const float inv = 1.0f / ((float)a.n * (float)a.n);
    field[a.out_off(t) + (int64_t)y * NF + x] = cscale(v, inv);
  }
};

}  // namespace apic
