// Darkfield half of the reconstruction (Fig. 2 lower part, Eq. 11-13) and the
// upsampled output.  For darkfield image j (known set P, unknown set U, linear
// region Q, excluded set E = (P - U) - Q, all plan tables):
//
//   P_hat(k) = O_hat(k) exp(j phi_c(k + k_j)) on P              (k_df_phat)
//   fpp      = fft2(|ifft2 P_hat|^2)        FP64 passes          (OpP*)
//   fimg     = fft2(I_j)                    FP64 passes          (OpImg*)
//   b(k)     = conj(fimg(k) - fpp(k)),  k in Q                   (OpR1)
//   G[u,u']  = sum_{k in Q} P_hat(u+k) conj(P_hat(u'+k)) / N^4   (k_df_gram)
//            = fpp(u - u') / N^2 - sum_{k in E} P_hat(u+k) conj(P_hat(u'+k)) / N^4
//   v[u]     = sum_{k in Q} P_hat(u+k) b(k) / N^2                (OpR*, k_df_rhs_gather)
//            = fft2(p . fft2(b))(u) / N^2,  p = ifft2(P_hat) (normalised)
//   x        = (G + lambda tr(G)/N_u I)^-1 v   FP64 Cholesky     (chol.hpp)
//   O_hat(u) = x(u) exp(-j phi_c(u + k_j)),  u in U              (k_chol_back)
//
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

__global__ __launch_bounds__(256) void k_df_phat(ClassArgs a, StepArgs s) {
  const int nn = a.n * a.n;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)a.T * nn) return;
  const int t = (int)(gid / nn), pix = (int)(gid % nn);
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
  a.at<c64>(t, a.lay.phat)[pix] = v;
}

// P chain, pass 1 (rows): row IFFT of P_hat.
template <int N> struct OpP1 {
  static constexpr bool INV1 = true, TWO = false, INV2 = false;
  ClassArgs a;
  __device__ int rows() const { return N; }
  __device__ int row_of(int r) const { return r; }
  __device__ c64 load(int t, int y, int x) const { return a.at<c64>(t, a.lay.phat)[y * N + x]; }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.dtmp)[y * N + x] = v; }
};
// Pass 2 (columns): column IFFT gives N^2 P; keep P (normalised) for the
// right-hand side; |P|^2 = |.|^2 / N^4; column FFT.
template <int N> struct OpP2 {
  static constexpr bool INV1 = true, TWO = true, INV2 = false;
  ClassArgs a;
  __device__ c64 load(int t, int y, int x) const { return a.at<c64>(t, a.lay.dtmp)[y * N + x]; }
  __device__ void mid(int t, int y, int x, c64 &v) const {
    constexpr double inv2 = 1.0 / ((double)N * N), inv4 = inv2 * inv2;
    a.at<c64>(t, a.lay.ptil)[y * N + x] = make_double2(v.x * inv2, v.y * inv2);
    v = make_double2((v.x * v.x + v.y * v.y) * inv4, 0.0);
  }
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.dtmp)[y * N + x] = v; }
};
// Pass 3 (rows): row FFT completes fpp = fft2(|P|^2).
template <int N> struct OpP3 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  __device__ int rows() const { return N; }
  __device__ int row_of(int r) const { return r; }
  __device__ c64 load(int t, int y, int x) const { return a.at<c64>(t, a.lay.dtmp)[y * N + x]; }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.fpp)[y * N + x] = v; }
};
// fft2 of the darkfield image in FP64: rows, then columns in place.
template <int N> struct OpImg1 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  int img;
  __device__ int rows() const { return N; }
  __device__ int row_of(int r) const { return r; }
  __device__ c64 load(int t, int y, int x) const {
    return make_double2((double)a.image(t, img)[y * N + x], 0.0);
  }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.fimg)[y * N + x] = v; }
};
template <int N> struct OpImg2 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  __device__ c64 load(int t, int y, int x) const { return a.at<c64>(t, a.lay.fimg)[y * N + x]; }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.fimg)[y * N + x] = v; }
};

// Right-hand side pass 1 (rows): b(k) = conj(fft2(I_j)(k) - fft2(|P|^2)(k))
// on Q (Eq. 13, conjugated), zero elsewhere; row FFT.
template <int N> struct OpR1 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  const uint64_t *qbits;
  __device__ int rows() const { return N; }
  __device__ int row_of(int r) const { return r; }
  __device__ c64 load(int t, int y, int x) const {
    const int pix = y * N + x;
    if (!((qbits[pix >> 6] >> (pix & 63)) & 1u)) return make_double2(0.0, 0.0);
    return cconj(csub(a.at<c64>(t, a.lay.fimg)[pix], a.at<c64>(t, a.lay.fpp)[pix]));
  }
  __device__ void mid(int, int, int, c64 &) const {}
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.dtmp)[y * N + x] = v; }
};
// Pass 2 (columns): column FFT completes fft2(b); times p; column FFT.
template <int N> struct OpR2 {
  static constexpr bool INV1 = false, TWO = true, INV2 = false;
  ClassArgs a;
  __device__ c64 load(int t, int y, int x) const { return a.at<c64>(t, a.lay.dtmp)[y * N + x]; }
  __device__ void mid(int t, int y, int x, c64 &v) const {
    v = cmul(v, a.at<c64>(t, a.lay.ptil)[y * N + x]);
  }
  __device__ void store(int t, int y, int x, c64 v) const { a.at<c64>(t, a.lay.dtmp)[y * N + x] = v; }
};
// Pass 3 (rows): row FFT completes N^2 v over the grid.
template <int N> struct OpR3 {
  static constexpr bool INV1 = false, TWO = false, INV2 = false;
  ClassArgs a;
  __device__ int rows() const { return N; }
  __device__ int row_of(int r) const { return r; }
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

// P_hat(u + k) for u in U, k in E: read with periodic indexing.  u + k lies
// within 3r of the darkfield support's centre and P within r of it, so a
// wrapped position (off by a multiple of N > 4r) never falls in P, where
// P_hat is nonzero: the periodic read equals the bounded one.
__device__ __forceinline__ c64 phat_at(const c64 *phat, int n, int ky, int kx) {
  return phat[fft_pos(ky, n) * n + fft_pos(kx, n)];
}

// Gram of the darkfield system in 32 x 32 blocks (I >= J) of the N_u x N_u
// Hermitian matrix, one wavefront per block: lane (ty, tx) = (lane / 8,
// lane % 8) holds rows ty + 8 i and columns tx + 8 j, so the lanes reading one
// LDS row read consecutive elements (no bank conflicts).
//
// A product P_hat(u + k) conj(P_hat(u' + k)) is nonzero only when both u + k
// and u' + k fall in P, so the E-sum is sparse.  Small blocks and chunks of
// kEChunk (2) excluded k follow that sparsity: only the chunks whose products
// can be nonzero for both blocks (plan masks) are visited, in ascending order,
// walking the mask words with wave-uniform state.  The operands of the next
// chunk are gathered into registers while the current chunk is multiplied
// from LDS.  A diagonal block has one operand and is formed whole (its upper
// half is not read by the Cholesky).
constexpr int kGramKC = kEChunk;
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
  __shared__ c64 sA[kGramKC][kGramUB];
  __shared__ c64 sB[kGramKC][kGramUB];
  __shared__ uint32_t su[2][kGramUB];
  const int lane = threadIdx.x;
  const int ty = lane >> 3, tx = lane & 7;
  if (lane < kGramUB) {
    const int ui = I * kGramUB + lane, uj = J * kGramUB + lane;
    su[0][lane] = ui < s.nu ? s.u[ui] : 0x7fff7fffu;  // padding: outside every support
    su[1][lane] = uj < s.nu ? s.u[uj] : 0x7fff7fffu;
  }
  // live chunks in ascending order, walked with wave-uniform state
  const uint64_t *mi = s.gmask + (int64_t)I * s.nwe, *mj = s.gmask + (int64_t)J * s.nwe;
  int mw = 0;
  uint64_t bits = s.nwe > 0 ? (mi[0] & mj[0]) : 0;
  auto next_chunk = [&]() -> int {
    while (bits == 0) {
      if (++mw >= s.nwe) return -1;
      bits = mi[mw] & mj[mw];
    }
    const int c = mw * 64 + __builtin_ctzll(bits);
    bits &= bits - 1;
    return c;
  };
  c64 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  __syncthreads();
  constexpr int NEL = kGramKC * kGramUB, PER = (NEL + 63) / 64;
  c64 pa[PER], pb[PER];
  auto gather = [&](int chunk) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = lane + m * 64;
      const int kk = e / kGramUB, uu = e % kGramUB;
      const int k = chunk * kGramKC + kk;
      pa[m] = make_double2(0.0, 0.0);
      pb[m] = make_double2(0.0, 0.0);
      if ((NEL % 64 == 0 || e < NEL) && k < s.ne) {
        const uint32_t kw = s.e[k];
        const int ky = kunpack_y(kw), kx = kunpack_x(kw);
        const uint32_t wa = su[0][uu], wb = su[1][uu];
        if (wa != 0x7fff7fffu) pa[m] = phat_at(phat, a.n, kunpack_y(wa) + ky, kunpack_x(wa) + kx);
        if (diag)
          pb[m] = pa[m];
        else if (wb != 0x7fff7fffu)
          pb[m] = phat_at(phat, a.n, kunpack_y(wb) + ky, kunpack_x(wb) + kx);
      }
    }
  };
  int cur = next_chunk();
  if (cur >= 0) gather(cur);
  while (cur >= 0) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = lane + m * 64;
      if (NEL % 64 == 0 || e < NEL) {
        sA[e / kGramUB][e % kGramUB] = pa[m];
        sB[e / kGramUB][e % kGramUB] = pb[m];
      }
    }
    __syncthreads();
    const int nxt = next_chunk();
    if (nxt >= 0) gather(nxt);
#pragma unroll 4
    for (int kk = 0; kk < kGramKC; ++kk) {
      c64 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[kk][ty + 8 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[kk][tx + 8 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {  // acc += a * conj(b)
          acc[i][j].x = fma(av[i].x, bv[j].x, fma(av[i].y, bv[j].y, acc[i][j].x));
          acc[i][j].y = fma(av[i].y, bv[j].x, fma(-av[i].x, bv[j].y, acc[i][j].y));
        }
    }
    __syncthreads();
    cur = nxt;
  }
  // G[r][c] = fft2(|P|^2)(u_r - u_c) / N^2 - acc / N^4
  const double n2 = (double)a.n * a.n, inv2 = 1.0 / n2, inv4 = inv2 * inv2;
  const c64 *fpp = a.at<c64>(t, a.lay.fpp);
  c64 *G = a.at<c64>(t, a.lay.gram);
  const int ld = a.nu_pad;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = I * kGramUB + ty + 8 * i;
    if (r >= s.nu) continue;
    const uint32_t wr = su[0][ty + 8 * i];
    const int ry = kunpack_y(wr), rx = kunpack_x(wr);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = J * kGramUB + tx + 8 * j;
      if (c >= s.nu) continue;
      const uint32_t wc = su[1][tx + 8 * j];
      const int dy = ry - kunpack_y(wc), dx = rx - kunpack_x(wc);
      const c64 tv = fpp[fft_pos(dy, a.n) * a.n + fft_pos(dx, a.n)];
      G[(int64_t)r * ld + c] = make_double2(tv.x * inv2 - acc[i][j].x * inv4,
                                            tv.y * inv2 - acc[i][j].y * inv4);
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
