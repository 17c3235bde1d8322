// Geometry plan builder (host only).  Builds, for one geometry class, the
// index sets the kernels consume:
//   - pupil rows: every overlapping pair i < l and every K != 0 in the overlap
//     S_il of Eq. 8, with the surrogate feature cell of the row;
//   - darkfield steps: for each darkfield image in processing order the known
//     set P, the unknown set U, the linear region Q of Eq. 13 and the excluded
//     part E of P - U (used by the gram identity), plus the map of the step at
//     which each frequency became known.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace apic {

namespace {

bool is_pow2_size(int n) { return n == 64 || n == 128 || n == 256 || n == 512; }

inline int signed_of(int idx, int n) { return idx < n / 2 ? idx : idx - n; }

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// Sort key of a signed frequency (ky, kx): the s x s square it falls in
// (rows of squares, then squares along a row), then raster inside the square.
int64_t square_key(std::pair<int, int> k, int s) {
  const int y = k.first + 4096, x = k.second + 4096;  // non-negative
  return (((int64_t(y / s) * 8192 + x / s) * s + y % s) * s) + x % s;
}

// Pair-angle bin (8 bins over (0, pi]) of two illumination vectors.
int angle_bin(int kix, int kiy, int klx, int kly) {
  const double dot = double(kix) * klx + double(kiy) * kly;
  const double ni = std::sqrt(double(kix) * kix + double(kiy) * kiy);
  const double nl = std::sqrt(double(klx) * klx + double(kly) * kly);
  double c = dot / (ni * nl);
  c = std::min(1.0, std::max(-1.0, c));
  const double ang = std::acos(c);
  double b = std::ceil(ang / (M_PI / 8.0) - 1e-9) - 1.0;
  b = std::min(7.0, std::max(0.0, b));
  return int(b);
}

// Radial band (4 bands of |K| / (2r) over (0, 1]).
int radial_band(int ky, int kx, double r) {
  const double rho = std::hypot(double(kx), double(ky)) / (2.0 * r);
  double b = std::ceil(4.0 * rho - 1e-9) - 1.0;
  b = std::min(3.0, std::max(0.0, b));
  return int(b);
}

}  // namespace

// Orthonormal Noll Z_1..Z_15 at (X, Y) = k / r, Cartesian form (host, double).
static void zernike15_host(double X, double Y, double z[15]) {
  const double r2 = X * X + Y * Y;
  const double c2 = X * X - Y * Y, s2 = 2.0 * X * Y;
  const double c3 = X * c2 - Y * s2, s3 = X * s2 + Y * c2;
  const double c4 = X * c3 - Y * s3, s4 = X * s3 + Y * c3;
  const double k3 = std::sqrt(3.0), k5 = std::sqrt(5.0), k6 = std::sqrt(6.0), k8 = std::sqrt(8.0),
               k10 = std::sqrt(10.0);
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

// Pixel tables of the pixel-domain pupil solve (see GeomPlan).
static void build_pixel_tables(GeomPlan &p, int n_bf) {
  const int n = p.n, h = n / 2;
  std::vector<int32_t> at(size_t(n) * n, -1);  // centred layout
  std::vector<uint32_t> pix;
  for (int ky = -h; ky < h; ++ky)
    for (int kx = -h; kx < h; ++kx)
      if (int64_t(kx) * kx + int64_t(ky) * ky <= p.r2) {
        at[size_t(ky + h) * n + (kx + h)] = int32_t(pix.size());
        pix.push_back(pack_k(ky, kx));
      }
  p.n_pix = int(pix.size());
  p.pix_ok = p.n_pix <= kPixIdxMax && p.n_rows > 0;
  p.pix_tab.clear();
  p.pix_ginv.clear();
  if (!p.pix_ok) return;
  auto idx = [&](int ky, int kx) { return uint32_t(at[size_t(ky + h) * n + (kx + h)]); };
  p.pix_tab = pix;
  for (int rI = 0; rI < p.n_rows; ++rI) {
    const int i = p.prow_il[rI] & 0xff, l = (p.prow_il[rI] >> 8) & 0xff;
    const int Ky = unpack_ky(p.prow_k[rI]), Kx = unpack_kx(p.prow_k[rI]);
    const uint32_t a = idx(Ky + p.kbf[2 * i + 1], Kx + p.kbf[2 * i]);
    const uint32_t b = idx(Ky + p.kbf[2 * l + 1], Kx + p.kbf[2 * l]);
    p.pix_tab.push_back(a | (b << 16));
  }
  for (int i = 0; i < n_bf; ++i) p.pix_tab.push_back(idx(p.kbf[2 * i + 1], p.kbf[2 * i]));
  // Gram matrix of Z_1..Z_15 over the pixels and its inverse (Gauss-Jordan)
  double G[15][30] = {};
  for (uint32_t w : pix) {
    double z[15];
    zernike15_host(unpack_kx(w) / p.r, unpack_ky(w) / p.r, z);
    for (int a = 0; a < 15; ++a)
      for (int b = 0; b < 15; ++b) G[a][b] += z[a] * z[b];
  }
  for (int a = 0; a < 15; ++a) G[a][15 + a] = 1.0;
  for (int c = 0; c < 15; ++c) {
    int piv = c;
    for (int a = c + 1; a < 15; ++a)
      if (std::fabs(G[a][c]) > std::fabs(G[piv][c])) piv = a;
    if (piv != c)
      for (int b = 0; b < 30; ++b) std::swap(G[c][b], G[piv][b]);
    const double d = 1.0 / G[c][c];
    for (int b = 0; b < 30; ++b) G[c][b] *= d;
    for (int a = 0; a < 15; ++a) {
      if (a == c) continue;
      const double f = G[a][c];
      for (int b = 0; b < 30; ++b) G[a][b] -= f * G[c][b];
    }
  }
  for (int a = 0; a < 15; ++a)
    for (int b = 0; b < 15; ++b) p.pix_ginv.push_back(G[a][15 + b]);
}

apic_status build_geom_plan(const apic_geometry &g, GeomPlan &p) {
  if (!is_pow2_size(g.n)) return APIC_EUNSUPPORTED;
  if (g.upsample != 1 && g.upsample != 2) return APIC_EUNSUPPORTED;
  if (g.n * g.upsample > 1024) return APIC_EUNSUPPORTED;
  if (g.n_bf < 4 || g.n_bf > kMaxBf || g.n_df < 0 || g.n_df > kMaxDf) return APIC_EUNSUPPORTED;
  if (!g.k_bf || (g.n_df > 0 && !g.k_df)) return APIC_EINVAL;
  if (!(g.dx_um > 0) || !(g.wavelength_um > 0) || !(g.na_obj > 0)) return APIC_EINVAL;
  if (!(g.ridge_pupil >= 0) || !(g.ridge_darkfield >= 0) || !(g.log_floor_rel > 0))
    return APIC_EINVAL;
  if (g.pupil_bands != 0 && g.pupil_bands != 1) return APIC_EINVAL;

  const int n = g.n;
  p.n = n;
  p.f = g.upsample;
  p.nf = n * g.upsample;
  p.n_bf = g.n_bf;
  p.n_df = g.n_df;
  p.dx = g.dx_um;
  p.lam = g.wavelength_um;
  p.na = g.na_obj;
  p.r = g.na_obj * n * g.dx_um / g.wavelength_um;
  p.r2 = (int64_t)std::floor(p.r * p.r);
  p.n_disk = 0;
  for (int y = -n / 2; y < n / 2; ++y)
    for (int x = -n / 2; x < n / 2; ++x) p.n_disk += int64_t(x) * x + int64_t(y) * y <= p.r2;
  p.ridge_pupil = g.ridge_pupil;
  p.ridge_df = g.ridge_darkfield;
  p.log_floor_rel = g.log_floor_rel;
  if (p.r < 2.0) return APIC_EUNSUPPORTED;
  // C^H b is formed as a circular correlation on the N x N grid; it equals
  // the linear one when no u + k (u in U, k in Q: within 3r of the darkfield
  // support's centre) can alias onto P (within r of it), i.e. when 4r < N.
  if (4.0 * p.r >= n) return APIC_EUNSUPPORTED;
  p.kbf.assign(g.k_bf, g.k_bf + 2 * g.n_bf);
  p.kdf.assign(g.k_df ? g.k_df : g.k_bf, (g.k_df ? g.k_df : g.k_bf) + 2 * g.n_df);

  auto circ = [&](int ky, int kx) { return int64_t(kx) * kx + int64_t(ky) * ky <= p.r2; };
  // Every shifted support must stay inside the grid: |k| + r < N/2.
  for (int i = 0; i < g.n_bf + g.n_df; ++i) {
    const int kx = i < g.n_bf ? p.kbf[2 * i] : p.kdf[2 * (i - g.n_bf)];
    const int ky = i < g.n_bf ? p.kbf[2 * i + 1] : p.kdf[2 * (i - g.n_bf) + 1];
    const double mag = std::sqrt(double(kx) * kx + double(ky) * ky);
    if (mag + p.r >= n / 2 - 1) return APIC_EUNSUPPORTED;
    if (i < g.n_bf && !circ(ky, kx)) return APIC_EINVAL;  // NA-matched must sit in the pupil
  }

  // ---- pupil rows (Eq. 8-10)
  p.row_il.clear();
  p.row_k.clear();
  p.n_pairs = 0;
  for (int i = 0; i < g.n_bf; ++i) {
    const int kix = p.kbf[2 * i], kiy = p.kbf[2 * i + 1];
    for (int l = i + 1; l < g.n_bf; ++l) {
      const int klx = p.kbf[2 * l], kly = p.kbf[2 * l + 1];
      const int abin = angle_bin(kix, kiy, klx, kly);
      size_t before = p.row_k.size();
      for (int y = 0; y < n; ++y) {
        const int ky = signed_of(y, n);
        for (int x = 0; x < n; ++x) {
          const int kx = signed_of(x, n);
          if (ky == 0 && kx == 0) continue;
          if (!circ(ky + kiy, kx + kix) || !circ(ky + kly, kx + klx)) continue;
          const int cell = abin * 4 + radial_band(ky, kx, p.r);
          p.row_il.push_back(uint32_t(i) | (uint32_t(l) << 8) | (uint32_t(cell) << 16));
          p.row_k.push_back(pack_k(ky, kx));
        }
      }
      if (p.row_k.size() > before) ++p.n_pairs;
    }
  }
  p.n_rows = int(p.row_k.size());
  p.n_chunks = std::max(1, (p.n_rows + kAbChunk - 1) / kAbChunk);
  // band of each row: the first f with Kx^2 + Ky^2 <= (f r)^2, kPupilBands
  // if none; rows sorted by band (stable), band passes = prefixes; the pair
  // order is kept for the pixel-domain solve
  p.prow_il = p.row_il;
  p.prow_k = p.row_k;
  {
    std::vector<int> band(p.n_rows);
    std::vector<int64_t> count(kPupilBands + 1, 0);
    for (int rI = 0; rI < p.n_rows; ++rI) {
      const double ky = unpack_ky(p.row_k[rI]), kx = unpack_kx(p.row_k[rI]);
      const double k2 = kx * kx + ky * ky;
      int b = kPupilBands;
      for (int f = 0; f < kPupilBands; ++f) {
        const double km = kPupilBandFrac[f] * p.r;
        if (k2 <= km * km) {
          b = f;
          break;
        }
      }
      band[rI] = b;
      ++count[b];
    }
    std::vector<int> order(p.n_rows);
    for (int rI = 0; rI < p.n_rows; ++rI) order[rI] = rI;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return band[x] < band[y]; });
    std::vector<uint32_t> il(p.n_rows), kk(p.n_rows);
    for (int rI = 0; rI < p.n_rows; ++rI) {
      il[rI] = p.row_il[order[rI]];
      kk[rI] = p.row_k[order[rI]];
    }
    p.row_il.swap(il);
    p.row_k.swap(kk);
    p.pupil_bands = g.pupil_bands != 0;
    p.band_rows.clear();
    int64_t cum = 0;
    for (int f = 0; f < kPupilBands; ++f) {
      cum += count[f];
      if (p.pupil_bands && cum >= kMinBandRows) p.band_rows.push_back(int(cum));
    }
  }
  build_pixel_tables(p, g.n_bf);

  // ---- darkfield sets (Eq. 11-13)
  const int nn = n * n;
  p.known_at.assign(nn, int16_t(32767));
  std::vector<uint8_t> known(nn, 0);
  for (int y = 0; y < n; ++y)
    for (int x = 0; x < n; ++x) {
      const int ky = signed_of(y, n), kx = signed_of(x, n);
      for (int i = 0; i < g.n_bf; ++i)
        if (circ(ky + p.kbf[2 * i + 1], kx + p.kbf[2 * i])) {
          known[y * n + x] = 1;
          p.known_at[y * n + x] = -1;
          break;
        }
    }
  const int W = 2 * n + 1;  // difference grid over [-N, N]^2
  std::vector<uint8_t> mpu(size_t(W) * W), mex(size_t(W) * W);
  p.steps.assign(g.n_df, DfStep());
  p.coords.clear();
  p.masks.clear();
  p.gram_chunk_pairs = 0;
  p.nu_max = p.np_max = p.m_max = p.ne_max = p.n_active = 0;
  for (int j = 0; j < g.n_df; ++j) {
    DfStep &st = p.steps[j];
    st.kx = p.kdf[2 * j];
    st.ky = p.kdf[2 * j + 1];
    std::vector<uint32_t> U, P;
    std::vector<std::pair<int, int>> Uc, Pc;
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const int ky = signed_of(y, n), kx = signed_of(x, n);
        if (!circ(ky + st.ky, kx + st.kx)) continue;
        if (known[y * n + x]) {
          P.push_back(pack_k(ky, kx));
          Pc.emplace_back(ky, kx);
        } else {
          U.push_back(pack_k(ky, kx));
          Uc.emplace_back(ky, kx);
        }
      }
    // Unknowns in bands of equal distance to P, each band ordered by angle
    // around the support's centre (alternating direction from band to band).
    // A product of the gram's E-sum is nonzero only if u + k lands in P, i.e.
    // for unknowns near P; blocks of kGramUB unknowns that are thin across the
    // P border and long along it therefore meet few E chunks.  Distances come
    // from a two-pass chamfer transform (steps 1 and sqrt 2) on the grid.
    {
      std::vector<float> dist(size_t(nn), 1e30f);
      auto at = [&](int ky, int kx) -> float & { return dist[size_t(ky + n / 2) * n + (kx + n / 2)]; };
      for (auto &q : Pc) at(q.first, q.second) = 0.f;
      const float d1 = 1.f, d2 = 1.41421356f;
      for (int y = -n / 2; y < n / 2; ++y)
        for (int x = -n / 2; x < n / 2; ++x) {
          float &v = at(y, x);
          if (x > -n / 2) v = std::min(v, at(y, x - 1) + d1);
          if (y > -n / 2) {
            v = std::min(v, at(y - 1, x) + d1);
            if (x > -n / 2) v = std::min(v, at(y - 1, x - 1) + d2);
            if (x < n / 2 - 1) v = std::min(v, at(y - 1, x + 1) + d2);
          }
        }
      for (int y = n / 2 - 1; y >= -n / 2; --y)
        for (int x = n / 2 - 1; x >= -n / 2; --x) {
          float &v = at(y, x);
          if (x < n / 2 - 1) v = std::min(v, at(y, x + 1) + d1);
          if (y < n / 2 - 1) {
            v = std::min(v, at(y + 1, x) + d1);
            if (x < n / 2 - 1) v = std::min(v, at(y + 1, x + 1) + d2);
            if (x > -n / 2) v = std::min(v, at(y + 1, x - 1) + d2);
          }
        }
      // angle measured from the direction -k_j (away from the known centre), so
      // the unknown crescent does not straddle the +-pi cut
      const double kn = std::max(1e-9, std::sqrt(double(st.kx) * st.kx + double(st.ky) * st.ky));
      const double dx = -st.kx / kn, dy = -st.ky / kn;
      std::vector<std::pair<int, double>> key(U.size());
      for (size_t i = 0; i < U.size(); ++i) {
        const double ry = Uc[i].first + st.ky, rx = Uc[i].second + st.kx;  // from the centre -k_j
        const double ang = std::atan2(dx * ry - dy * rx, dx * rx + dy * ry);
        const int band = int(at(Uc[i].first, Uc[i].second) / 4.f);
        key[i] = {band, (band & 1) ? -ang : ang};
      }
      std::vector<int> ord(U.size());
      for (size_t i = 0; i < ord.size(); ++i) ord[i] = int(i);
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return key[a] < key[b]; });
      std::vector<uint32_t> U2(U.size());
      std::vector<std::pair<int, int>> Uc2(U.size());
      for (size_t i = 0; i < ord.size(); ++i) {
        U2[i] = U[ord[i]];
        Uc2[i] = Uc[ord[i]];
      }
      U.swap(U2);
      Uc.swap(Uc2);
    }
    st.nu = int(U.size());
    st.np = int(P.size());
    st.off_u = int64_t(p.coords.size());
    p.coords.insert(p.coords.end(), U.begin(), U.end());
    st.off_p = int64_t(p.coords.size());
    p.coords.insert(p.coords.end(), P.begin(), P.end());
    st.off_q = st.off_e = int64_t(p.coords.size());
    if (U.empty()) continue;
    std::fill(mpu.begin(), mpu.end(), 0);
    std::fill(mex.begin(), mex.end(), 0);
    for (auto &u : Uc) {
      for (auto &q : Pc) mpu[size_t(q.first - u.first + n) * W + (q.second - u.second + n)] = 1;
      for (auto &q : Uc) mex[size_t(q.first - u.first + n) * W + (q.second - u.second + n)] = 1;
    }
    for (auto &q : Pc)  // U - P: a - b with a in U, b in P
      for (auto &u : Uc) mex[size_t(u.first - q.first + n) * W + (u.second - q.second + n)] = 1;
    int64_t n_pu = 0;
    for (size_t i = 0; i < mpu.size(); ++i) n_pu += mpu[i];
    std::vector<uint32_t> Q, E;
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const int ky = signed_of(y, n), kx = signed_of(x, n);
        const size_t o = size_t(ky + n) * W + (kx + n);
        if (!mpu[o]) continue;
        (mex[o] ? E : Q).push_back(pack_k(ky, kx));
      }
    if (int64_t(Q.size() + E.size()) != n_pu) return APIC_EUNSUPPORTED;  // would wrap
    // excluded k in 2 x 2 squares: a chunk of 2 (half a square) is spatially compact
    std::stable_sort(E.begin(), E.end(), [&](uint32_t a, uint32_t b) {
      return square_key({unpack_ky(a), unpack_kx(a)}, 2) <
             square_key({unpack_ky(b), unpack_kx(b)}, 2);
    });
    st.m = int(Q.size());
    st.ne = int(E.size());
    {
      int dlo = n, dhi = -n, qlo = n, qhi = -n;
      for (auto &c : Pc) dlo = std::min(dlo, c.first), dhi = std::max(dhi, c.first);
      for (auto &c : Uc) dlo = std::min(dlo, c.first), dhi = std::max(dhi, c.first);
      for (uint32_t w : Q) qlo = std::min(qlo, unpack_ky(w)), qhi = std::max(qhi, unpack_ky(w));
      st.d_lo = dlo;  // U is not empty here
      st.d_hi = dhi;
      int ulo = n, uhi = -n;
      for (auto &c : Uc) ulo = std::min(ulo, c.first), uhi = std::max(uhi, c.first);
      st.z_lo = -(uhi - ulo);
      st.z_hi = uhi - ulo;
      if (!Q.empty()) {
        st.q_lo = qlo;
        st.q_hi = qhi;
        st.z_lo = std::min({st.z_lo, qlo, -qhi});
        st.z_hi = std::max({st.z_hi, qhi, -qlo});
      }
    }
    st.off_q = int64_t(p.coords.size());
    p.coords.insert(p.coords.end(), Q.begin(), Q.end());
    st.off_e = int64_t(p.coords.size());
    p.coords.insert(p.coords.end(), E.begin(), E.end());
    // block-sparsity masks: dilate P by each half-block (kGramHB unknowns);
    // a gram block (two halves) visits the k marked in either half, and
    // skips its 16 x 16 quadrants whose two halves do not both hold that k
    {
      std::vector<uint8_t> live(size_t(W) * W);
      const int nhb = (st.nu + kGramHB - 1) / kGramHB;
      const int nec = (st.ne + kEChunk - 1) / kEChunk;
      st.nwe = (nec + 63) / 64;
      st.off_gmask = int64_t(p.masks.size());
      p.masks.resize(p.masks.size() + size_t(nhb + 1) * st.nwe, 0);  // + an empty half
      for (int b = 0; b < nhb; ++b) {
        std::fill(live.begin(), live.end(), 0);
        for (int ui = b * kGramHB; ui < std::min(st.nu, (b + 1) * kGramHB); ++ui)
          for (auto &q : Pc)  // k with u + k in P: k = q - u
            live[size_t(q.first - Uc[ui].first + n) * W + (q.second - Uc[ui].second + n)] = 1;
        auto is_live = [&](uint32_t w) {
          return live[size_t(unpack_ky(w) + n) * W + (unpack_kx(w) + n)] != 0;
        };
        for (int e = 0; e < st.ne; ++e)
          if (is_live(E[e])) {
            const int c = e / kEChunk;
            p.masks[st.off_gmask + size_t(b) * st.nwe + c / 64] |= uint64_t(1) << (c % 64);
          }
      }
      // issued work: live (quadrant of a lower block pair, k) pairs
      const int nub = (st.nu + kGramUB - 1) / kGramUB;
      auto hm = [&](int h, int w) { return p.masks[st.off_gmask + size_t(h) * st.nwe + w]; };
      for (int I = 0; I < nub; ++I)
        for (int J = 0; J <= I; ++J)
          for (int w = 0; w < st.nwe; ++w) {
            int64_t c = 0;
            for (int hi = 0; hi < 2; ++hi)
              for (int hj = 0; hj < 2; ++hj)
                c += __builtin_popcountll(hm(2 * I + hi, w) & hm(2 * J + hj, w));
            st.gram_live += c;
            if (I == J) st.gram_live_diag += c;
          }
      p.gram_chunk_pairs += st.gram_live;
    }
    // Q membership over the grid
    st.off_qbits = int64_t(p.masks.size());
    p.masks.resize(p.masks.size() + size_t(nn + 63) / 64, 0);
    for (uint32_t w : Q) {
      const int y = (unpack_ky(w) + n) % n, x = (unpack_kx(w) + n) % n;
      const int pix = y * n + x;
      p.masks[st.off_qbits + pix / 64] |= uint64_t(1) << (pix % 64);
    }
    for (auto &u : Uc) {
      const int y = (u.first + n) % n, x = (u.second + n) % n;
      known[y * n + x] = 1;
      p.known_at[y * n + x] = int16_t(j);
    }
    ++p.n_active;
    p.nu_max = std::max(p.nu_max, st.nu);
    p.np_max = std::max(p.np_max, st.np);
    p.m_max = std::max(p.m_max, st.m);
    p.ne_max = std::max(p.ne_max, st.ne);
  }
  // one spare row: the Cholesky carries the right-hand side as row n
  p.nu_pad = (p.nu_max + 1 + kGramBlock - 1) / kGramBlock * kGramBlock;

  // ---- per-tile workspace layout
  TileLayout &L = p.lay;
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    int64_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const int64_t c32 = 8, c64 = 16;
  const int64_t stack_bytes = std::max<int64_t>(int64_t(p.n_bf) * nn * c32,
                                                int64_t(p.nf) * p.nf * c32);
  L.stack = take(stack_bytes);
  L.ohat = take(int64_t(nn) * c32);
  L.phat = take(int64_t(nn) * c64);
  L.dtmp = take(int64_t(nn) * c64);
  L.fpp = take(int64_t(nn) * c64);
  L.ptil = take(int64_t(nn) * c64);
  L.vec = take(int64_t(p.nu_pad) * c64);
  // the gram block also serves the pixel-domain pupil solve (a separate call):
  // per-row weights and phases (float) and two double vectors over the pixels
  // (the iterate and the residual); beyond the LDS bound also the search
  // direction, the operator's image and the per-tile iteration state
  const int64_t pix_vecs = p.n_pix > kPixMax ? 4 : 2;
  const int64_t pix_need =
      p.pix_ok ? 2 * align256(int64_t(p.n_rows) * 4) +
                     pix_vecs * align256(int64_t(p.n_pix) * 8) + (p.n_pix > kPixMax ? 256 : 0)
               : 0;
  L.gram = take(std::max<int64_t>(p.n_active ? int64_t(p.nu_pad) * p.nu_pad * c64 : 256, pix_need));
  L.linv = take(int64_t(p.nu_pad / kGramBlock) * kGramBlock * kGramBlock * c64);
  L.part = take(int64_t(p.n_chunks) * kAbEntries * 8);
  L.sums = take(128 * 8);
  L.coef = take((16 + kMaxImg) * 4);
  L.sur = take(16 * 4);
  L.seed = take(16 * 4);
  L.eps = take(kMaxImg * 4);
  L.stride = o;
  return APIC_OK;
}

}  // namespace apic
