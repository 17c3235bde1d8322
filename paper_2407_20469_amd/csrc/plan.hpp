// Host-side geometry plan: every index set of the method depends only on the
// tile size, the pupil radius and the illumination vectors, so it is built
// once per geometry class on the host and reused for every tile of the class.
#pragma once

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/apic.h"

namespace apic {

constexpr int kMaxBf = 32;
constexpr int kMaxDf = 64;
constexpr int kMaxImg = kMaxBf + kMaxDf;
constexpr int kNumJ = 12;           // Noll 4..15 carried by the pupil solve
constexpr int kNumFeat = 32;        // 8 pair-angle bins x 4 radial bands
constexpr int kAbEntries = 78 + 12 + 2 + kNumFeat;  // A upper, b, sbb, sw, cells
constexpr int kAbChunk = 2048;      // pupil rows per workgroup
constexpr int kGramBlock = 64;      // gram storage / Cholesky padding granularity
constexpr int kGramUB = 32;         // unknowns per gram block
constexpr int kGramHB = 16;         // unknowns per half-block (block-sparsity masks)
constexpr int kEChunk = 1;          // E rows per bit of the gram's block masks
constexpr int kPixMax = 7936;       // pupil pixels of the one-workgroup pixel solve (LDS bound)
constexpr int kPixIdxMax = 65536;   // pupil pixels of the pixel solve (16-bit pixel indices)
// Coarse-to-fine continuation of the pupil solve: bands |K| <= f r for these
// f, each band used when it holds at least kMinBandRows rows.
constexpr int kPupilBands = 6;
constexpr double kPupilBandFrac[kPupilBands] = {0.05, 0.1, 0.2, 0.4, 0.8, 1.6};
constexpr int kMinBandRows = 32;
// Ridge of the band solves (relative, mu tr(A) / 12): keeps each band's
// increment near zero in the directions its low-|K| rows hardly constrain.
constexpr double kPupilBandRidge = 0.1;
constexpr uint32_t kPlanMagic = 0x41504943u;  // "APIC"

// Signed (ky, kx) packed in one word: low half ky, high half kx (int16 each).
inline uint32_t pack_k(int ky, int kx) {
  return (uint32_t)(uint16_t)(int16_t)ky | ((uint32_t)(uint16_t)(int16_t)kx << 16);
}
inline int unpack_ky(uint32_t w) { return (int)(int16_t)(uint16_t)(w & 0xffffu); }
inline int unpack_kx(uint32_t w) { return (int)(int16_t)(uint16_t)(w >> 16); }

// One darkfield image's index sets (Eq. 11-13).
struct DfStep {
  int32_t kx = 0, ky = 0;
  int32_t nu = 0, np = 0, m = 0, ne = 0;
  int64_t off_u = 0, off_p = 0, off_q = 0, off_e = 0;  // into GeomPlan::coords
  // Block-sparsity masks (into GeomPlan::masks): for each block of kGramUB
  // unknowns, one bit per chunk of kEChunk rows of E that holds a k with
  // u + k in P for some u of the block.  Then the membership bitmap of Q over
  // the N x N grid (FFT order, bit y N + x).
  int32_t nwe = 0;                   // 64-bit words per block of kGramUB unknowns
  int64_t off_gmask = 0, off_qbits = 0;
  int64_t gram_live = 0;             // live (quadrant of an I >= J block pair, E row) pairs
  int64_t gram_live_diag = 0;        // the I = J part of gram_live
  // Signed row spans (ky) of D = P + U (the shifted pupil's points: where
  // P_hat and the unknowns lie) and of Q (where b is nonzero); the FFT passes
  // of P_hat and of the right-hand side skip the rows outside them.
  int32_t d_lo = 0, d_hi = -1, q_lo = 0, q_hi = -1;
  // Signed row span where z = fft2(|P|^2 + i I_j) is read: the rows of Q and
  // of -Q (right-hand side) and the row differences of U (the gram's Toeplitz
  // term at u - u' and u' - u).
  int32_t z_lo = 0, z_hi = -1;
};

// Per-tile workspace layout (byte offsets from the tile's base).
struct TileLayout {
  int64_t stack = 0, ohat = 0, phat = 0, dtmp = 0, fpp = 0, ptil = 0, vec = 0,
          gram = 0, linv = 0, part = 0, sums = 0, coef = 0, sur = 0, seed = 0, eps = 0, stride = 0;
};

struct GeomPlan {
  int n = 0, f = 1, nf = 0, n_bf = 0, n_df = 0;
  double dx = 0, lam = 0, na = 0, r = 0;
  int64_t r2 = 0;                    // floor(r * r): Circ(k) <=> kx^2 + ky^2 <= r2
  int64_t n_disk = 0;                // grid points inside Circ
  double ridge_pupil = 1e-9, ridge_df = 1e-4, log_floor_rel = 1e-6;
  std::vector<int32_t> kbf, kdf;     // (kx, ky) pairs
  // pupil rows (Eq. 8-10): one row per (pair, K) with K in S_il, K != 0,
  // sorted by the first continuation band that holds them (stable, so pairs
  // stay in order inside a band)
  int n_pairs = 0, n_rows = 0, n_chunks = 0;
  std::vector<uint32_t> row_il;      // i | l << 8 | feature cell << 16
  std::vector<uint32_t> row_k;       // packed K
  // row counts of the continuation's band passes (rows with |K| <= f r, for
  // the bands holding at least kMinBandRows); empty for the single pass
  bool pupil_bands = true;
  std::vector<int> band_rows;
  // the same rows in pair order (pairs i < l, then K raster): the row order
  // of the pixel-domain solve, whose passes sum each pair's rows in one run
  std::vector<uint32_t> prow_il, prow_k;
  // pupil pixels (Eq. 10 with one unknown per pixel), raster order over the
  // disk (ky ascending, then kx): built when n_pix <= kPixIdxMax.  pix_tab holds
  // the pixels' packed k, then per pupil row (in pair order, prow_*) the pixel
  // indices of K + K_i (low half) and K + K_l (high half), then the pixel index of each
  // NA-matched k_i.  pix_ginv is the inverse Gram matrix of Noll Z_1..Z_15 over
  // the pixels (15 x 15, row-major), for the Zernike summary.
  int n_pix = 0;
  bool pix_ok = false;
  std::vector<uint32_t> pix_tab;
  std::vector<double> pix_ginv;
  // darkfield (Eq. 11-13)
  std::vector<int16_t> known_at;     // N*N in FFT order: -1 brightfield, j solved at step j,
                                     // 32767 never known
  std::vector<DfStep> steps;
  std::vector<uint32_t> coords;      // packed U, P, Q, E lists of all steps
  std::vector<uint64_t> masks;       // block-sparsity masks of all steps
  int64_t gram_chunk_pairs = 0;      // live (block pair, E chunk) triples, all steps
  int nu_max = 0, np_max = 0, m_max = 0, ne_max = 0, n_active = 0, nu_pad = 0;
  TileLayout lay;
  // device copies (owned; filled by upload)
  void *d_row_il = nullptr, *d_row_k = nullptr, *d_known_at = nullptr, *d_coords = nullptr,
       *d_masks = nullptr, *d_pix_tab = nullptr, *d_pix_ginv = nullptr, *d_prow_il = nullptr,
       *d_prow_k = nullptr;
};

// Build the host tables of one geometry; returns APIC_OK or an error code.
apic_status build_geom_plan(const apic_geometry &g, GeomPlan &out);

}  // namespace apic

struct apic_plan {
  uint32_t magic = apic::kPlanMagic;
  std::vector<apic::GeomPlan> geoms;
  int device = -1;
  bool uploaded = false;
};
