// C ABI of the per-tile APIC reconstruction: plan lifecycle, workspace
// layout, and the enqueue sequences of the entry points declared in apic.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <complex>
#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/apic.h"
#include "common.hpp"
#include "fft.hpp"
#include "kernels_bf.hpp"
#include "kernels_df.hpp"
#include "kernels_pix.hpp"
#include "kernels_asm.hpp"
#include "kernels_rgb.hpp"
#include "chol.hpp"
#include "calib.hpp"
#include "rowspan.hpp"
#include "mlp.hpp"
#include "plan.hpp"

namespace apic {
namespace {

#define APIC_HIP(call)                        \
  do {                                        \
    if ((call) != hipSuccess) return APIC_EHIP; \
  } while (0)
#define APIC_LAUNCHED()                                 \
  do {                                                  \
    if (hipGetLastError() != hipSuccess) return APIC_EHIP; \
  } while (0)
#define APIC_CHECK(...)                     \
  do {                                      \
    const apic_status rc_ = (__VA_ARGS__);  \
    if (rc_ != APIC_OK) return rc_;         \
  } while (0)

// ------------------------------------------------------------ twiddles
std::mutex g_tw_mu;
bool g_tw_ready[64] = {};

apic_status ensure_twiddles() {
  int dev = 0;
  APIC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return APIC_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  if (g_tw_ready[dev]) return APIC_OK;
  std::vector<c32> t32(kTwTotal);
  std::vector<c64> t64(kTwTotal);
  for (int L = 64; L <= 1024; L *= 2)
    for (int t = 0; t < L; ++t) {
      // exp(-2 pi j t / L), angle reduced to the first octant for accuracy
      const long double ang = -2.0L * 3.14159265358979323846264338327950288L * t / L;
      const double c = (double)cosl(ang), s = (double)sinl(ang);
      t64[L - 64 + t] = make_double2(c, s);
      t32[L - 64 + t] = make_float2((float)c, (float)s);
    }
  APIC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_tw32), t32.data(), sizeof(c32) * kTwTotal));
  APIC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_tw64), t64.data(), sizeof(c64) * kTwTotal));
  g_tw_ready[dev] = true;
  return APIC_OK;
}

bool plan_ok(const apic_plan *p) { return p && p->magic == kPlanMagic && !p->geoms.empty(); }

// ------------------------------------------------------------ profiling
// Opt-in: HIP events recorded on the launch stream around each kernel group,
// with the group's algorithmic work (flops or bytes) per launch.
struct ProfEntry {
  hipEvent_t e0, e1;
  double work;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfEntry> g_prof[APIC_PROF_GROUPS];

struct ProfScope {
  int id;
  double work;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ProfScope(int id_, double work_, hipStream_t st_) : id(id_), work(work_), st(st_) {
    if (!g_prof_on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return;
    (void)hipEventRecord(e0, st);
  }
  ~ProfScope() {
    if (!e0 || !e1) return;
    (void)hipEventRecord(e1, st);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof[id].push_back({e0, e1, work});
  }
};

void prof_clear() {
  for (auto &v : g_prof) {
    for (auto &e : v) {
      (void)hipEventDestroy(e.e0);
      (void)hipEventDestroy(e.e1);
    }
    v.clear();
  }
}

template <class T> apic_status upload_vec(const std::vector<T> &v, void **dst) {
  const size_t bytes = std::max<size_t>(sizeof(T), v.size() * sizeof(T));
  APIC_HIP(hipMalloc(dst, bytes));
  if (!v.empty()) APIC_HIP(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return APIC_OK;
}

void free_geom(GeomPlan &g) {
  void **ptrs[] = {&g.d_row_il, &g.d_row_k, &g.d_known_at, &g.d_coords, &g.d_masks,
                   &g.d_pix_tab, &g.d_pix_ginv, &g.d_prow_il, &g.d_prow_k};
  for (void **p : ptrs)
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
}

// ------------------------------------------------------------ call setup
struct ClassRun {
  int geom = 0;
  bool skip_df = false;
  bool affine = false;   // offsets and batch indices are affine in the class index
  std::vector<int64_t> img_off, out_off;
  std::vector<int32_t> gidx, flags;
  int64_t desc_at = 0;   // byte offset of this class's descriptor arrays
  int64_t ws_at = 0;     // byte offset of tile 0's block
};

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

// Group tiles by (geometry, skip-darkfield) and lay out the workspace:
// descriptor arrays first, then one block per tile.
apic_status layout_call(const apic_plan *p, int32_t n_tiles, const apic_tile_desc *tiles,
                        std::vector<ClassRun> &runs, int64_t &total) {
  if (n_tiles < 0) return APIC_EINVAL;
  if (n_tiles > 0 && !tiles) return APIC_EINVAL;
  runs.clear();
  const int ng = (int)p->geoms.size();
  std::vector<int> slot(2 * ng, -1);
  for (int t = 0; t < n_tiles; ++t) {
    const apic_tile_desc &d = tiles[t];
    if (d.geom < 0 || d.geom >= ng) return APIC_EINVAL;
    if (d.image_offset < 0 || d.field_offset < 0) return APIC_EINVAL;
    const int key = 2 * d.geom + ((d.flags & APIC_TILE_SKIP_DARKFIELD) ? 1 : 0);
    if (slot[key] < 0) {
      slot[key] = (int)runs.size();
      runs.emplace_back();
      runs.back().geom = d.geom;
      runs.back().skip_df = (key & 1) != 0;
    }
    ClassRun &r = runs[slot[key]];
    r.img_off.push_back(d.image_offset);
    r.out_off.push_back(d.field_offset);
    r.gidx.push_back(t);
    r.flags.push_back(d.flags);
  }
  for (ClassRun &r : runs) {
    const size_t T = r.gidx.size();
    r.affine = true;
    for (size_t t = 2; t < T && r.affine; ++t)
      r.affine = r.img_off[t] - r.img_off[t - 1] == r.img_off[1] - r.img_off[0] &&
                 r.out_off[t] - r.out_off[t - 1] == r.out_off[1] - r.out_off[0] &&
                 r.gidx[t] - r.gidx[t - 1] == r.gidx[1] - r.gidx[0];
  }
  int64_t o = 0;
  for (ClassRun &r : runs) {
    r.desc_at = o;
    const int64_t T = (int64_t)r.gidx.size();
    o = align256(o + T * (8 + 8 + 4 + 4));
  }
  for (ClassRun &r : runs) {
    r.ws_at = o;
    o += (int64_t)r.gidx.size() * p->geoms[r.geom].lay.stride;
  }
  total = std::max<int64_t>(o, 256);
  return APIC_OK;
}

ClassArgs make_args(const apic_plan *p, const ClassRun &r, const float *images, char *ws,
                    uint32_t *status, const char *desc_base = nullptr) {
  const GeomPlan &g = p->geoms[r.geom];
  ClassArgs a;
  memset(&a, 0, sizeof(a));
  a.n = g.n;
  a.nf = g.nf;
  a.n_bf = g.n_bf;
  a.n_df = g.n_df;
  a.n_img = g.n_bf + g.n_df;
  a.T = (int)r.gidx.size();
  a.r2 = (int)g.r2;
  a.r = (float)g.r;
  a.inv_r = (float)(1.0 / g.r);
  a.r_d = g.r;
  a.log_floor_rel = (float)g.log_floor_rel;
  a.n_rows = g.n_rows;
  a.n_chunks = g.n_chunks;
  a.n_band = (int)g.band_rows.size();
  for (int b = 0; b < a.n_band; ++b) a.band_rows[b] = g.band_rows[b];
  a.nu_pad = g.nu_pad;
  a.ridge_pupil = g.ridge_pupil;
  a.ridge_df = g.ridge_df;
  for (int i = 0; i < g.n_bf; ++i) {
    a.kx[i] = g.kbf[2 * i];
    a.ky[i] = g.kbf[2 * i + 1];
  }
  for (int j = 0; j < g.n_df; ++j) {
    a.kx[g.n_bf + j] = g.kdf[2 * j];
    a.ky[g.n_bf + j] = g.kdf[2 * j + 1];
  }
  a.images = images;
  const int64_t T = a.T;
  const char *d = (desc_base ? desc_base : ws) + r.desc_at;
  a.affine = r.affine ? 1 : 0;
  a.img0 = r.img_off[0];
  a.out0 = r.out_off[0];
  a.g0 = r.gidx[0];
  a.img_step = T > 1 ? r.img_off[1] - r.img_off[0] : 0;
  a.out_step = T > 1 ? r.out_off[1] - r.out_off[0] : 0;
  a.g_step = T > 1 ? r.gidx[1] - r.gidx[0] : 0;
  a.d_img_off = reinterpret_cast<const int64_t *>(d);
  a.d_out_off = reinterpret_cast<const int64_t *>(d + 8 * T);
  a.d_gidx = reinterpret_cast<const int32_t *>(d + 16 * T);
  a.ws = ws + r.ws_at;
  a.stride = g.lay.stride;
  a.lay = g.lay;
  a.status = status;
  a.row_il = (const uint32_t *)g.d_row_il;
  a.row_k = (const uint32_t *)g.d_row_k;
  a.known_at = (const int16_t *)g.d_known_at;
  a.coords = (const uint32_t *)g.d_coords;
  a.masks = (const uint64_t *)g.d_masks;
  a.n_pix = g.pix_ok ? g.n_pix : 0;
  a.pix_tab = (const uint32_t *)g.d_pix_tab;
  a.pix_ginv = (const double *)g.d_pix_ginv;
  return a;
}

// Irregular descriptor lists go to the workspace with a blocking copy, after
// the stream has drained (earlier work on it may still read that region).
apic_status upload_descriptors(const std::vector<ClassRun> &runs, char *ws, hipStream_t st) {
  bool synced = false;
  for (const ClassRun &r : runs) {
    if (r.affine) continue;
    if (!synced) {
      APIC_HIP(hipStreamSynchronize(st));
      synced = true;
    }
    const int64_t T = (int64_t)r.gidx.size();
    std::vector<char> buf(T * 24);
    memcpy(buf.data(), r.img_off.data(), 8 * T);
    memcpy(buf.data() + 8 * T, r.out_off.data(), 8 * T);
    memcpy(buf.data() + 16 * T, r.gidx.data(), 4 * T);
    memcpy(buf.data() + 20 * T, r.flags.data(), 4 * T);
    APIC_HIP(hipMemcpy(ws + r.desc_at, buf.data(), buf.size(), hipMemcpyHostToDevice));
  }
  return APIC_OK;
}

__global__ void k_fill_u32(uint32_t *p, int n, uint32_t v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_status_or_all(ClassArgs a, uint32_t bits) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t < a.T) status_or(a, t, bits);
}
// Copy a caller spectrum (complex N x N at out_off) into / out of O_hat.
__global__ void k_spec_copy(ClassArgs a, float *spec, int to_ohat) {
  const int nn = a.n * a.n;
  const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (int64_t)a.T * nn) return;
  const int t = (int)(gid / nn), pix = (int)(gid % nn);
  c32 *s = reinterpret_cast<c32 *>(spec) + a.out_off(t) + pix;
  c32 *o = a.at<c32>(t, a.lay.ohat) + pix;
  if (to_ohat) *o = *s;
  else *s = *o;
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// ------------------------------------------------------------ stage runners
// A column pass of the class with its panel variant (a.fft_var).
template <class C, int L, class Op>
apic_status launch_cols(const ClassArgs &a, int arrays, const Op &op, hipStream_t st) {
  if (a.fft_var == 1) {
    constexpr int NS = ColShapeAlt<C, L>::NSEQ;
    hipLaunchKernelGGL((k_cols<C, L, Op, NS>), dim3(col_blocks<C, L, NS>(arrays)),
                       dim3(kFftThreads), 0, st, op);
  } else {
    hipLaunchKernelGGL((k_cols<C, L, Op>), dim3(col_blocks<C, L>(arrays)), dim3(kFftThreads), 0,
                       st, op);
  }
  APIC_LAUNCHED();
  return APIC_OK;
}

template <int N> apic_status run_kk(const ClassArgs &a, c32 *kk_out, hipStream_t st) {
  const int arrays = a.T * a.n_bf;
  // bytes: image read twice (stats, pass 1), 4 complex64 read+write passes minus pass-1 read
  ProfScope ps(APIC_PROF_KK, (double)arrays * N * N * (4.0 + 4.0 + 8.0 * 7.0), st);
  hipLaunchKernelGGL(k_image_stats, dim3(arrays), dim3(256), 0, st, a);
  APIC_LAUNCHED();
  hipLaunchKernelGGL((k_rows<c32, N, OpKK1<N>>), dim3(row_blocks<c32, N>(arrays, N)),
                     dim3(kFftThreads), 0, st, OpKK1<N>{a});
  APIC_LAUNCHED();
  APIC_CHECK(launch_cols<c32, N>(a, arrays, OpKK2<N>{a}, st));
  hipLaunchKernelGGL((k_rows<c32, N, OpKK3<N>>), dim3(row_blocks<c32, N>(arrays, N)),
                     dim3(kFftThreads), 0, st, OpKK3<N>{a});
  APIC_LAUNCHED();
  APIC_CHECK(launch_cols<c32, N>(a, arrays, OpKK4<N>{a, kk_out}, st));
  return APIC_OK;
}

// One pass of Eq. 8-10 over the first ab.n_rows rows: partial sums, their
// fixed-order reduction, and (unless sums_only) the 12x12 solve.
apic_status pupil_pass(const ClassArgs &ab, const float *caller_seed, int seed_src, int final_pass,
                       bool sums_only, float *zout, float *diag, float *feat, hipStream_t st) {
  hipLaunchKernelGGL(k_pupil_partial, dim3(ab.T * ab.n_chunks), dim3(256), 0, st, ab, caller_seed,
                     seed_src);
  APIC_LAUNCHED();
  hipLaunchKernelGGL(k_pupil_reduce, dim3(ab.T), dim3(128), 0, st, ab);
  APIC_LAUNCHED();
  if (sums_only) return APIC_OK;
  hipLaunchKernelGGL(k_pupil_solve, dim3(blocks_for(ab.T, 64)), dim3(64), 0, st, ab, caller_seed,
                     seed_src, final_pass, zout, diag, feat);
  APIC_LAUNCHED();
  return APIC_OK;
}

// A band pass of the continuation: the first `rows` of the class's sorted
// pupil rows, solved with the band ridge.
ClassArgs band_args(const ClassArgs &a, int rows) {
  ClassArgs ab = a;
  ab.n_rows = rows;
  ab.n_chunks = std::max(1, (rows + kAbChunk - 1) / kAbChunk);
  ab.ridge_pupil = kPupilBandRidge;
  return ab;
}

// Eq. 8-10 for every tile of the class.  With a caller's seed: one seeded
// pass.  Otherwise the coarse-to-fine continuation: each band pass solves on
// the rows with |K| <= f r, re-wrapped about the previous band's solution
// (kept in the tile's seed block), and the final pass over every row is
// seeded by the last band.  *final_src receives the seed source of the final
// pass (its sums are re-wrapped about that seed).
apic_status run_pupil(const ClassArgs &a, const float *caller_seed, float *zout, float *diag,
                      float *feat, int *final_src, hipStream_t st) {
  int64_t rows = a.n_rows;
  if (!caller_seed)
    for (int b = 0; b < a.n_band; ++b) rows += a.band_rows[b];
  ProfScope ps(APIC_PROF_PUPIL, (double)a.T * rows * 16.0, st);  // two complex64 reads per row
  int src = caller_seed ? kSeedCaller : kSeedNone;
  if (!caller_seed) {
    for (int b = 0; b < a.n_band; ++b) {
      apic_status rc = pupil_pass(band_args(a, a.band_rows[b]), nullptr,
                                  b == 0 ? kSeedNone : kSeedBand, 0, false, nullptr, nullptr,
                                  nullptr, st);
      if (rc) return rc;
    }
    if (a.n_band > 0) src = kSeedBand;
  }
  if (final_src) *final_src = src;
  return pupil_pass(a, caller_seed, src, 1, false, zout, diag, feat, st);
}

// Pixel-domain solve beyond the LDS bound: CG with its vectors in the
// workspace, each iteration a many-workgroup row pass and a per-tile step;
// every kPixPoll iterations the host reads the number of live tiles and stops
// when none is left (the call blocks the host there).
constexpr int kPixPoll = 32;
static apic_status run_pixel_wide(const ClassArgs &a, double tol, int max_iter, float *phi_out,
                                  float *zout, int32_t *iters_out, hipStream_t st) {
  const int wgs = std::max(1, (a.n_rows + 4 * kPixgRowsPerWave - 1) / (4 * kPixgRowsPerWave));
  hipLaunchKernelGGL(k_pixg_clear, dim3(blocks_for(a.n_pix, 256), a.T), dim3(256), 0, st, a);
  APIC_LAUNCHED();
  hipLaunchKernelGGL(k_pixg_apply, dim3((unsigned)(a.T * wgs)), dim3(256), 0, st, a, 1, wgs);
  APIC_LAUNCHED();
  hipLaunchKernelGGL(k_pixg_init, dim3(a.T), dim3(kPixThreads), 0, st, a, tol);
  APIC_LAUNCHED();
  const void *active_dev =
      a.ws + a.lay.gram + pixg_vec_off(a.n_rows, a.n_pix, 4) + offsetof(PixState, active);
  for (int it = 1; it <= max_iter; ++it) {
    hipLaunchKernelGGL(k_pixg_apply, dim3((unsigned)(a.T * wgs)), dim3(256), 0, st, a, 0, wgs);
    APIC_LAUNCHED();
    hipLaunchKernelGGL(k_pixg_step, dim3(a.T), dim3(kPixThreads), 0, st, a, max_iter);
    APIC_LAUNCHED();
    if (it % kPixPoll == 0 && it < max_iter) {
      hipLaunchKernelGGL(k_pixg_count, dim3(1), dim3(256), 0, st, a);
      APIC_LAUNCHED();
      int active = 0;
      if (hipMemcpyAsync(&active, active_dev, sizeof(int), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return APIC_EHIP;
      if (active == 0) break;
    }
  }
  hipLaunchKernelGGL(k_pixg_finish, dim3(a.T), dim3(kPixThreads), 0, st, a, phi_out, zout,
                     iters_out);
  APIC_LAUNCHED();
  return APIC_OK;
}

apic_status run_stitch(const ClassArgs &a, int64_t n_disk, float *spec_out, hipStream_t st) {
  // bytes: each KK spectrum read on its support, O_hat written
  ProfScope ps(APIC_PROF_STITCH, (double)a.T * 8.0 * ((double)a.n_bf * n_disk + a.n * a.n), st);
  hipLaunchKernelGGL(k_coef_led_phase, dim3(blocks_for(a.T, 64)), dim3(64), 0, st, a);
  APIC_LAUNCHED();
  hipLaunchKernelGGL(k_pupil_phasor, dim3(blocks_for((int64_t)a.T * a.n * a.n, 256)), dim3(256), 0,
                     st, a);
  APIC_LAUNCHED();
  hipLaunchKernelGGL(k_stitch, dim3(blocks_for((int64_t)a.T * a.n * a.n, 256)), dim3(256), 0, st,
                     a, spec_out);
  APIC_LAUNCHED();
  return APIC_OK;
}

template <int N>
apic_status run_darkfield(const apic_plan *p, const ClassRun &r, const ClassArgs &a,
                          hipStream_t st) {
  const GeomPlan &g = p->geoms[r.geom];
  bool skipped = false;
  constexpr int RW = RowShape<c64, N>::ROWS;
  // rows of P_hat that may be nonzero: all of them before the first image
  // (the workspace holds an earlier call's data), then the last image's D
  RowRange prev;
  prev.y0 = 0;
  prev.n = N;
  for (int j = 0; j < g.n_df; ++j) {
    const DfStep &d = g.steps[j];
    if (d.nu == 0) {
      skipped = true;
      continue;
    }
    StepArgs s;
    s.j = j;
    s.img = g.n_bf + j;
    s.kx = d.kx;
    s.ky = d.ky;
    s.nu = d.nu;
    s.np = d.np;
    s.m = d.m;
    s.ne = d.ne;
    s.u = a.coords + d.off_u;
    s.p = a.coords + d.off_p;
    s.q = a.coords + d.off_q;
    s.e = a.coords + d.off_e;
    s.gmask = a.masks + d.off_gmask;
    s.nwe = d.nwe;
    s.qbits = a.masks + d.off_qbits;
    // row ranges of the pruned passes, whole row-pass workgroups
    const RowRange rd = rows_of_span(d.d_lo, d.d_hi, N, RW);
    const RowRange rq = rows_of_span(d.q_lo, d.q_hi, N, RW);
    const RowRange rz = rows_of_span(d.z_lo, d.z_hi, N, RW);
    // P_hat's pass: this image's D and the previous one's, which it clears
    const RowRange rp = cyclic_hull(prev, rd, N, RW);
    prev = rd;
    s.dy0 = rd.y0;
    s.dn = rd.n;
    s.qy0 = rq.y0;
    s.qn = rq.n;
    s.zy0 = rz.y0;
    s.zn = rz.n;
    s.py0 = rp.y0;
    s.pn = rp.n;
    const int64_t pix = (int64_t)a.T * N * N;
    const double nu = d.nu, T = a.T, fd = (double)s.dn / N, fq = (double)s.qn / N,
                 fz = (double)s.zn / N, fp = (double)s.pn / N;
    {
      // three FP64 passes: P_hat formed in the first (read O_hat 8 B, write
      // P_hat 16 B on its rows, write 16 B on the rows of D), then read (rows
      // of D), write P, read the image (20 B + 16 B on D + 16 B on the rows
      // where z is read), then read, write on those rows (32 B)
      ProfScope ps(APIC_PROF_DF_FFT, (double)pix * (20.0 + 24.0 * fp + 32.0 * fd + 48.0 * fz),
                   st);
      hipLaunchKernelGGL((k_rows<c64, N, OpP1<N>>), dim3(row_blocks<c64, N>(a.T, s.pn)),
                         dim3(kFftThreads), 0, st, OpP1<N>{a, s});
      APIC_LAUNCHED();
      APIC_CHECK(launch_cols<c64, N>(a, a.T, OpP2<N>{a, s}, st));
      hipLaunchKernelGGL((k_rows<c64, N, OpP3<N>>), dim3(row_blocks<c64, N>(a.T, s.zn)),
                         dim3(kFftThreads), 0, st, OpP3<N>{a, s});
      APIC_LAUNCHED();
    }
    {
      // three FP64 passes: on the rows of Q the Q bitmap, z(k) and z(-k) on
      // Q, write (16 B per pixel + 32 B per Q point); read (rows of Q), read
      // P, write (rows of D) (16 B + 16 B on Q + 16 B on D); read, write on
      // the rows of D (32 B); then N_u gathers (32 B each)
      ProfScope ps(APIC_PROF_DF_RHS,
                   (double)pix * (16.125 * fq + 16.0 + 16.0 * fq + 48.0 * fd) +
                       T * (32.0 * d.m + 32.0 * nu),
                   st);
      hipLaunchKernelGGL((k_rows<c64, N, OpR1<N>>), dim3(row_blocks<c64, N>(a.T, s.qn)),
                         dim3(kFftThreads), 0, st, OpR1<N>{a, s});
      APIC_LAUNCHED();
      APIC_CHECK(launch_cols<c64, N>(a, a.T, OpR2<N>{a, s}, st));
      hipLaunchKernelGGL((k_rows<c64, N, OpR3<N>>), dim3(row_blocks<c64, N>(a.T, s.dn)),
                         dim3(kFftThreads), 0, st, OpR3<N>{a, s});
      APIC_LAUNCHED();
      hipLaunchKernelGGL(k_df_rhs_gather, dim3(blocks_for(d.nu, 256), a.T), dim3(256), 0, st,
                         a, s);
      APIC_LAUNCHED();
    }
    {
      // algorithmic flops of the gram: 8 per complex MAC over the E-sum of the
      // Hermitian lower triangle
      ProfScope ps(APIC_PROF_GRAM, T * 8.0 * d.ne * nu * (nu + 1) / 2, st);
      const int nb = (d.nu + kGramUB - 1) / kGramUB;
      hipLaunchKernelGGL(k_df_gram, dim3((unsigned)(a.T * (nb * (nb + 1) / 2))), dim3(64), 0, st,
                         a, s);
      APIC_LAUNCHED();
    }
    {
      // complex Cholesky (4/3) n^3 flops plus the two triangular solves 8 n^2
      ProfScope ps(APIC_PROF_CHOL, T * (4.0 / 3.0 * nu * nu * nu + 8.0 * nu * nu), st);
      const int n = d.nu;
      for (int kb = 0; kb < n; kb += kCW) {
        const int pe = std::min(n, kb + kCW);
        for (int sb = kb; sb < pe; sb += kCB) {
          const int bs = std::min(kCB, n - sb);
          const CholArgs ca{n, sb, a.lay.linv, bs, sb + bs, pe};
          hipLaunchKernelGGL(k_chol_potrf, dim3(a.T), dim3(256), 0, st, a, ca);
          APIC_LAUNCHED();
          const int nrb = (n + 1 - (sb + bs) + kCB - 1) / kCB;
          if (nrb > 0) {
            hipLaunchKernelGGL(k_chol_trsm, dim3((unsigned)(a.T * nrb)), dim3(256), 0, st, a, ca);
            APIC_LAUNCHED();
          }
          if (sb + bs < pe) {  // the panel's remaining columns
            hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(a.T * upd_tiles(ca))), dim3(256), 0,
                               st, a, ca);
            APIC_LAUNCHED();
          }
        }
        if (pe < n) {  // the trailing matrix, once per wide panel
          const CholArgs cu{n, kb, a.lay.linv, pe - kb, pe, n};
          hipLaunchKernelGGL(k_chol_update, dim3((unsigned)(a.T * upd_tiles(cu))), dim3(256), 0,
                             st, a, cu);
          APIC_LAUNCHED();
        }
      }
      hipLaunchKernelGGL(k_chol_back, dim3(a.T), dim3(256), 0, st, a, s, n, a.lay.linv);
      APIC_LAUNCHED();
    }
  }
  if (skipped) {
    hipLaunchKernelGGL(k_status_or_all, dim3(blocks_for(a.T, 256)), dim3(256), 0, st, a,
                       (uint32_t)APIC_TILE_DF_SKIPPED);
    APIC_LAUNCHED();
  }
  return APIC_OK;
}

template <int N, int NF>
apic_status run_output_nf(const ClassArgs &a, const c32 *src, float *field, hipStream_t st) {
  // read N^2 spectrum, write/read N x NF row results, write NF^2 field (complex64)
  ProfScope ps(APIC_PROF_OUT, (double)a.T * 8.0 * ((double)N * N + 2.0 * N * NF + (double)NF * NF),
               st);
  hipLaunchKernelGGL((k_rows<c32, NF, OpOut1<NF>>), dim3(row_blocks<c32, NF>(a.T, N)),
                     dim3(kFftThreads), 0, st, OpOut1<NF>{a, src});
  APIC_LAUNCHED();
  APIC_CHECK(launch_cols<c32, NF>(a, a.T, OpOut2<NF>{a, reinterpret_cast<c32 *>(field)}, st));
  return APIC_OK;
}
template <int N>
apic_status run_output(const ClassArgs &a, const c32 *src, float *field, hipStream_t st) {
  if (a.nf == N) return run_output_nf<N, N>(a, src, field, st);
  if constexpr (2 * N <= 1024) return run_output_nf<N, 2 * N>(a, src, field, st);
  return APIC_EUNSUPPORTED;
}

enum Stage : unsigned {
  S_KK = 1, S_PUPIL = 2, S_COEF_IN = 4, S_STITCH = 8, S_SPEC_IN = 16, S_DF = 32, S_SPEC_OUT = 64,
  S_OUT = 128, S_SUR = 256, S_BG = 512, S_PIX = 1024
};

struct CallIO {
  const float *seed = nullptr;
  const float *zin = nullptr;
  float *zout = nullptr, *diag = nullptr, *feat = nullptr;
  float *kk_out = nullptr, *spec_out = nullptr, *spec_io = nullptr, *field = nullptr;
  const float *spec_src = nullptr;
  SurrogateArgs sur{};
  float *zcf = nullptr, *zsur = nullptr;
  float *bg_out = nullptr;
  float *phi_out = nullptr;
  int32_t *pix_iters = nullptr;
  double pix_tol = 1e-10;
  int pix_max_iter = 1000;
};

template <int N>
apic_status run_class_n(const apic_plan *p, const ClassRun &r, const ClassArgs &a, unsigned st_mask,
                        const CallIO &io, hipStream_t st) {
  apic_status rc = APIC_OK;
  if (st_mask & S_BG) {
    hipLaunchKernelGGL(k_bg_stat, dim3(a.T), dim3(kBgThreads), 0, st, a, io.bg_out);
    APIC_LAUNCHED();
  }
  if (st_mask & S_KK) {
    rc = run_kk<N>(a, reinterpret_cast<c32 *>(io.kk_out), st);
    if (rc) return rc;
  }
  int pupil_src = io.seed ? kSeedCaller : kSeedNone;
  const bool sur_seeds = (st_mask & S_SUR) && io.sur.seed_mode;
  if ((st_mask & S_PUPIL) && !sur_seeds) {
    rc = run_pupil(a, io.seed, io.zout, io.diag, io.feat, &pupil_src, st);
    if (rc) return rc;
  }
  if ((st_mask & S_PUPIL) && sur_seeds) {
    // the surrogate seeds the solve: a plain pass gives the features, the
    // surrogate predicts, and one pass re-wrapped about its prediction gives
    // the closed form that judges it
    ProfScope ps(APIC_PROF_PUPIL, (double)a.T * a.n_rows * 32.0, st);
    rc = pupil_pass(a, nullptr, kSeedNone, 1, true, nullptr, nullptr, nullptr, st);
    if (rc) return rc;
    hipLaunchKernelGGL(k_surrogate_predict, dim3(blocks_for(a.T, kMlpTile)), dim3(256), 0, st, a,
                       io.sur);
    APIC_LAUNCHED();
    rc = pupil_pass(a, nullptr, kSeedSur, 1, false, io.zout, io.diag, io.feat, st);
    if (rc) return rc;
    pupil_src = kSeedSur;
  }
  if (st_mask & S_PIX) {
    if (a.n_pix == 0) return APIC_EUNSUPPORTED;
    // the pixel-domain passes walk the rows in pair order (their tables)
    ClassArgs ap = a;
    ap.row_il = (const uint32_t *)p->geoms[r.geom].d_prow_il;
    ap.row_k = (const uint32_t *)p->geoms[r.geom].d_prow_k;
    hipLaunchKernelGGL(k_pix_rows, dim3(ap.T * ap.n_chunks), dim3(256), 0, st, ap);
    APIC_LAUNCHED();
    if (ap.n_pix <= kPixMax) {
      hipLaunchKernelGGL(k_pix_cg, dim3(ap.T), dim3(kPixThreads), 0, st, ap, io.pix_tol,
                         io.pix_max_iter, io.phi_out, io.zout, io.pix_iters);
      APIC_LAUNCHED();
    } else {
      rc = run_pixel_wide(ap, io.pix_tol, io.pix_max_iter, io.phi_out, io.zout, io.pix_iters, st);
      if (rc) return rc;
    }
  }
  if (st_mask & S_SUR) {
    if (!sur_seeds) {
      hipLaunchKernelGGL(k_surrogate_predict, dim3(blocks_for(a.T, kMlpTile)), dim3(256), 0, st,
                         a, io.sur);
      APIC_LAUNCHED();
    }
    hipLaunchKernelGGL(k_surrogate_decide, dim3(blocks_for(a.T, 64)), dim3(64), 0, st, a, io.sur,
                       io.seed, pupil_src, io.zout, io.zcf, io.zsur);
    APIC_LAUNCHED();
  }
  if (st_mask & S_COEF_IN) {
    hipLaunchKernelGGL(k_coef_load, dim3(blocks_for(a.T, 64)), dim3(64), 0, st, a, io.zin);
    APIC_LAUNCHED();
  }
  if (st_mask & S_STITCH) {
    rc = run_stitch(a, p->geoms[r.geom].n_disk, io.spec_out, st);
    if (rc) return rc;
  } else if (st_mask & (S_DF | S_SPEC_IN)) {
    hipLaunchKernelGGL(k_coef_led_phase, dim3(blocks_for(a.T, 64)), dim3(64), 0, st, a);
    APIC_LAUNCHED();
  }
  if (st_mask & S_SPEC_IN) {
    hipLaunchKernelGGL(k_spec_copy, dim3(blocks_for((int64_t)a.T * N * N, 256)), dim3(256), 0, st,
                       a, io.spec_io, 1);
    APIC_LAUNCHED();
  }
  if ((st_mask & S_DF) && !r.skip_df) {
    rc = run_darkfield<N>(p, r, a, st);
    if (rc) return rc;
  }
  if (st_mask & S_SPEC_OUT) {
    hipLaunchKernelGGL(k_spec_copy, dim3(blocks_for((int64_t)a.T * N * N, 256)), dim3(256), 0, st,
                       a, io.spec_io, 0);
    APIC_LAUNCHED();
  }
  if (st_mask & S_OUT) {
    rc = run_output<N>(a, reinterpret_cast<const c32 *>(io.spec_src), io.field, st);
    if (rc) return rc;
  }
  return APIC_OK;
}

apic_status run_class(const apic_plan *plan, const ClassRun &r, const ClassArgs &a,
                      unsigned st_mask, const CallIO &io, hipStream_t st) {
  switch (a.n) {
    case 64: return run_class_n<64>(plan, r, a, st_mask, io, st);
    case 128: return run_class_n<128>(plan, r, a, st_mask, io, st);
    case 256: return run_class_n<256>(plan, r, a, st_mask, io, st);
    case 512: return run_class_n<512>(plan, r, a, st_mask, io, st);
    default: return APIC_EUNSUPPORTED;
  }
}

// Arguments of tiles [c0, c0 + cn) of a class, sharing the class's workspace
// block from its start (chunks of one class run in stream order).
ClassArgs chunk_args(ClassArgs a, int c0, int cn) {
  if (a.affine) {
    a.img0 += (int64_t)c0 * a.img_step;
    a.out0 += (int64_t)c0 * a.out_step;
    a.g0 += c0 * a.g_step;
  } else {
    a.d_img_off += c0;
    a.d_out_off += c0;
    a.d_gidx += c0;
  }
  a.T = cn;
  return a;
}

apic_status run_call(const apic_plan *plan, int32_t n_tiles, const apic_tile_desc *tiles,
                     const float *images, uint32_t *status, void *workspace, size_t ws_bytes,
                     void *stream, unsigned st_mask, const CallIO &io) {
  if (!plan_ok(plan)) return APIC_EPLAN;
  std::vector<ClassRun> runs;
  int64_t need = 0;
  apic_status rc = layout_call(plan, n_tiles, tiles, runs, need);
  if (rc) return rc;
  if (n_tiles == 0) return APIC_OK;
  if (!workspace || (int64_t)ws_bytes < need) return APIC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return APIC_EINVAL;
  rc = apic_plan_upload(const_cast<apic_plan *>(plan));
  if (rc) return rc;
  rc = ensure_twiddles();
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char *ws = reinterpret_cast<char *>(workspace);
  if (status) {
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n_tiles, 256)), dim3(256), 0, st, status,
                       n_tiles, 0u);
    APIC_LAUNCHED();
  }
  rc = upload_descriptors(runs, ws, st);
  if (rc) return rc;
  for (const ClassRun &r : runs) {
    const ClassArgs a = make_args(plan, r, images, ws, status);
    rc = run_class(plan, r, a, st_mask, io, st);
    if (rc) return rc;
  }
  return APIC_OK;
}

template <class C, int L>
apic_status fft2_l(int batch, bool inv, const void *in, void *out, hipStream_t st) {
  const C *src = reinterpret_cast<const C *>(in);
  C *dst = reinterpret_cast<C *>(out);
  if (inv) {
    hipLaunchKernelGGL((k_rows<C, L, OpPlainRows<C, L, true>>), dim3(row_blocks<C, L>(batch, L)),
                       dim3(kFftThreads), 0, st, OpPlainRows<C, L, true>{src, dst});
    APIC_LAUNCHED();
    hipLaunchKernelGGL((k_cols<C, L, OpPlainCols<C, L, true>>), dim3(col_blocks<C, L>(batch)),
                       dim3(kFftThreads), 0, st, OpPlainCols<C, L, true>{dst});
  } else {
    hipLaunchKernelGGL((k_rows<C, L, OpPlainRows<C, L, false>>), dim3(row_blocks<C, L>(batch, L)),
                       dim3(kFftThreads), 0, st, OpPlainRows<C, L, false>{src, dst});
    APIC_LAUNCHED();
    hipLaunchKernelGGL((k_cols<C, L, OpPlainCols<C, L, false>>), dim3(col_blocks<C, L>(batch)),
                       dim3(kFftThreads), 0, st, OpPlainCols<C, L, false>{dst});
  }
  APIC_LAUNCHED();
  return APIC_OK;
}
template <class C>
apic_status fft2_c(int l, int batch, bool inv, const void *in, void *out, hipStream_t st) {
  switch (l) {
    case 64: return fft2_l<C, 64>(batch, inv, in, out, st);
    case 128: return fft2_l<C, 128>(batch, inv, in, out, st);
    case 256: return fft2_l<C, 256>(batch, inv, in, out, st);
    case 512: return fft2_l<C, 512>(batch, inv, in, out, st);
    case 1024: return fft2_l<C, 1024>(batch, inv, in, out, st);
    default: return APIC_EUNSUPPORTED;
  }
}

// ------------------------------------------------------------ static scratch
// Scratch of apic_reconstruct_tiles_static: one array per device.  Host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in): it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
static __device__ __align__(256) char scratch[APIC_STATIC_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void *g_scratch_at[64] = {};

apic_status static_scratch(void **out) {
  int dev = 0;
  APIC_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return APIC_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void *p = nullptr;
    APIC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255) != 0) return APIC_EHIP;
    g_scratch_at[dev] = p;
  }
  *out = g_scratch_at[dev];
  return APIC_OK;
}

}  // namespace
}  // namespace apic

// A prepared batch: class grouping and descriptor tables resident on the
// device, side streams and events for running the geometry classes
// concurrently, and an optional captured graph of one whole reconstruction.
struct apic_batch {
  uint32_t magic = 0x42415443u;  // "BATC"
  apic_plan *plan = nullptr;
  int32_t n_tiles = 0;
  std::vector<apic::ClassRun> runs;
  std::vector<int32_t> chunk;    // tiles per launch sequence, per class
  std::vector<int32_t> lanes;    // chunks of a class in flight at once (1 or 2)
  std::vector<int32_t> fft_var;  // column-pass panel variant per class (0 or 1)
  std::vector<int64_t> cls_ws;   // workspace offset of each class's chunk blocks
  std::vector<hipStream_t> lane_stream;         // a class's second lane
  std::vector<hipEvent_t> lane_fork, lane_join;
  int64_t ws_bytes = 0;
  void *d_desc = nullptr;
  std::vector<hipStream_t> side;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_sur = false;           // pupil stage with the surrogate and fallback rule
  apic::SurrogateArgs sur{};
};

using namespace apic;

extern "C" {

const char *apic_version(void) { return "apic-mi355x 0.1 (gfx950)"; }

apic_status apic_profile(int32_t enable) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_clear();
  g_prof_on = enable != 0;
  return APIC_OK;
}

apic_status apic_profile_read(int32_t group, double *total_ms, int64_t *launches,
                              double *total_work) {
  if (group < 0 || group >= APIC_PROF_GROUPS || !total_ms || !launches || !total_work)
    return APIC_EINVAL;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double ms = 0.0, work = 0.0;
  for (auto &e : g_prof[group]) {
    APIC_HIP(hipEventSynchronize(e.e1));
    float t = 0.f;
    APIC_HIP(hipEventElapsedTime(&t, e.e0, e.e1));
    ms += t;
    work += e.work;
  }
  *total_ms = ms;
  *launches = (int64_t)g_prof[group].size();
  *total_work = work;
  return APIC_OK;
}

apic_status apic_plan_create(const apic_geometry *geoms, int32_t n_geom, apic_plan **out) {
  if (!out) return APIC_EINVAL;
  *out = nullptr;
  if (!geoms || n_geom <= 0 || n_geom > 64) return APIC_EINVAL;
  apic_plan *p = new (std::nothrow) apic_plan();
  if (!p) return APIC_ENOMEM;
  p->geoms.resize(n_geom);
  for (int i = 0; i < n_geom; ++i) {
    const apic_status rc = build_geom_plan(geoms[i], p->geoms[i]);
    if (rc != APIC_OK) {
      delete p;
      return rc;
    }
  }
  *out = p;
  return APIC_OK;
}

apic_status apic_plan_destroy(apic_plan *plan) {
  if (!plan) return APIC_OK;
  if (plan->magic != kPlanMagic) return APIC_EPLAN;
  for (GeomPlan &g : plan->geoms) free_geom(g);
  plan->magic = 0;
  delete plan;
  return APIC_OK;
}

apic_status apic_plan_upload(apic_plan *plan) {
  if (!plan_ok(plan)) return APIC_EPLAN;
  int dev = 0;
  APIC_HIP(hipGetDevice(&dev));
  if (plan->uploaded) return plan->device == dev ? APIC_OK : APIC_EPLAN;
  for (GeomPlan &g : plan->geoms) {
    apic_status rc;
    if ((rc = upload_vec(g.row_il, &g.d_row_il)) || (rc = upload_vec(g.row_k, &g.d_row_k)) ||
        (rc = upload_vec(g.known_at, &g.d_known_at)) || (rc = upload_vec(g.coords, &g.d_coords)) ||
        (rc = upload_vec(g.masks, &g.d_masks)) || (rc = upload_vec(g.pix_tab, &g.d_pix_tab)) ||
        (rc = upload_vec(g.pix_ginv, &g.d_pix_ginv)) ||
        (rc = upload_vec(g.pix_ok ? g.prow_il : std::vector<uint32_t>(), &g.d_prow_il)) ||
        (rc = upload_vec(g.pix_ok ? g.prow_k : std::vector<uint32_t>(), &g.d_prow_k))) {
      for (GeomPlan &h : plan->geoms) free_geom(h);
      return rc;
    }
  }
  plan->device = dev;
  plan->uploaded = true;
  return ensure_twiddles();
}

apic_status apic_workspace_bytes(const apic_plan *plan, int32_t n_tiles,
                                 const apic_tile_desc *tiles, size_t *bytes) {
  if (!plan_ok(plan)) return APIC_EPLAN;
  if (!bytes) return APIC_EINVAL;
  std::vector<ClassRun> runs;
  int64_t need = 0;
  const apic_status rc = layout_call(plan, n_tiles, tiles, runs, need);
  if (rc) return rc;
  *bytes = (size_t)need;
  return APIC_OK;
}

apic_status apic_plan_query(const apic_plan *plan, int32_t geom, int32_t what, int32_t j,
                            int32_t *out, int64_t cap, int64_t *len) {
  if (!plan_ok(plan)) return APIC_EPLAN;
  if (!len || geom < 0 || geom >= (int)plan->geoms.size()) return APIC_EINVAL;
  const GeomPlan &g = plan->geoms[geom];
  std::vector<int32_t> v;
  if (what >= 0 && what <= 3) {
    if (j < 0 || j >= g.n_df) return APIC_EINVAL;
    const DfStep &d = g.steps[j];
    const int64_t off[] = {d.off_u, d.off_p, d.off_q, d.off_e};
    const int cnt[] = {d.nu, d.np, d.m, d.ne};
    for (int i = 0; i < cnt[what]; ++i) {
      const uint32_t w = g.coords[off[what] + i];
      v.push_back(unpack_ky(w));
      v.push_back(unpack_kx(w));
    }
  } else if (what == 4) {
    for (int i = 0; i < g.n_rows; ++i) {
      v.push_back(g.row_il[i] & 0xff);
      v.push_back((g.row_il[i] >> 8) & 0xff);
      v.push_back(unpack_ky(g.row_k[i]));
      v.push_back(unpack_kx(g.row_k[i]));
      v.push_back((int32_t)(g.row_il[i] >> 16));
    }
  } else if (what == 5) {
    v = {g.n_pairs, g.n_rows, g.nu_max, g.m_max, g.ne_max, g.n_active, kGramUB, kEChunk,
         g.n_pix};
  } else if (what == 7) {
    v.assign(g.band_rows.begin(), g.band_rows.end());
  } else if (what == 8) {
    for (const DfStep &d : g.steps) {
      const int32_t sp[] = {d.d_lo, d.d_hi, d.q_lo, d.q_hi, d.z_lo, d.z_hi};
      v.insert(v.end(), sp, sp + 6);
    }
  } else if (what == 6) {
    for (const DfStep &d : g.steps) {
      v.push_back(d.nu);
      v.push_back(d.m);
      v.push_back(d.ne);
      v.push_back((int32_t)std::min<int64_t>(d.gram_live, INT32_MAX));
      v.push_back((int32_t)std::min<int64_t>(d.gram_live_diag, INT32_MAX));
    }
  } else {
    return APIC_EINVAL;
  }
  *len = (int64_t)v.size();
  if (out) {
    if (cap < (int64_t)v.size()) return APIC_EINVAL;
    std::copy(v.begin(), v.end(), out);
  }
  return APIC_OK;
}

apic_status apic_reconstruct_tiles(const apic_plan *plan, int32_t n_tiles,
                                   const apic_tile_desc *tiles, const float *images,
                                   const float *zernike_seed, float *zernike_out,
                                   float *field_out, uint32_t *tile_status, void *workspace,
                                   size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !zernike_out || !field_out || !tile_status)) return APIC_EINVAL;
  CallIO io;
  io.seed = zernike_seed;
  io.zout = zernike_out;
  io.field = field_out;
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_KK | S_PUPIL | S_STITCH | S_DF | S_OUT, io);
}

apic_status apic_reconstruct_tiles_static(const apic_plan *plan, int32_t n_tiles,
                                          const apic_tile_desc *tiles, const float *images,
                                          const float *zernike_seed, float *zernike_out,
                                          float *field_out, uint32_t *tile_status, void *stream) {
  if (!plan_ok(plan)) return APIC_EPLAN;
  if (n_tiles > 0 && (!images || !zernike_out || !field_out || !tile_status)) return APIC_EINVAL;
  std::vector<ClassRun> runs;
  int64_t need = 0;
  apic_status rc = layout_call(plan, n_tiles, tiles, runs, need);
  if (rc) return rc;
  if (n_tiles == 0) return APIC_OK;
  if (need > (int64_t)APIC_STATIC_SCRATCH_BYTES) return APIC_ENOMEM;
  for (const ClassRun &r : runs)
    if (!r.affine) return APIC_EUNSUPPORTED;
  int dev = 0;
  APIC_HIP(hipGetDevice(&dev));
  if (!plan->uploaded || plan->device != dev) return APIC_EPLAN;
  void *ws = nullptr;
  rc = static_scratch(&ws);
  if (rc) return rc;
  // with the plan uploaded and regular descriptors, run_call neither
  // allocates nor copies from the host
  CallIO io;
  io.seed = zernike_seed;
  io.zout = zernike_out;
  io.field = field_out;
  return run_call(plan, n_tiles, tiles, images, tile_status, ws, (size_t)APIC_STATIC_SCRATCH_BYTES,
                  stream, S_KK | S_PUPIL | S_STITCH | S_DF | S_OUT, io);
}

apic_status apic_estimate_pupil(const apic_plan *plan, int32_t n_tiles,
                                const apic_tile_desc *tiles, const float *images,
                                const float *zernike_seed, float *zernike_out, float *diag_out,
                                float *features_out, uint32_t *tile_status, void *workspace,
                                size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !zernike_out || !tile_status)) return APIC_EINVAL;
  CallIO io;
  io.seed = zernike_seed;
  io.zout = zernike_out;
  io.diag = diag_out;
  io.feat = features_out;
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_KK | S_PUPIL, io);
}

apic_status apic_background_stat(const apic_plan *plan, int32_t n_tiles,
                                 const apic_tile_desc *tiles, const float *images,
                                 float *stat_out, void *workspace, size_t workspace_bytes,
                                 void *stream) {
  if (n_tiles > 0 && (!images || !stat_out)) return APIC_EINVAL;
  // the statistic streams the images with 16-byte loads
  if ((reinterpret_cast<uintptr_t>(images) & 15) != 0) return APIC_EINVAL;
  for (int32_t t = 0; t < n_tiles; ++t)
    if (tiles && (tiles[t].image_offset & 3) != 0) return APIC_EINVAL;
  CallIO io;
  io.bg_out = stat_out;
  return run_call(plan, n_tiles, tiles, images, nullptr, workspace, workspace_bytes, stream, S_BG,
                  io);
}

apic_status apic_estimate_pupil_pixel(const apic_plan *plan, int32_t n_tiles,
                                      const apic_tile_desc *tiles, const float *images,
                                      double tol, int32_t max_iter, float *phi_out,
                                      float *zernike_out, int32_t *iters_out,
                                      uint32_t *tile_status, void *workspace,
                                      size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !phi_out || !zernike_out || !tile_status)) return APIC_EINVAL;
  if (!(tol > 0.0 && tol < 1.0) || max_iter < 1) return APIC_EINVAL;
  if (!plan_ok(plan)) return APIC_EPLAN;
  if (plan->geoms.size() != 1) return APIC_EUNSUPPORTED;
  if (!plan->geoms[0].pix_ok) return APIC_EUNSUPPORTED;
  CallIO io;
  io.phi_out = phi_out;
  io.zout = zernike_out;
  io.pix_iters = iters_out;
  io.pix_tol = tol;
  io.pix_max_iter = max_iter;
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_KK | S_PIX, io);
}

apic_status apic_kk_spectra(const apic_plan *plan, int32_t n_tiles, const apic_tile_desc *tiles,
                            const float *images, float *spectra_out, uint32_t *tile_status,
                            void *workspace, size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !spectra_out || !tile_status)) return APIC_EINVAL;
  if (plan_ok(plan) && plan->geoms.size() != 1) return APIC_EUNSUPPORTED;
  CallIO io;
  io.kk_out = spectra_out;
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_KK, io);
}

apic_status apic_stitch_brightfield(const apic_plan *plan, int32_t n_tiles,
                                    const apic_tile_desc *tiles, const float *images,
                                    const float *zernike, float *spectrum_out,
                                    uint32_t *tile_status, void *workspace,
                                    size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !zernike || !spectrum_out || !tile_status)) return APIC_EINVAL;
  CallIO io;
  io.zin = zernike;
  io.spec_out = spectrum_out;
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_KK | S_COEF_IN | S_STITCH, io);
}

apic_status apic_extend_darkfield(const apic_plan *plan, int32_t n_tiles,
                                  const apic_tile_desc *tiles, const float *images,
                                  const float *zernike, float *spectrum_inout,
                                  uint32_t *tile_status, void *workspace,
                                  size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !zernike || !spectrum_inout || !tile_status)) return APIC_EINVAL;
  CallIO io;
  io.zin = zernike;
  io.spec_io = spectrum_inout;
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_COEF_IN | S_SPEC_IN | S_DF | S_SPEC_OUT, io);
}

apic_status apic_upsample_field(const apic_plan *plan, int32_t n_tiles,
                                const apic_tile_desc *tiles, const float *spectrum_in,
                                float *field_out, void *workspace, size_t workspace_bytes,
                                void *stream) {
  if (n_tiles > 0 && (!spectrum_in || !field_out)) return APIC_EINVAL;
  if (plan_ok(plan) && plan->geoms.size() != 1) return APIC_EUNSUPPORTED;
  CallIO io;
  io.spec_src = spectrum_in;
  io.field = field_out;
  return run_call(plan, n_tiles, tiles, nullptr, nullptr, workspace, workspace_bytes, stream,
                  S_OUT, io);
}

apic_status apic_calib_fma64(double *out, int32_t blocks, int32_t iters, void *stream) {
  if (!out || blocks <= 0 || iters < 0) return APIC_EINVAL;
  hipLaunchKernelGGL(k_calib_fma64, dim3(blocks), dim3(256), 0, reinterpret_cast<hipStream_t>(stream),
                     out, iters, 0.999999, 1e-7);
  APIC_LAUNCHED();
  return APIC_OK;
}

apic_status apic_calib_mfma64(double *out, int32_t blocks, int32_t iters, void *stream) {
  if (!out || blocks <= 0 || iters < 0) return APIC_EINVAL;
  hipLaunchKernelGGL(k_calib_mfma64, dim3(blocks), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), out, iters, 0.5, 0.25);
  APIC_LAUNCHED();
  return APIC_OK;
}

apic_status apic_calib_copy(const void *in, void *out, int64_t bytes, void *stream) {
  if (!in || !out || bytes <= 0 || (bytes % 16) != 0) return APIC_EINVAL;
  hipLaunchKernelGGL(k_calib_copy, dim3(256 * 64), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const float4 *>(in),
                     reinterpret_cast<float4 *>(out), bytes / 16);
  APIC_LAUNCHED();
  return APIC_OK;
}

apic_status apic_mlp_forward(const apic_mlp_model *model, int32_t n, const float *inputs,
                             float *outputs, void *stream) {
  if (!model || !model->theta || !model->in_mean || !model->in_std || n < 0) return APIC_EINVAL;
  if (n == 0) return APIC_OK;
  if (!inputs || !outputs) return APIC_EINVAL;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(n, kMlpTile)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), model->theta, model->in_mean,
                     model->in_std, n, inputs, outputs);
  APIC_LAUNCHED();
  return APIC_OK;
}

static apic_status mlp_train_impl(float *theta, float *m, float *v, float *grad, const float *mean,
                                  const float *stdv, int32_t n, const float *inputs,
                                  const float *targets, const int32_t *order, int32_t steps,
                                  int32_t batch, int32_t t0, float lr, float *loss_out,
                                  int grad_only, void *stream) {
  if (!theta || !grad || !mean || !stdv || !inputs || !targets || !order) return APIC_EINVAL;
  if (!grad_only && (!m || !v)) return APIC_EINVAL;
  if (n <= 0 || steps <= 0 || batch <= 0 || t0 < 0 || !(lr >= 0.f)) return APIC_EINVAL;
  MlpTrainArgs a;
  a.theta = theta;
  a.m = m;
  a.v = v;
  a.grad = grad;
  a.inputs = inputs;
  a.targets = targets;
  a.mean = mean;
  a.stdv = stdv;
  a.order = order;
  a.n = n;
  a.steps = steps;
  a.batch = batch;
  a.t0 = t0;
  a.lr = lr;
  a.beta1 = 0.9f;
  a.beta2 = 0.999f;
  a.eps = 1e-8f;
  a.loss_out = loss_out;
  a.grad_only = grad_only;
  hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), a);
  APIC_LAUNCHED();
  return APIC_OK;
}

apic_status apic_mlp_train(float *theta, float *adam_m, float *adam_v, float *grad,
                           const float *in_mean, const float *in_std, int32_t n,
                           const float *inputs, const float *targets, const int32_t *order,
                           int32_t steps, int32_t batch, int32_t t0, float lr, float *loss_out,
                           void *stream) {
  return mlp_train_impl(theta, adam_m, adam_v, grad, in_mean, in_std, n, inputs, targets, order,
                        steps, batch, t0, lr, loss_out, 0, stream);
}

apic_status apic_mlp_grad(const float *theta, float *grad, const float *in_mean,
                          const float *in_std, int32_t n, const float *inputs,
                          const float *targets, const int32_t *order, int32_t batch,
                          float *loss_out, void *stream) {
  return mlp_train_impl(const_cast<float *>(theta), nullptr, nullptr, grad, in_mean, in_std, n,
                        inputs, targets, order, 1, batch, 0, 0.f, loss_out, 1, stream);
}

apic_status apic_bf16_gemm(int32_t m, int32_t n, int32_t k, const uint16_t *a, const uint16_t *b,
                           float *c, void *stream) {
  auto ok = [](int x) { return x >= 16 && x <= 64 && x % 16 == 0; };
  if (!ok(m) || !ok(n) || !ok(k) || !a || !b || !c) return APIC_EINVAL;
  hipLaunchKernelGGL(k_bf16_gemm, dim3(1), dim3(256), 0, reinterpret_cast<hipStream_t>(stream), m,
                     n, k, a, b, c);
  APIC_LAUNCHED();
  return APIC_OK;
}

static bool model_ok(const apic_mlp_model *m) {
  return m && m->theta && m->in_mean && m->in_std && (m->seeds_solve == 0 || m->seeds_solve == 1);
}

apic_status apic_estimate_pupil_sur(const apic_plan *plan, int32_t n_tiles,
                                    const apic_tile_desc *tiles, const float *images,
                                    const float *positions, const apic_mlp_model *model,
                                    float rho_max, float kappa_max, float resid_max,
                                    float *zernike_out, float *zernike_cf_out,
                                    float *zernike_sur_out,
                                    float *diag_out, uint32_t *tile_status, void *workspace,
                                    size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !zernike_out || !tile_status || !positions || !model_ok(model)))
    return APIC_EINVAL;
  CallIO io;
  io.diag = diag_out;
  io.zout = zernike_out;  // closed form first, then the surrogate stage's choice
  io.sur = SurrogateArgs{model ? model->theta : nullptr, model ? model->in_mean : nullptr,
                         model ? model->in_std : nullptr, positions, rho_max, kappa_max,
                         resid_max, model ? model->seeds_solve : 0};
  io.zcf = zernike_cf_out;
  io.zsur = zernike_sur_out;
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_KK | S_PUPIL | S_SUR, io);
}

apic_status apic_reconstruct_tiles_sur(const apic_plan *plan, int32_t n_tiles,
                                       const apic_tile_desc *tiles, const float *images,
                                       const float *positions, const apic_mlp_model *model,
                                       float rho_max, float kappa_max, float resid_max,
                                       float *zernike_out, float *field_out,
                                       uint32_t *tile_status, void *workspace,
                                       size_t workspace_bytes, void *stream) {
  if (n_tiles > 0 && (!images || !zernike_out || !field_out || !tile_status || !positions ||
                      !model_ok(model)))
    return APIC_EINVAL;
  CallIO io;
  io.zout = zernike_out;
  io.field = field_out;
  io.sur = SurrogateArgs{model ? model->theta : nullptr, model ? model->in_mean : nullptr,
                         model ? model->in_std : nullptr, positions, rho_max, kappa_max,
                         resid_max, model ? model->seeds_solve : 0};
  return run_call(plan, n_tiles, tiles, images, tile_status, workspace, workspace_bytes, stream,
                  S_KK | S_PUPIL | S_SUR | S_STITCH | S_DF | S_OUT, io);
}

static bool batch_ok(const apic_batch *b) { return b && b->magic == 0x42415443u && b->plan; }

// Workspace of a batch: one block of lanes x chunk x stride bytes per class
// (classes run concurrently; a class's chunks alternate between its lanes,
// each lane with its own chunk block).
static void batch_layout(apic_batch *b) {
  int64_t o = 0;
  b->cls_ws.assign(b->runs.size(), 0);
  for (size_t c = 0; c < b->runs.size(); ++c) {
    b->cls_ws[c] = o;
    o = align256(o + (int64_t)std::max(1, b->chunk[c]) * b->lanes[c] *
                         b->plan->geoms[b->runs[c].geom].lay.stride);
  }
  b->ws_bytes = std::max<int64_t>(o, 256);
}

static void batch_drop_graph(apic_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

// Enqueue tiles [first, first + count) of class c on stream st, chunk by chunk.
static apic_status batch_run_class(apic_batch *b, size_t c, int first, int count,
                                   const float *images, char *ws, uint32_t *status,
                                   const CallIO &io, hipStream_t st) {
  const unsigned mask = S_KK | S_PUPIL | S_STITCH | S_DF | S_OUT | (b->use_sur ? S_SUR : 0u);
  CallIO iol = io;
  iol.sur = b->sur;
  const ClassRun &r = b->runs[c];
  ClassArgs a = make_args(b->plan, r, images, ws, status, reinterpret_cast<const char *>(b->d_desc));
  a.ws = ws + b->cls_ws[c];
  a.fft_var = b->fft_var[c];
  const int step = std::max(1, b->chunk[c]);  // chunks are >= 1 by construction
  // with two lanes, chunk i runs on lane i % 2 in that lane's workspace block:
  // one chunk's latency-bound kernels overlap the other's throughput-bound ones
  const bool two = b->lanes[c] == 2 && count > step;
  const int64_t lane_bytes = (int64_t)step * b->plan->geoms[r.geom].lay.stride;
  if (two) {
    APIC_HIP(hipEventRecord(b->lane_fork[c], st));
    APIC_HIP(hipStreamWaitEvent(b->lane_stream[c], b->lane_fork[c], 0));
  }
  int i = 0;
  for (int c0 = first; c0 < first + count; c0 += step, ++i) {
    ClassArgs ac = chunk_args(a, c0, std::min(step, first + count - c0));
    hipStream_t sc = st;
    if (two && (i & 1)) {
      ac.ws += lane_bytes;
      sc = b->lane_stream[c];
    }
    const apic_status rc = run_class(b->plan, r, ac, mask, iol, sc);
    if (rc) return rc;
  }
  if (two) {
    APIC_HIP(hipEventRecord(b->lane_join[c], b->lane_stream[c]));
    APIC_HIP(hipStreamWaitEvent(st, b->lane_join[c], 0));
  }
  return APIC_OK;
}

static void batch_free(apic_batch *b) {
  batch_drop_graph(b);
  for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
  for (hipStream_t s : b->lane_stream) (void)hipStreamDestroy(s);
  for (hipEvent_t e : b->lane_fork) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->lane_join) (void)hipEventDestroy(e);
  for (hipEvent_t e : b->join) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->d_desc) (void)hipFree(b->d_desc);
  b->magic = 0;
  delete b;
}

apic_status apic_batch_create(apic_plan *plan, int32_t n_tiles, const apic_tile_desc *tiles,
                              apic_batch **out) {
  if (!out) return APIC_EINVAL;
  *out = nullptr;
  if (!plan_ok(plan)) return APIC_EPLAN;
  apic_batch *b = new (std::nothrow) apic_batch();
  if (!b) return APIC_ENOMEM;
  b->plan = plan;
  b->n_tiles = n_tiles;
  int64_t plain_bytes = 0;
  apic_status rc = layout_call(plan, n_tiles, tiles, b->runs, plain_bytes);
  for (const ClassRun &r : b->runs) {
    b->chunk.push_back((int32_t)r.gidx.size());
    b->lanes.push_back(1);
    b->fft_var.push_back(0);
  }
  batch_layout(b);
  if (rc == APIC_OK) rc = apic_plan_upload(plan);
  if (rc == APIC_OK) rc = ensure_twiddles();
  if (rc != APIC_OK) {
    batch_free(b);
    return rc;
  }
  // descriptor tables of every class, same offsets as in a workspace
  int64_t desc_bytes = 256;
  for (const ClassRun &r : b->runs) desc_bytes = std::max<int64_t>(desc_bytes, r.desc_at + 24 * (int64_t)r.gidx.size());
  std::vector<char> host(desc_bytes, 0);
  for (const ClassRun &r : b->runs) {
    const int64_t T = (int64_t)r.gidx.size();
    memcpy(host.data() + r.desc_at, r.img_off.data(), 8 * T);
    memcpy(host.data() + r.desc_at + 8 * T, r.out_off.data(), 8 * T);
    memcpy(host.data() + r.desc_at + 16 * T, r.gidx.data(), 4 * T);
    memcpy(host.data() + r.desc_at + 20 * T, r.flags.data(), 4 * T);
  }
  bool ok = hipMalloc(&b->d_desc, desc_bytes) == hipSuccess &&
            hipMemcpy(b->d_desc, host.data(), desc_bytes, hipMemcpyHostToDevice) == hipSuccess &&
            hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
  for (size_t c = 0; ok && c < b->runs.size() && b->runs.size() > 1; ++c) {
    hipStream_t s = nullptr;
    hipEvent_t e = nullptr;
    ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    if (ok) b->side.push_back(s);
    ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
    if (ok) b->join.push_back(e);
  }
  for (size_t c = 0; ok && c < b->runs.size(); ++c) {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
    if (ok) b->lane_stream.push_back(s);
    ok = ok && hipEventCreateWithFlags(&e0, hipEventDisableTiming) == hipSuccess;
    if (ok) b->lane_fork.push_back(e0);
    ok = ok && hipEventCreateWithFlags(&e1, hipEventDisableTiming) == hipSuccess;
    if (ok) b->lane_join.push_back(e1);
  }
  if (!ok) {
    batch_free(b);
    return APIC_EHIP;
  }
  *out = b;
  return APIC_OK;
}

apic_status apic_batch_destroy(apic_batch *batch) {
  if (!batch) return APIC_OK;
  if (!batch_ok(batch)) return APIC_EINVAL;
  batch_free(batch);
  return APIC_OK;
}

apic_status apic_batch_workspace_bytes(const apic_batch *batch, size_t *bytes) {
  if (!batch_ok(batch) || !bytes) return APIC_EINVAL;
  *bytes = (size_t)batch->ws_bytes;
  return APIC_OK;
}

apic_status apic_batch_reconstruct(apic_batch *batch, const float *images,
                                   const float *zernike_seed, float *zernike_out, float *field_out,
                                   uint32_t *tile_status, void *workspace, size_t workspace_bytes,
                                   void *stream) {
  if (!batch_ok(batch)) return APIC_EINVAL;
  if (batch->n_tiles == 0) return APIC_OK;
  if (!images || !zernike_out || !field_out || !tile_status) return APIC_EINVAL;
  if (!workspace || (int64_t)workspace_bytes < batch->ws_bytes) return APIC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return APIC_EINVAL;
  if (zernike_seed && batch->use_sur && batch->sur.seed_mode) return APIC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char *ws = reinterpret_cast<char *>(workspace);
  CallIO io;
  io.seed = zernike_seed;
  io.zout = zernike_out;
  io.field = field_out;
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(batch->n_tiles, 256)), dim3(256), 0, st,
                     tile_status, batch->n_tiles, 0u);
  APIC_LAUNCHED();
  if (batch->runs.size() == 1)
    return batch_run_class(batch, 0, 0, (int)batch->runs[0].gidx.size(), images, ws, tile_status,
                           io, st);
  APIC_HIP(hipEventRecord(batch->fork, st));
  for (size_t c = 0; c < batch->runs.size(); ++c) {
    APIC_HIP(hipStreamWaitEvent(batch->side[c], batch->fork, 0));
    const apic_status rc = batch_run_class(batch, c, 0, (int)batch->runs[c].gidx.size(), images,
                                           ws, tile_status, io, batch->side[c]);
    if (rc) return rc;
    APIC_HIP(hipEventRecord(batch->join[c], batch->side[c]));
  }
  for (size_t c = 0; c < batch->runs.size(); ++c) APIC_HIP(hipStreamWaitEvent(st, batch->join[c], 0));
  return APIC_OK;
}

apic_status apic_batch_capture(apic_batch *batch, const float *images, const float *zernike_seed,
                               float *zernike_out, float *field_out, uint32_t *tile_status,
                               void *workspace, size_t workspace_bytes, void *stream) {
  if (!batch_ok(batch) || !stream) return APIC_EINVAL;
  // capture is offered only for one lane per class without the surrogate
  // stage: the capture of a two-lane batch with the surrogate ended in a
  // host-side crash whose cause is not known, so both are refused here,
  // before any capture starts
  if (batch->use_sur) return APIC_EUNSUPPORTED;
  for (const int32_t l : batch->lanes)
    if (l != 1) return APIC_EUNSUPPORTED;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  batch_drop_graph(batch);
  APIC_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const apic_status rc = apic_batch_reconstruct(batch, images, zernike_seed, zernike_out, field_out,
                                                tile_status, workspace, workspace_bytes, stream);
  hipGraph_t g = nullptr;
  const hipError_t end = hipStreamEndCapture(st, &g);
  if (rc != APIC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (end != hipSuccess || !g) return APIC_EHIP;
  batch->graph = g;
  APIC_HIP(hipGraphInstantiate(&batch->exec, g, nullptr, nullptr, 0));
  return APIC_OK;
}

apic_status apic_batch_launch(apic_batch *batch, void *stream) {
  if (!batch_ok(batch) || !batch->exec) return APIC_EINVAL;
  APIC_HIP(hipGraphLaunch(batch->exec, reinterpret_cast<hipStream_t>(stream)));
  return APIC_OK;
}

apic_status apic_batch_classes(const apic_batch *batch, int32_t *n_classes, int32_t *geom,
                               int32_t *n_tiles, int32_t *chunk, int32_t *lanes,
                               int64_t *tile_bytes) {
  if (!batch_ok(batch) || !n_classes) return APIC_EINVAL;
  const int32_t cap = *n_classes;
  *n_classes = (int32_t)batch->runs.size();
  for (int32_t c = 0; c < std::min(cap, *n_classes); ++c) {
    const ClassRun &r = batch->runs[c];
    if (geom) geom[c] = r.geom;
    if (n_tiles) n_tiles[c] = (int32_t)r.gidx.size();
    if (chunk) chunk[c] = batch->chunk[c];
    if (lanes) lanes[c] = batch->lanes[c];
    if (tile_bytes) tile_bytes[c] = batch->plan->geoms[r.geom].lay.stride;
  }
  return APIC_OK;
}

apic_status apic_batch_set_surrogate(apic_batch *batch, const apic_mlp_model *model,
                                     const float *positions, float rho_max, float kappa_max,
                                     float resid_max) {
  if (!batch_ok(batch)) return APIC_EINVAL;
  if (model && (!model_ok(model) || !positions)) return APIC_EINVAL;
  batch->use_sur = model != nullptr;
  batch->sur = model ? SurrogateArgs{model->theta, model->in_mean, model->in_std, positions,
                                     rho_max, kappa_max, resid_max, model->seeds_solve}
                     : SurrogateArgs{};
  batch_drop_graph(batch);
  return APIC_OK;
}

apic_status apic_batch_set_chunk(apic_batch *batch, int32_t cls, int32_t tiles, int32_t lanes) {
  if (!batch_ok(batch) || cls < 0 || cls >= (int32_t)batch->runs.size()) return APIC_EINVAL;
  if (lanes != 1 && lanes != 2) return APIC_EINVAL;
  const int32_t T = (int32_t)batch->runs[cls].gidx.size();
  batch->chunk[cls] = tiles <= 0 ? T : std::min(tiles, T);
  batch->lanes[cls] = lanes;
  batch_layout(batch);
  batch_drop_graph(batch);
  return APIC_OK;
}

apic_status apic_batch_set_fft(apic_batch *batch, int32_t cls, int32_t variant) {
  if (!batch_ok(batch) || cls < 0 || cls >= (int32_t)batch->runs.size()) return APIC_EINVAL;
  if (variant != 0 && variant != 1) return APIC_EINVAL;
  batch->fft_var[cls] = variant;
  batch_drop_graph(batch);
  return APIC_OK;
}

apic_status apic_batch_fft_panel(const apic_batch *batch, int32_t cls, int32_t *variant,
                                 int32_t *panel_columns) {
  if (!batch_ok(batch) || cls < 0 || cls >= (int32_t)batch->runs.size()) return APIC_EINVAL;
  const int v = batch->fft_var[cls];
  if (variant) *variant = v;
  if (panel_columns) {
    int cols = 0;
    switch (batch->plan->geoms[batch->runs[cls].geom].n) {
      case 64: cols = v ? ColShapeAlt<c64, 64>::NSEQ : ColShape<c64, 64>::NSEQ; break;
      case 128: cols = v ? ColShapeAlt<c64, 128>::NSEQ : ColShape<c64, 128>::NSEQ; break;
      case 256: cols = v ? ColShapeAlt<c64, 256>::NSEQ : ColShape<c64, 256>::NSEQ; break;
      case 512: cols = v ? ColShapeAlt<c64, 512>::NSEQ : ColShape<c64, 512>::NSEQ; break;
      default: return APIC_EUNSUPPORTED;
    }
    *panel_columns = cols;
  }
  return APIC_OK;
}

apic_status apic_batch_fit(apic_batch *batch, size_t workspace_bytes) {
  if (!batch_ok(batch)) return APIC_EINVAL;
  // the classes run concurrently: halve the largest blocks until they fit together
  const std::vector<int32_t> saved = batch->chunk;
  batch_layout(batch);
  while (batch->ws_bytes > (int64_t)workspace_bytes) {
    size_t big = 0;
    int64_t big_bytes = -1;
    for (size_t c = 0; c < batch->runs.size(); ++c) {
      const int64_t b = (int64_t)batch->chunk[c] * batch->lanes[c] *
                        batch->plan->geoms[batch->runs[c].geom].lay.stride;
      if (batch->chunk[c] > 1 && b > big_bytes) {
        big = c;
        big_bytes = b;
      }
    }
    if (big_bytes < 0) {  // one tile per class does not fit
      batch->chunk = saved;
      batch_layout(batch);
      return APIC_EINVAL;
    }
    batch->chunk[big] = (batch->chunk[big] + 1) / 2;
    batch_layout(batch);
  }
  batch_drop_graph(batch);
  return APIC_OK;
}

apic_status apic_batch_autotune(apic_batch *batch, int32_t cls, const float *images,
                                float *zernike_out, float *field_out, uint32_t *tile_status,
                                void *workspace, size_t workspace_bytes, void *stream,
                                double slack, double *ms_per_tile) {
  if (!batch_ok(batch) || cls >= (int32_t)batch->runs.size()) return APIC_EINVAL;
  if (batch->n_tiles == 0) return APIC_OK;
  if (!images || !zernike_out || !field_out || !tile_status || !workspace) return APIC_EINVAL;
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0) return APIC_EINVAL;
  if (!(slack >= 0.0)) return APIC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  APIC_HIP(hipStreamIsCapturing(st, &cs));
  if (cs != hipStreamCaptureStatusNone) return APIC_EINVAL;
  char *ws = reinterpret_cast<char *>(workspace);
  CallIO io;
  io.zout = zernike_out;
  io.field = field_out;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  APIC_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return APIC_EHIP;
  }
  apic_status rc = APIC_OK;
  const std::vector<int32_t> saved = batch->chunk, saved_lanes = batch->lanes,
                             saved_fft = batch->fft_var;
  std::vector<int64_t> saved_ws = batch->cls_ws;
  // time tiles [0, count) of class c with the current chunk and lanes, from
  // offset 0 of the workspace
  auto time_class = [&](size_t c, int count, float &ms) -> apic_status {
    batch->cls_ws[c] = 0;
    hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(batch->n_tiles, 256)), dim3(256), 0, st,
                       tile_status, batch->n_tiles, 0u);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e0, st) != hipSuccess) return APIC_EHIP;
    const apic_status r = batch_run_class(batch, c, 0, count, images, ws, tile_status, io, st);
    if (r != APIC_OK) return r;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return APIC_EHIP;
    return APIC_OK;
  };
  for (size_t c = 0; c < batch->runs.size() && rc == APIC_OK; ++c) {
    if (cls >= 0 && (int32_t)c != cls) continue;
    const int32_t T = (int32_t)batch->runs[c].gidx.size();
    const int64_t stride = batch->plan->geoms[batch->runs[c].geom].lay.stride;
    std::vector<int32_t> cand;
    for (int32_t k = 1; k < T; k *= 2) cand.push_back(k);
    cand.push_back(T);
    double best = 1e300;
    int32_t pick = 0;
    std::vector<double> per_tile;
    for (size_t i = 0; i < cand.size() && rc == APIC_OK; ++i) {
      const int32_t k = cand[i];
      if ((int64_t)k * stride > (int64_t)workspace_bytes) break;
      // tiles [0, k) of the class as one chunk (one lane)
      batch->chunk[c] = k;
      batch->lanes[c] = 1;
      float ms = 0.f;
      for (int rep = 0; rep < (i == 0 ? 2 : 1) && rc == APIC_OK; ++rep) rc = time_class(c, k, ms);
      const double tile_ms = (double)ms / k;
      const double prev = per_tile.empty() ? 1e300 : per_tile.back();
      per_tile.push_back(tile_ms);
      if (tile_ms < best) {
        best = tile_ms;
        pick = k;
      }
      // stop once doubling the chunk gains under 3% (past 4 tiles), or after 10 s
      if ((k >= 4 && tile_ms > 0.97 * prev) || ms > 10000.f) break;
    }
    if (rc != APIC_OK) break;
    if (per_tile.empty()) {
      rc = APIC_EINVAL;  // not even one tile of this class fits the workspace
      break;
    }
    // smallest chunk within (1 + slack) of the best time per tile (the best
    // itself qualifies, so pick >= 1)
    for (size_t i = 0; i < per_tile.size(); ++i)
      if (per_tile[i] <= best * (1.0 + slack)) {
        pick = cand[i];
        break;
      }
    if (ms_per_tile) ms_per_tile[c] = best;
    batch->chunk[c] = pick;
    batch->lanes[c] = 1;
    // two lanes of half the chunk (same workspace): one chunk's latency-bound
    // kernels run beside the other's; kept if 2% faster over the same tiles
    if (pick >= 2) {
      const int span = std::min(T, 2 * pick);
      float ms1 = 0.f, ms2 = 0.f;
      rc = time_class(c, span, ms1);
      if (rc == APIC_OK) {
        batch->chunk[c] = (pick + 1) / 2;
        batch->lanes[c] = 2;
        rc = time_class(c, span, ms2);
      }
      if (rc == APIC_OK && !(ms2 < 0.98f * ms1)) {
        batch->chunk[c] = pick;
        batch->lanes[c] = 1;
      }
      if (rc == APIC_OK && ms_per_tile) ms_per_tile[c] = std::min(ms1, ms2) / span;
    }
    // the column passes' panel width (LDS tiling): kept if 2% faster over
    // the chosen chunk
    if (rc == APIC_OK) {
      const int span = std::min(T, batch->chunk[c] * batch->lanes[c]);
      float ms0 = 0.f, ms1 = 0.f;
      batch->fft_var[c] = 0;
      rc = time_class(c, span, ms0);
      if (rc == APIC_OK) {
        batch->fft_var[c] = 1;
        rc = time_class(c, span, ms1);
      }
      if (rc == APIC_OK && !(ms1 < 0.98f * ms0)) batch->fft_var[c] = 0;
      if (rc == APIC_OK && ms_per_tile) ms_per_tile[c] = std::min(ms0, ms1) / span;
    }
    batch->cls_ws = saved_ws;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != APIC_OK) {
    batch->chunk = saved;
    batch->lanes = saved_lanes;
    batch->fft_var = saved_fft;
    batch_layout(batch);
    batch_drop_graph(batch);
    return rc;
  }
  batch_layout(batch);
  batch_drop_graph(batch);
  return cls < 0 ? apic_batch_fit(batch, workspace_bytes) : APIC_OK;
}

apic_status apic_fft2(int32_t l, int32_t batch, int32_t inverse, int32_t precision,
                      const void *in, void *out, void *stream) {
  if (batch < 0 || !in || !out) return APIC_EINVAL;
  if (batch == 0) return APIC_OK;
  if (precision != 0 && precision != 1) return APIC_EINVAL;
  const apic_status rc = ensure_twiddles();
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  return precision == 0 ? fft2_c<c32>(l, batch, inverse != 0, in, out, st)
                        : fft2_c<c64>(l, batch, inverse != 0, in, out, st);
}

}  // extern "C"

// ------------------------------------------------------------ slide stream
// Tiles whose images live in host memory go through `nbuf` device staging
// buffers, one default-priority stream each.  Chunk c uses buffer c % nbuf:
// copy in, background statistic, the method on the chunk's non-background
// tiles, copy out.  The host enqueues chunk c's copy-in before it waits for
// chunk c - 1's statistic and enqueues that chunk's method, so one chunk's
// copies run under the earlier chunks' kernels.
struct apic_streamer {
  uint32_t magic = 0x5354524du;  // "STRM"
  apic_plan *plan = nullptr;
  int geom = 0, chunk = 0, nbuf = 0;
  int64_t img_elems = 0;   // floats per tile image stack
  int64_t fld_elems = 0;   // complex elements per tile field
  size_t ws_bytes = 0;     // workspace of one chunk
  struct Buf {
    hipStream_t s = nullptr;
    hipEvent_t stat_ready = nullptr, done = nullptr;
    void *dev = nullptr;     // one allocation: images, field, workspace, small arrays
    void *host = nullptr;    // pinned staging of the small per-tile arrays
    float *d_img = nullptr, *d_field = nullptr, *d_z = nullptr, *d_pos = nullptr, *d_bg = nullptr;
    uint32_t *d_status = nullptr;
    char *d_ws = nullptr;
    float *h_bg = nullptr, *h_z = nullptr, *h_pos = nullptr;
    uint32_t *h_status = nullptr;
    int first = 0, count = 0;
    std::vector<int> live;   // slots of the chunk's reconstructed tiles
    bool pending = false;    // results not yet copied to the caller's arrays
  };
  std::vector<Buf> bufs;
  size_t dev_bytes = 0;
};

static bool streamer_ok(const apic_streamer *s) {
  return s && s->magic == 0x5354524du && s->plan;
}

static void streamer_free(apic_streamer *s) {
  for (apic_streamer::Buf &b : s->bufs) {
    if (b.s) (void)hipStreamSynchronize(b.s);
    if (b.s) (void)hipStreamDestroy(b.s);
    if (b.stat_ready) (void)hipEventDestroy(b.stat_ready);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.dev) (void)hipFree(b.dev);
    if (b.host) (void)hipHostFree(b.host);
  }
  s->magic = 0;
  delete s;
}

// Descriptors of the given staging slots (slot i holds the chunk's i-th tile).
static std::vector<apic_tile_desc> slot_descs(const apic_streamer *s, const std::vector<int> &slots) {
  std::vector<apic_tile_desc> d(slots.size());
  for (size_t k = 0; k < slots.size(); ++k) {
    d[k].geom = s->geom;
    d[k].flags = 0;
    d[k].image_offset = (int64_t)slots[k] * s->img_elems;
    d[k].field_offset = (int64_t)slots[k] * s->fld_elems;
    d[k].pos_x = d[k].pos_y = 0.f;
  }
  return d;
}

apic_status apic_streamer_create(apic_plan *plan, int32_t geom, int32_t chunk, int32_t n_buffers,
                                 apic_streamer **out) {
  if (!out) return APIC_EINVAL;
  *out = nullptr;
  if (!plan_ok(plan)) return APIC_EPLAN;
  if (geom < 0 || geom >= (int32_t)plan->geoms.size() || chunk < 1 || n_buffers < 2 ||
      n_buffers > 4)
    return APIC_EINVAL;
  apic_status rc = apic_plan_upload(plan);
  if (rc) return rc;
  rc = ensure_twiddles();
  if (rc) return rc;
  apic_streamer *s = new (std::nothrow) apic_streamer();
  if (!s) return APIC_ENOMEM;
  const GeomPlan &g = plan->geoms[geom];
  s->plan = plan;
  s->geom = geom;
  s->chunk = chunk;
  s->nbuf = n_buffers;
  s->img_elems = (int64_t)(g.n_bf + g.n_df) * g.n * g.n;
  s->fld_elems = (int64_t)g.nf * g.nf;
  std::vector<int> all(chunk);
  for (int i = 0; i < chunk; ++i) all[i] = i;
  // the whole chunk's layout (descriptor lists included) bounds every subset's
  const std::vector<apic_tile_desc> d = slot_descs(s, all);
  std::vector<ClassRun> runs;
  int64_t need = 0;
  rc = layout_call(plan, chunk, d.data(), runs, need);
  if (rc) {
    delete s;
    return rc;
  }
  s->ws_bytes = (size_t)align256(need);
  const int64_t img_b = align256(4 * s->img_elems * chunk);
  const int64_t fld_b = align256(8 * s->fld_elems * chunk);
  const int64_t small_b = align256(4 * (int64_t)chunk * (15 + 2 + 1 + 1));
  const size_t per = (size_t)(img_b + fld_b + (int64_t)s->ws_bytes + small_b);
  s->dev_bytes = per * n_buffers;
  s->bufs.resize(n_buffers);
  bool ok = true;
  for (apic_streamer::Buf &b : s->bufs) {
    ok = ok && hipStreamCreateWithFlags(&b.s, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b.stat_ready, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&b.done, hipEventDisableTiming) == hipSuccess &&
         hipMalloc(&b.dev, per) == hipSuccess &&
         hipHostMalloc(&b.host, (size_t)small_b, hipHostMallocDefault) == hipSuccess;
    if (!ok) break;
    char *p = reinterpret_cast<char *>(b.dev);
    b.d_img = reinterpret_cast<float *>(p);
    b.d_field = reinterpret_cast<float *>(p + img_b);
    b.d_ws = p + img_b + fld_b;
    float *sm = reinterpret_cast<float *>(b.d_ws + s->ws_bytes);
    b.d_z = sm;
    b.d_pos = sm + 15 * chunk;
    b.d_bg = sm + 17 * chunk;
    b.d_status = reinterpret_cast<uint32_t *>(sm + 18 * chunk);
    float *hs = reinterpret_cast<float *>(b.host);
    b.h_z = hs;
    b.h_pos = hs + 15 * chunk;
    b.h_bg = hs + 17 * chunk;
    b.h_status = reinterpret_cast<uint32_t *>(hs + 18 * chunk);
  }
  if (!ok) {
    streamer_free(s);
    return APIC_EHIP;
  }
  *out = s;
  return APIC_OK;
}

apic_status apic_streamer_destroy(apic_streamer *s) {
  if (!s) return APIC_OK;
  if (!streamer_ok(s)) return APIC_EINVAL;
  streamer_free(s);
  return APIC_OK;
}

apic_status apic_streamer_device_bytes(const apic_streamer *s, size_t *bytes) {
  if (!streamer_ok(s) || !bytes) return APIC_EINVAL;
  *bytes = s->dev_bytes;
  return APIC_OK;
}

apic_status apic_streamer_run(apic_streamer *s, int32_t n_tiles, const float *const *host_images,
                              float *const *host_fields, const float *positions,
                              const apic_mlp_model *model, float rho_max, float kappa_max,
                              float resid_max, float bg_threshold, float *zernike_out,
                              uint32_t *tile_status, float *bg_stat_out) {
  if (!streamer_ok(s) || n_tiles < 0) return APIC_EINVAL;
  if (n_tiles == 0) return APIC_OK;
  if (!host_images || !host_fields || !zernike_out || !tile_status) return APIC_EINVAL;
  if (model && (!model_ok(model) || !positions)) return APIC_EINVAL;
  for (int32_t t = 0; t < n_tiles; ++t)
    if (!host_images[t] || !host_fields[t]) return APIC_EINVAL;
  const size_t img_bytes = 4 * (size_t)s->img_elems, fld_bytes = 8 * (size_t)s->fld_elems;
  unsigned mask = S_KK | S_PUPIL | S_STITCH | S_DF | S_OUT;
  CallIO io;
  if (model) {
    mask |= S_SUR;
    io.sur = SurrogateArgs{model->theta, model->in_mean, model->in_std, nullptr, rho_max,
                           kappa_max, resid_max, model->seeds_solve};
  }
  const int nch = (n_tiles + s->chunk - 1) / s->chunk;

  // copy in + statistic of chunk c
  auto stage_in = [&](int c) -> apic_status {
    apic_streamer::Buf &b = s->bufs[c % s->nbuf];
    b.first = c * s->chunk;
    b.count = std::min(s->chunk, n_tiles - b.first);
    for (int i = 0; i < b.count; ++i)
      APIC_HIP(hipMemcpyAsync(b.d_img + (int64_t)i * s->img_elems, host_images[b.first + i],
                              img_bytes, hipMemcpyHostToDevice, b.s));
    std::vector<int> all(b.count);
    for (int i = 0; i < b.count; ++i) all[i] = i;
    const std::vector<apic_tile_desc> d = slot_descs(s, all);
    CallIO bio;
    bio.bg_out = b.d_bg;
    apic_status rc = run_call(s->plan, b.count, d.data(), b.d_img, nullptr, b.d_ws, s->ws_bytes,
                              b.s, S_BG, bio);
    if (rc) return rc;
    APIC_HIP(hipMemcpyAsync(b.h_bg, b.d_bg, 4 * (size_t)b.count, hipMemcpyDeviceToHost, b.s));
    APIC_HIP(hipEventRecord(b.stat_ready, b.s));
    return APIC_OK;
  };
  // background decision, method and copy out of chunk c
  auto run_chunk = [&](int c) -> apic_status {
    apic_streamer::Buf &b = s->bufs[c % s->nbuf];
    APIC_HIP(hipEventSynchronize(b.stat_ready));
    b.live.clear();
    for (int i = 0; i < b.count; ++i) {
      const int t = b.first + i;
      const float st = b.h_bg[i];
      if (bg_stat_out) bg_stat_out[t] = st;
      if (bg_threshold > 0.f && st < bg_threshold) {
        tile_status[t] = APIC_TILE_BACKGROUND;
        for (int j = 0; j < 15; ++j) zernike_out[15 * (int64_t)t + j] = 0.f;
      } else {
        b.live.push_back(i);
      }
    }
    if (!b.live.empty()) {
      const std::vector<apic_tile_desc> d = slot_descs(s, b.live);
      CallIO cio = io;
      cio.zout = b.d_z;
      cio.field = b.d_field;
      if (model) {
        for (size_t k = 0; k < b.live.size(); ++k) {
          b.h_pos[2 * k] = positions[2 * (int64_t)(b.first + b.live[k])];
          b.h_pos[2 * k + 1] = positions[2 * (int64_t)(b.first + b.live[k]) + 1];
        }
        APIC_HIP(hipMemcpyAsync(b.d_pos, b.h_pos, 8 * b.live.size(), hipMemcpyHostToDevice, b.s));
        cio.sur.positions = b.d_pos;
      }
      apic_status rc = run_call(s->plan, (int32_t)b.live.size(), d.data(), b.d_img, b.d_status,
                                b.d_ws, s->ws_bytes, b.s, mask, cio);
      if (rc) return rc;
      for (size_t k = 0; k < b.live.size(); ++k)
        APIC_HIP(hipMemcpyAsync(host_fields[b.first + b.live[k]],
                                b.d_field + 2 * (int64_t)b.live[k] * s->fld_elems, fld_bytes,
                                hipMemcpyDeviceToHost, b.s));
      APIC_HIP(hipMemcpyAsync(b.h_z, b.d_z, 60 * b.live.size(), hipMemcpyDeviceToHost, b.s));
      APIC_HIP(hipMemcpyAsync(b.h_status, b.d_status, 4 * b.live.size(), hipMemcpyDeviceToHost,
                              b.s));
    }
    APIC_HIP(hipEventRecord(b.done, b.s));
    b.pending = true;
    return APIC_OK;
  };
  // results of the chunk last run on buffer b into the caller's arrays
  auto harvest = [&](apic_streamer::Buf &b) -> apic_status {
    if (!b.pending) return APIC_OK;
    APIC_HIP(hipEventSynchronize(b.done));
    for (size_t k = 0; k < b.live.size(); ++k) {
      const int64_t t = b.first + b.live[k];
      for (int j = 0; j < 15; ++j) zernike_out[15 * t + j] = b.h_z[15 * k + j];
      tile_status[t] = b.h_status[k];
    }
    b.pending = false;
    return APIC_OK;
  };

  apic_status rc = APIC_OK;
  for (int c = 0; c <= nch && rc == APIC_OK; ++c) {
    if (c < nch) {
      rc = harvest(s->bufs[c % s->nbuf]);
      if (rc == APIC_OK) rc = stage_in(c);
    }
    if (rc == APIC_OK && c >= 1) rc = run_chunk(c - 1);
  }
  for (apic_streamer::Buf &b : s->bufs) {
    if (rc != APIC_OK) {
      (void)hipStreamSynchronize(b.s);  // host buffers may still be in flight
      b.pending = false;
    } else {
      rc = harvest(b);
    }
  }
  return rc;
}

// ------------------------------------------------------------ patch assembly
namespace {

bool asm_args_ok(int32_t T, int32_t n, const int32_t *pos) {
  return T >= 0 && n >= 1 && n <= 4096 && (T == 0 || pos);
}

// Overlapping pairs (t < u) with at least min_ov rows and columns in common.
std::vector<apic::AsmPair> asm_pairs(int32_t T, int32_t n, const int32_t *pos, int32_t min_ov) {
  std::vector<apic::AsmPair> out;
  for (int t = 0; t < T; ++t)
    for (int u = t + 1; u < T; ++u) {
      const int y0 = std::max(pos[2 * t], pos[2 * u]), y1 = std::min(pos[2 * t], pos[2 * u]) + n;
      const int x0 = std::max(pos[2 * t + 1], pos[2 * u + 1]),
                x1 = std::min(pos[2 * t + 1], pos[2 * u + 1]) + n;
      if (y1 - y0 >= min_ov && x1 - x0 >= min_ov) out.push_back({t, u, y0, y1, x0, x1});
    }
  return out;
}

// Per canvas block (kAsmBlock square, row-major) the tiles that cover part of it.
void asm_blocks(int32_t T, int32_t n, const int32_t *pos, int32_t H, int32_t W,
                std::vector<int32_t> &start, std::vector<int32_t> &tiles) {
  const int bh = (H + apic::kAsmBlock - 1) / apic::kAsmBlock;
  const int bw = (W + apic::kAsmBlock - 1) / apic::kAsmBlock;
  std::vector<std::vector<int32_t>> lists((size_t)bh * bw);
  for (int t = 0; t < T; ++t) {
    const int y0 = std::max(0, pos[2 * t]), y1 = std::min(H, pos[2 * t] + n);
    const int x0 = std::max(0, pos[2 * t + 1]), x1 = std::min(W, pos[2 * t + 1] + n);
    if (y0 >= y1 || x0 >= x1) continue;
    for (int by = y0 / apic::kAsmBlock; by <= (y1 - 1) / apic::kAsmBlock; ++by)
      for (int bx = x0 / apic::kAsmBlock; bx <= (x1 - 1) / apic::kAsmBlock; ++bx)
        lists[(size_t)by * bw + bx].push_back(t);
  }
  start.assign(lists.size() + 1, 0);
  tiles.clear();
  for (size_t b = 0; b < lists.size(); ++b) {
    tiles.insert(tiles.end(), lists[b].begin(), lists[b].end());
    start[b + 1] = (int32_t)tiles.size();
  }
}

// Leading eigenvector phases of each connected group of the overlap graph
// (angular synchronisation), the group's lowest tile at 0.  Power iteration
// on C + sigma I (sigma = the largest absolute row sum, so every eigenvalue is
// >= 0 and the largest one leads) from the phases propagated along a
// breadth-first tree of the group.
void asm_synchronise(int32_t T, const std::vector<apic::AsmPair> &pairs,
                     const std::vector<c64> &corr, float *theta) {
  std::vector<std::vector<std::pair<int, std::complex<double>>>> adj(T);
  for (size_t k = 0; k < pairs.size(); ++k) {
    const std::complex<double> c(corr[k].x, corr[k].y);
    if (c == 0.0) continue;
    adj[pairs[k].t].push_back({pairs[k].u, c});
    adj[pairs[k].u].push_back({pairs[k].t, std::conj(c)});
  }
  std::vector<int> group_of(T, -1);
  for (int s = 0; s < T; ++s) theta[s] = 0.f;
  for (int s = 0; s < T; ++s) {
    if (group_of[s] >= 0) continue;
    std::vector<int> order{s};
    std::vector<std::complex<double>> v0;
    group_of[s] = s;
    std::vector<double> phi(T, 0.0);
    for (size_t h = 0; h < order.size(); ++h) {
      const int t = order[h];
      for (const auto &e : adj[t])
        if (group_of[e.first] < 0) {
          group_of[e.first] = s;
          phi[e.first] = phi[t] - std::arg(e.second);  // C_tu ~ exp(j (theta_t - theta_u))
          order.push_back(e.first);
        }
    }
    if (order.size() == 1) continue;
    std::sort(order.begin(), order.end());
    std::vector<int> local(T, -1);
    for (size_t i = 0; i < order.size(); ++i) local[order[i]] = (int)i;
    double sigma = 0.0;
    for (int t : order) {
      double row = 0.0;
      for (const auto &e : adj[t]) row += std::abs(e.second);
      sigma = std::max(sigma, row);
    }
    const size_t m = order.size();
    std::vector<std::complex<double>> v(m), w(m);
    for (size_t i = 0; i < m; ++i) v[i] = std::polar(1.0, phi[order[i]]);
    for (int it = 0; it < 200000; ++it) {
      double nrm = 0.0;
      for (size_t i = 0; i < m; ++i) {
        std::complex<double> acc = sigma * v[i];
        for (const auto &e : adj[order[i]]) acc += e.second * v[local[e.first]];
        w[i] = acc;
        nrm = std::max(nrm, std::abs(acc));
      }
      double change = 0.0;
      for (size_t i = 0; i < m; ++i) {
        w[i] /= nrm;
        change = std::max(change, std::abs(w[i] - v[i]));
      }
      v.swap(w);
      if (change < 1e-14) break;
    }
    const std::complex<double> ref = std::conj(v[0]) / std::abs(v[0]);
    for (size_t i = 0; i < m; ++i) theta[order[i]] = (float)std::arg(v[i] * ref);
  }
}

}  // namespace

// A prepared assembly: overlapping pairs and per-block tile lists resident
// on the device.
struct apic_assembly {
  uint32_t magic = 0x41534d42u;  // "ASMB"
  int32_t T = 0, n = 0, H = 0, W = 0, bw = 0, nb = 0;
  std::vector<int32_t> pos;
  std::vector<apic::AsmPair> pairs;
  void *dev = nullptr;  // pos, pairs, correlations, block starts, block tiles
  int32_t *d_pos = nullptr, *d_start = nullptr, *d_tiles = nullptr;
  apic::AsmPair *d_pairs = nullptr;
  c64 *d_corr = nullptr;
};

static bool assembly_ok(const apic_assembly *a) { return a && a->magic == 0x41534d42u; }

apic_status apic_assembly_create(int32_t n_tiles, int32_t n, const int32_t *pos,
                                 int32_t min_overlap, int32_t canvas_h, int32_t canvas_w,
                                 apic_assembly **out) {
  if (!out) return APIC_EINVAL;
  *out = nullptr;
  if (!asm_args_ok(n_tiles, n, pos) || n_tiles < 1 || canvas_h < 1 || canvas_w < 1)
    return APIC_EINVAL;
  apic_assembly *a = new (std::nothrow) apic_assembly();
  if (!a) return APIC_ENOMEM;
  a->T = n_tiles;
  a->n = n;
  a->H = canvas_h;
  a->W = canvas_w;
  a->pos.assign(pos, pos + 2 * (size_t)n_tiles);
  a->pairs = asm_pairs(n_tiles, n, pos, std::max(1, min_overlap));
  std::vector<int32_t> start, tiles;
  asm_blocks(n_tiles, n, pos, canvas_h, canvas_w, start, tiles);
  a->nb = (int32_t)(start.size() - 1);
  a->bw = (canvas_w + kAsmBlock - 1) / kAsmBlock;
  const size_t P = a->pairs.size();
  const int64_t o_pairs = align256(8 * (int64_t)n_tiles);
  const int64_t o_corr = o_pairs + align256(24 * (int64_t)P);
  const int64_t o_start = o_corr + align256(16 * (int64_t)P);
  const int64_t o_tiles = o_start + align256(4 * (int64_t)start.size());
  const int64_t total = o_tiles + align256(4 * (int64_t)std::max<size_t>(1, tiles.size()));
  bool ok = hipMalloc(&a->dev, (size_t)total) == hipSuccess;
  if (ok) {
    char *d = reinterpret_cast<char *>(a->dev);
    a->d_pos = reinterpret_cast<int32_t *>(d);
    a->d_pairs = reinterpret_cast<AsmPair *>(d + o_pairs);
    a->d_corr = reinterpret_cast<c64 *>(d + o_corr);
    a->d_start = reinterpret_cast<int32_t *>(d + o_start);
    a->d_tiles = reinterpret_cast<int32_t *>(d + o_tiles);
    ok = hipMemcpy(a->d_pos, pos, 8 * (size_t)n_tiles, hipMemcpyHostToDevice) == hipSuccess &&
         (P == 0 || hipMemcpy(a->d_pairs, a->pairs.data(), sizeof(AsmPair) * P,
                              hipMemcpyHostToDevice) == hipSuccess) &&
         hipMemcpy(a->d_start, start.data(), 4 * start.size(), hipMemcpyHostToDevice) ==
             hipSuccess &&
         (tiles.empty() || hipMemcpy(a->d_tiles, tiles.data(), 4 * tiles.size(),
                                     hipMemcpyHostToDevice) == hipSuccess);
  }
  if (!ok) {
    if (a->dev) (void)hipFree(a->dev);
    delete a;
    return APIC_EHIP;
  }
  *out = a;
  return APIC_OK;
}

apic_status apic_assembly_destroy(apic_assembly *a) {
  if (!a) return APIC_OK;
  if (!assembly_ok(a)) return APIC_EINVAL;
  if (a->dev) (void)hipFree(a->dev);
  a->magic = 0;
  delete a;
  return APIC_OK;
}

apic_status apic_assemble_phases(apic_assembly *a, const float *fields, float *theta_out,
                                 void *stream) {
  if (!assembly_ok(a) || !fields || !theta_out) return APIC_EINVAL;
  for (int t = 0; t < a->T; ++t) theta_out[t] = 0.f;
  if (a->pairs.empty()) return APIC_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_overlap_corr, dim3((unsigned)a->pairs.size()), dim3(256), 0, st,
                     reinterpret_cast<const c32 *>(fields), a->n, a->d_pos, a->d_pairs,
                     a->d_corr);
  APIC_LAUNCHED();
  std::vector<c64> corr(a->pairs.size());
  APIC_HIP(hipStreamSynchronize(st));
  APIC_HIP(hipMemcpy(corr.data(), a->d_corr, sizeof(c64) * corr.size(), hipMemcpyDeviceToHost));
  asm_synchronise(a->T, a->pairs, corr, theta_out);
  return APIC_OK;
}

apic_status apic_blend(const apic_assembly *a, const float *fields, const float *theta,
                       float ramp_width, float *canvas, void *stream) {
  if (!assembly_ok(a) || !fields || !canvas || !(ramp_width >= 1.f)) return APIC_EINVAL;
  hipLaunchKernelGGL(k_blend, dim3((unsigned)a->nb), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), reinterpret_cast<const c32 *>(fields),
                     a->n, a->d_pos, a->d_start, a->d_tiles, theta, 1.f / ramp_width,
                     reinterpret_cast<c32 *>(canvas), a->H, a->W, a->bw);
  APIC_LAUNCHED();
  return APIC_OK;
}

// ------------------------------------------------------------ colour image
apic_status apic_rgb_combine(int32_t n_tiles, int32_t nf, const float *field_r,
                             const float *field_g, const float *field_b, const float *gains,
                             float *rgb_out, float *gains_out, void *workspace,
                             size_t workspace_bytes, void *stream) {
  if (n_tiles < 0 || nf < 1) return APIC_EINVAL;
  if (n_tiles == 0) return APIC_OK;
  if (!field_r || !field_g || !field_b || !rgb_out) return APIC_EINVAL;
  if (!gains && (!workspace || workspace_bytes < sizeof(double) * 3 * kRgbBlocks ||
                 (reinterpret_cast<uintptr_t>(workspace) & 255) != 0))
    return APIC_EINVAL;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int64_t plane = (int64_t)nf * nf, count = plane * n_tiles;
  const c32 *fr = reinterpret_cast<const c32 *>(field_r);
  const c32 *fg = reinterpret_cast<const c32 *>(field_g);
  const c32 *fb = reinterpret_cast<const c32 *>(field_b);
  float g[3] = {1.f, 1.f, 1.f};
  if (gains) {
    for (int c = 0; c < 3; ++c) g[c] = gains[c];
  } else {
    double *partial = reinterpret_cast<double *>(workspace);
    hipLaunchKernelGGL(k_rgb_mean, dim3(kRgbBlocks), dim3(256), 0, st, fr, fg, fb, count,
                       partial);
    APIC_LAUNCHED();
    std::vector<double> host(3 * kRgbBlocks);
    APIC_HIP(hipStreamSynchronize(st));
    APIC_HIP(hipMemcpy(host.data(), partial, sizeof(double) * host.size(), hipMemcpyDeviceToHost));
    double m[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < kRgbBlocks; ++b)
      for (int c = 0; c < 3; ++c) m[c] += host[3 * b + c];
    const double mean = (m[0] + m[1] + m[2]) / 3.0;
    for (int c = 0; c < 3; ++c) g[c] = m[c] > 0.0 ? (float)(mean / m[c]) : 1.f;
  }
  if (gains_out)
    for (int c = 0; c < 3; ++c) gains_out[c] = g[c];
  const unsigned blocks = (unsigned)std::min<int64_t>(8192, (count + 255) / 256);
  hipLaunchKernelGGL(k_rgb_combine, dim3(blocks), dim3(256), 0, st, fr, fg, fb, plane, count,
                     g[0], g[1], g[2], rgb_out);
  APIC_LAUNCHED();
  return APIC_OK;
}
