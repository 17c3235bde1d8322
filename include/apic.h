/*
 * apic.h -- C ABI of the MI355X (gfx950) per-tile closed-form APIC
 * reconstruction (angular ptychographic imaging with closed-form solution,
 * as used for whole-slide scanning in arXiv 2407.20469).
 *
 * What the library computes, for every tile of a batch (paper Sec. 2.3, Fig. 2):
 *   1. Kramers-Kronig field recovery from each NA-matched image
 *      (Eq. 4-6: log, 2D FFT, half-plane mask, inverse FFT, exp; Eq. 7: FFT and
 *      pupil support);
 *   2. pupil-aberration estimate from the phase differences of overlapping
 *      spectra (Eq. 8-10), in the orthonormal Noll Zernike basis j = 4..15;
 *   3. aberration correction and stitching of the brightfield spectrum
 *      (text after Eq. 10);
 *   4. darkfield extension (Eq. 11-13): for each darkfield image in the order
 *      given, a regularised least-squares solve for the unknown part of the
 *      spectrum from the cross-correlation terms;
 *   5. the complex field on a grid upsampled by f (inverse FFT of the
 *      zero-embedded spectrum, times f^2).
 *
 * Conventions shared by every entry point
 *   - Arrays are row-major [y][x], x fastest.  Spectra are in FFT order (DC at
 *     [0][0]); a frequency index is the signed pair (ky, kx) in [-N/2, N/2)^2.
 *     DFTs are unnormalised forward (exp(-2 pi j k.n/N)) and 1/N^2 inverse.
 *   - Pupil radius r = na_obj * n * dx_um / wavelength_um bins;
 *     Circ(k) = [kx^2 + ky^2 <= r^2].
 *   - Illumination vectors are integer (kx, ky) DFT bins.  NA-matched ones must
 *     satisfy |k| <= r; every |k| + r must stay below N/2 (no wrap).
 *   - Zernike vectors are 15 floats per tile, Noll j = 1..15, RMS-normalised
 *     (radians); j = 1..3 (piston, tip, tilt) are outputs of 0 and ignored on
 *     input.  theta = atan2(ky, kx), rho = |k| / r.
 *   - Complex values are interleaved float pairs (complex64).
 *
 * Memory and ownership
 *   - Every data pointer (images, outputs, workspace, seeds) is DEVICE memory
 *     owned by the caller, except where an entry point says HOST (the slide
 *     streamer's image and field buffers, assembly positions and phases,
 *     colour gains).  apic_geometry and apic_tile_desc arrays are HOST
 *     memory, read during the call and not retained.  Exception:
 *     apic_batch_set_surrogate keeps the model's and the positions' device
 *     pointers until the surrogate is switched off or the batch destroyed.
 *   - A plan owns its host tables; it uploads its device tables on first use
 *     (or on apic_plan_upload) to the current device and owns them until
 *     apic_plan_destroy.  Calls never allocate: scratch comes from the
 *     caller's workspace, sized by apic_workspace_bytes.  The prepared
 *     objects are the exception, once, at creation: apic_batch_create
 *     (descriptor tables, streams), apic_streamer_create (staging buffers,
 *     pinned host staging, streams) and apic_assembly_create (pair and block
 *     lists); their destroy calls free it.
 *   - Calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *     stream) unless they say they synchronise.  A plan is immutable after
 *     upload; concurrent calls need separate workspaces.
 *
 * Errors
 *   - Argument errors return a negative apic_status before anything is
 *     enqueued.  HIP launch errors return APIC_EHIP.
 *   - Numerical conditions never fail a call: they set bits of the per-tile
 *     status word (APIC_TILE_*).
 */
#ifndef APIC_H
#define APIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  APIC_OK = 0,
  APIC_EINVAL = -1,       /* bad argument (null pointer, size, offset, workspace too small) */
  APIC_EUNSUPPORTED = -2, /* geometry outside what the kernels are built for, or a
                             configuration the call does not offer */
  APIC_EHIP = -3,         /* a HIP runtime call failed */
  APIC_ENOMEM = -4,       /* plan allocation failed */
  APIC_EPLAN = -5         /* plan invalid, corrupted, or not uploaded to this device */
} apic_status;

/* Per-tile status bits (uint32 per tile, OR-ed by the kernels). */
#define APIC_TILE_NONFINITE_INPUT 0x001u /* NaN/Inf in an NA-matched image            */
#define APIC_TILE_LOG_FLOOR       0x002u /* some intensity clamped to the log floor   */
#define APIC_TILE_PUPIL_ILLCOND   0x004u /* kappa(A) of Eq. 10's normal matrix > 1e6  */
#define APIC_TILE_PUPIL_CHOL_FAIL 0x008u /* non-positive pivot in the 12x12 solve     */
#define APIC_TILE_DF_CHOL_FAIL    0x010u /* non-positive pivot in a darkfield solve   */
#define APIC_TILE_DF_SKIPPED      0x020u /* a darkfield image had no unknowns         */
#define APIC_TILE_SEEDED          0x040u /* the pupil solve was re-wrapped on a seed  */
#define APIC_TILE_NONFINITE_OUT   0x080u /* NaN/Inf in the pupil coefficients         */
#define APIC_TILE_SURROGATE_USED  0x100u /* the surrogate's coefficients were used    */
#define APIC_TILE_FALLBACK_USED   0x200u /* the closed form replaced the surrogate    */
#define APIC_TILE_BACKGROUND      0x400u /* not reconstructed: background statistic
                                            under the threshold (slide stream)       */
#define APIC_TILE_PIXEL_NOT_CONVERGED 0x800u /* pixel-domain pupil solve stopped at
                                                max_iter before its tolerance        */

/* Tile flags (apic_tile_desc.flags). */
#define APIC_TILE_SKIP_DARKFIELD 0x1  /* stop after the brightfield stitch */

typedef struct apic_plan apic_plan; /* opaque */

/* One geometry class (host memory; copied by apic_plan_create). */
typedef struct {
  int32_t n;               /* tile side N: 64, 128, 256 or 512                     */
  int32_t upsample;        /* output factor f: 1 or 2 (f*N <= 1024)                 */
  double dx_um;            /* sample-plane pixel pitch                              */
  double wavelength_um;    /* illumination wavelength                               */
  double na_obj;           /* objective NA                                          */
  int32_t n_bf;            /* NA-matched images, 4..32                              */
  int32_t n_df;            /* darkfield images, 0..64                               */
  const int32_t *k_bf;     /* [n_bf][2] (kx, ky) bins                               */
  const int32_t *k_df;     /* [n_df][2] (kx, ky) bins, in processing order         */
  double ridge_pupil;      /* mu: ridge mu * tr(A)/12 in Eq. 10 (default 1e-9)      */
  double ridge_darkfield;  /* lambda: ridge lambda * tr(G)/N_u in Eq. 13 (1e-4)     */
  double log_floor_rel;    /* eps = log_floor_rel * mean(I) before the log (1e-6)   */
  int32_t pupil_bands;     /* 1 (default): solve Eq. 10 coarse to fine, first on the
                              rows with |K| <= f r for f = 0.05, 0.1, 0.2, 0.4, 0.8,
                              1.6 (bands of fewer than 32 rows skipped), each band
                              re-wrapping beta about the previous band's solution
                              (the seeded variant) and solved with a ridge of
                              0.1 tr(A)/12, then on every row; phase
                              differences near K = 0 stay unwrapped however large
                              the aberration.  0: the single pass of Eq. 10.
                              Without effect when a seed is given.               */
} apic_geometry;

/* One tile of a batch (host memory). */
typedef struct {
  int32_t geom;            /* index into the plan's geometry list                   */
  int32_t flags;           /* APIC_TILE_SKIP_DARKFIELD                              */
  int64_t image_offset;    /* float elements into `images` of this tile's stack of
                              n_bf + n_df images [img][N][N], NA-matched first     */
  int64_t field_offset;    /* complex elements into the tile's output array:
                              fN x fN field (reconstruct, upsample) or N x N
                              spectrum (stitch, extend_darkfield)                  */
  float pos_x, pos_y;      /* normalised field position in [-1, 1]                  */
} apic_tile_desc;

/* Build a plan for n_geom geometry classes (host work only; no GPU needed).
 * Returns APIC_EUNSUPPORTED for sizes the kernels do not cover. */
apic_status apic_plan_create(const apic_geometry *geoms, int32_t n_geom, apic_plan **out);

/* Free the plan and its device tables.  NULL is accepted. */
apic_status apic_plan_destroy(apic_plan *plan);

/* Upload the plan's device tables to the current device (idempotent). */
apic_status apic_plan_upload(apic_plan *plan);

/* Workspace bytes a call over these tiles needs (same for every entry point). */
apic_status apic_workspace_bytes(const apic_plan *plan, int32_t n_tiles,
                                 const apic_tile_desc *tiles, size_t *bytes);

/* Plan-introspection for host-side tests: copies a plan table of geometry
 * `geom` into `out` (int32 values, capacity `cap`), returns its length in *len.
 *   what = 0: darkfield step j's unknown set U      (ky, kx pairs)
 *          1: darkfield step j's known set P        (ky, kx pairs)
 *          2: darkfield step j's linear region Q    (ky, kx pairs)
 *          3: darkfield step j's excluded set E     (ky, kx pairs)
 *          4: pupil rows (i, l, ky, kx, cell) quintuples over all pairs, in
 *             the plan's order: sorted (stably) by the first band of the
 *             pupil continuation that holds them
 *          7: row counts of the continuation's band passes (empty when
 *             pupil_bands is 0)
 *          5: sizes: n_pairs, n_rows, nu_max, m_max, ne_max, n_active_steps,
 *             unknowns per gram block, E rows per gram chunk, pupil pixels
 *          6: per darkfield step (N_u, |Q|, |E|, live gram work of all lower
 *             block pairs, of the diagonal blocks), the work counted in
 *             (16 x 16 quadrant, excluded k) pairs, i.e. in units of 256
 *             complex MACs: the products the gram issues; U and E
 *             are in the plan's processing order (compact squares), P and Q
 *             in FFT raster order
 *          8: per darkfield step the signed row spans (ky) the FFT passes
 *             of that step are restricted to: (lo, hi) of P + U, of Q, and
 *             of the rows where fft2(|P|^2 + i I_j) is read (Q, -Q and the
 *             row differences of U); (0, -1) for an empty span and for
 *             steps without unknowns */
apic_status apic_plan_query(const apic_plan *plan, int32_t geom, int32_t what, int32_t j,
                            int32_t *out, int64_t cap, int64_t *len);

/* Whole method: KK -> pupil -> stitch -> darkfield -> fN x fN field
 * (paper Sec. 2.3 and Fig. 2: Eq. 4-7 field recovery, Eq. 8-10 aberration
 * correction, Eq. 11-13 darkfield extension, then the up-sampled field).
 *   images        float   [per tile: n_bf + n_df][N][N]   (device, at image_offset)
 *   zernike_seed  float   [T][15] or NULL: re-wrap the pupil phases around it
 *   zernike_out   float   [T][15]
 *   field_out     complex [per tile: fN][fN]             (at field_offset)
 *   tile_status   uint32  [T]  (zeroed by the call, then OR-ed) */
apic_status apic_reconstruct_tiles(const apic_plan *plan, int32_t n_tiles,
                                   const apic_tile_desc *tiles, const float *images,
                                   const float *zernike_seed, float *zernike_out,
                                   float *field_out, uint32_t *tile_status, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* apic_reconstruct_tiles without a caller workspace, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The scratch is one static device array of
 * APIC_STATIC_SCRATCH_BYTES (256 MiB) per GPU, held from the first call on
 * that GPU until the process ends; the call itself allocates nothing and
 * copies nothing from the host.  Arguments as apic_reconstruct_tiles.
 * Preconditions, checked before anything is enqueued:
 *   - the plan was uploaded to the current device (apic_plan_upload, which
 *     allocates the plan's tables): else APIC_EPLAN;
 *   - the workspace the tiles need (apic_workspace_bytes) fits the array:
 *     else APIC_ENOMEM (e.g. 8 tiles of 256^2 with 16 + 32 images fit);
 *   - the descriptors of each geometry class are regular (tile t of the
 *     class at base + t * step in images, outputs and batch index; any list
 *     of one or two tiles is): irregular lists would need a host copy, so
 *     they return APIC_EUNSUPPORTED.
 * Every call on a GPU uses that GPU's one array, which keeps the last call's
 * contents (nothing in it needs clearing: every kernel writes what it later
 * reads); calls that overlap on one GPU (several streams or threads) race. */
#define APIC_STATIC_SCRATCH_BYTES (256ll << 20)
apic_status apic_reconstruct_tiles_static(const apic_plan *plan, int32_t n_tiles,
                                          const apic_tile_desc *tiles, const float *images,
                                          const float *zernike_seed, float *zernike_out,
                                          float *field_out, uint32_t *tile_status, void *stream);

/* Fig. 2 upper half, Eq. 4-10 only.
 *   diag_out      float [T][4]: linearised residual R(c) (rad^2), kappa(A),
 *                 total weight sum w, smallest Cholesky pivot
 *   features_out  float [T][32] or NULL: log1p of the weight sums per
 *                 (pair-angle bin 0..7) x (|K|/(2r) band 0..3), over N^4 */
apic_status apic_estimate_pupil(const apic_plan *plan, int32_t n_tiles,
                                const apic_tile_desc *tiles, const float *images,
                                const float *zernike_seed, float *zernike_out, float *diag_out,
                                float *features_out, uint32_t *tile_status, void *workspace,
                                size_t workspace_bytes, void *stream);

/* Eq. 10 as the paper writes it: one unknown per pupil pixel.  phi(k) for
 * every integer k with kx^2 + ky^2 <= r^2, rows phi(K+K_i) - phi(K+K_l) -
 * phi(K_i) + phi(K_l) = beta over the same pairs, K, phase differences and
 * weights as apic_estimate_pupil.  The paper names no solver; phi is the
 * minimum-norm weighted least-squares solution (no piston, tip or tilt, nor
 * any other component the rows cannot see), computed per tile by conjugate
 * gradients on the normal equations from phi = 0, stopped when the residual
 * norm falls under tol (0 < tol < 1) times its first value or after max_iter
 * iterations (status APIC_TILE_PIXEL_NOT_CONVERGED).
 *   phi_out      float [T][N][N] in FFT order, 0 outside the pupil
 *                (contiguous per tile at phi_out + t * N * N)
 *   zernike_out  float [T][15]: least-squares fit of Noll Z_1..Z_15 to phi
 *                over the pupil pixels, c_1..c_3 reported as 0
 *   iters_out    int32 [T] or NULL: iterations taken
 * Single-geometry plans (APIC_EUNSUPPORTED otherwise); every valid plan's
 * pupil (4r < N, N fN <= 1024) stays under the 65536 pupil pixels the
 * tables' 16-bit indices allow.  Up to 7936 pupil pixels (N <= 256)
 * one workgroup per tile holds the CG vectors in LDS; beyond that the
 * vectors stay in the workspace, the row passes are spread over many
 * workgroups per tile (FP64 atomics in L2), and the call waits on the host
 * every 32 iterations to stop once every tile has converged. */
apic_status apic_estimate_pupil_pixel(const apic_plan *plan, int32_t n_tiles,
                                      const apic_tile_desc *tiles, const float *images,
                                      double tol, int32_t max_iter, float *phi_out,
                                      float *zernike_out, int32_t *iters_out,
                                      uint32_t *tile_status, void *workspace,
                                      size_t workspace_bytes, void *stream);

/* Background statistic of each tile (Sec. 3.2, reconstruction time of the
 * slide: patches whose low-resolution images vary less than a threshold are
 * treated as empty glass and skipped).  The paper gives neither the exact
 * statistic nor the threshold; here it is the mean over the tile's NA-matched
 * images of var(I_i) / mean(I_i)^2 (population variance over the N x N
 * pixels, FP64 accumulation), which does not depend on LED brightness or
 * exposure.  stat_out float [T] (device, batch order).  `images` must be
 * 16-byte aligned and every image_offset a multiple of 4 (else APIC_EINVAL).
 * The workspace (apic_workspace_bytes) only holds descriptor lists. */
apic_status apic_background_stat(const apic_plan *plan, int32_t n_tiles,
                                 const apic_tile_desc *tiles, const float *images,
                                 float *stat_out, void *workspace, size_t workspace_bytes,
                                 void *stream);

/* KK spectra of the NA-matched images (Eq. 4-7), complex [T][n_bf][N][N]
 * contiguous per tile at spectra_out + t * n_bf * N * N (single geometry). */
apic_status apic_kk_spectra(const apic_plan *plan, int32_t n_tiles,
                            const apic_tile_desc *tiles, const float *images,
                            float *spectra_out, uint32_t *tile_status, void *workspace,
                            size_t workspace_bytes, void *stream);

/* Corrected, stitched brightfield spectrum (text after Eq. 10) for given
 * Zernike coefficients: complex N x N per tile at field_offset of spectrum_out. */
apic_status apic_stitch_brightfield(const apic_plan *plan, int32_t n_tiles,
                                    const apic_tile_desc *tiles, const float *images,
                                    const float *zernike, float *spectrum_out,
                                    uint32_t *tile_status, void *workspace,
                                    size_t workspace_bytes, void *stream);

/* Fig. 2 lower half, Eq. 11-13: extend each tile's stitched brightfield
 * spectrum (complex N x N at field_offset of spectrum_inout, zero outside the
 * brightfield known set) through every darkfield image, in place. */
apic_status apic_extend_darkfield(const apic_plan *plan, int32_t n_tiles,
                                  const apic_tile_desc *tiles, const float *images,
                                  const float *zernike, float *spectrum_inout,
                                  uint32_t *tile_status, void *workspace,
                                  size_t workspace_bytes, void *stream);

/* fN x fN field from an N x N spectrum (zero embedding, inverse FFT, f^2):
 * reads tile t's spectrum at spectrum_in + t * N * N (contiguous per tile,
 * single geometry), writes the field at field_offset of field_out. */
apic_status apic_upsample_field(const apic_plan *plan, int32_t n_tiles,
                                const apic_tile_desc *tiles, const float *spectrum_in,
                                float *field_out, void *workspace, size_t workspace_bytes,
                                void *stream);

/* Batched 2D complex FFT of `batch` contiguous L x L arrays, L in
 * {64, 128, 256, 512, 1024}, unnormalised in both directions, out of place
 * allowed (in == out allowed).  Precision: 0 = complex64, 1 = complex128. */
apic_status apic_fft2(int32_t l, int32_t batch, int32_t inverse, int32_t precision,
                      const void *in, void *out, void *stream);

/* ---------------------------------------------------------------- batches
 * A prepared batch of tiles (tile batcher).  apic_batch_create groups the
 * tiles by geometry class and copies their descriptors to device memory owned
 * by the batch (needs the device; call it outside any graph capture), and
 * creates one default-priority side stream per class.  apic_batch_reconstruct
 * then enqueues the whole method with no host synchronisation, copy or
 * allocation: the classes run concurrently on the side streams, forked from
 * and joined back to `stream` with events, so an uneven batch of mixed tile
 * sizes and LED counts overlaps its classes.  apic_batch_capture records one
 * such call on `stream` (not the NULL stream) into a graph owned by the batch;
 * apic_batch_launch replays it (same buffers; contents may change between
 * replays); it returns APIC_EUNSUPPORTED, before any capture starts, for a
 * batch with a two-lane class (apic_batch_set_chunk) or with the surrogate on
 * (apic_batch_set_surrogate), which run eagerly only.  Outputs and workspace
 * as apic_reconstruct_tiles; the workspace
 * size is apic_batch_workspace_bytes.  A batch keeps a pointer to its plan:
 * destroy the batch first. */
typedef struct apic_batch apic_batch;
apic_status apic_batch_create(apic_plan *plan, int32_t n_tiles, const apic_tile_desc *tiles,
                              apic_batch **out);
apic_status apic_batch_destroy(apic_batch *batch);
apic_status apic_batch_workspace_bytes(const apic_batch *batch, size_t *bytes);
apic_status apic_batch_reconstruct(apic_batch *batch, const float *images,
                                   const float *zernike_seed, float *zernike_out, float *field_out,
                                   uint32_t *tile_status, void *workspace, size_t workspace_bytes,
                                   void *stream);
apic_status apic_batch_capture(apic_batch *batch, const float *images, const float *zernike_seed,
                               float *zernike_out, float *field_out, uint32_t *tile_status,
                               void *workspace, size_t workspace_bytes, void *stream);
apic_status apic_batch_launch(apic_batch *batch, void *stream);

/* Classes of a batch, in the order the batch runs them: on entry *n_classes
 * is the capacity of the (nullable) arrays, on return the class count; per
 * class its geometry index, tile count, current chunk (tiles per launch
 * sequence), lanes and workspace bytes per tile. */
apic_status apic_batch_classes(const apic_batch *batch, int32_t *n_classes, int32_t *geom,
                               int32_t *n_tiles, int32_t *chunk, int32_t *lanes,
                               int64_t *tile_bytes);
/* Run class `cls` in chunks of `tiles` tiles (<= 0: the whole class at once)
 * on `lanes` (1 or 2) streams: with one lane the chunks run one after another
 * reusing one chunk's workspace; with two they alternate between the class's
 * stream and a second default-priority stream, each with its own chunk
 * workspace, so one chunk's latency-bound kernels (the diagonal Cholesky
 * factors) overlap the other's.  Changes apic_batch_workspace_bytes and drops
 * a captured graph. */
apic_status apic_batch_set_chunk(apic_batch *batch, int32_t cls, int32_t tiles, int32_t lanes);
/* LDS tiling of class `cls`'s FFT column passes: variant 0 takes panels of
 * up to 16 adjacent columns and 2048 elements per workgroup, variant 1 panels
 * twice as wide (when the panel stays within 64 KiB of LDS and 16 columns,
 * else half as wide).  Each column's transform is the same either way, so the
 * results are identical; only the access pattern and the workgroup count
 * change.  apic_batch_fft_panel reports a class's variant and its panel width
 * in columns for complex128 passes of the class's N.  Drops a captured graph;
 * APIC_EINVAL for a bad class or variant. */
apic_status apic_batch_set_fft(apic_batch *batch, int32_t cls, int32_t variant);
apic_status apic_batch_fft_panel(const apic_batch *batch, int32_t cls, int32_t *variant,
                                 int32_t *panel_columns);
/* Autotuner.  For class `cls` (all classes when cls < 0), times the method
 * (with the surrogate stage when apic_batch_set_surrogate switched it on) on
 * its first k tiles for k = 1, 2, 4, ... up to the class size, as long as k
 * tiles' workspace fits `workspace_bytes` (and stops once doubling k gains
 * under 3% past k = 4, or after a run longer than 10 s).  It then sets the
 * class's chunk to the smallest k whose time per tile is within (1 + slack)
 * of the best, tries two lanes of half that chunk over the same tiles (same
 * workspace) and keeps them if 2% faster, then times the class's FFT column
 * passes with their two panel widths (apic_batch_set_fft) over the chosen
 * chunk and keeps the alternative if 2% faster.  If the classes' chunk blocks
 * together exceed `workspace_bytes` (they run concurrently), the largest
 * blocks are halved until they fit.
 * Synchronises the host with `stream` after every run (not
 * capturable); writes outputs and status of the timed tiles.  `ms_per_tile`
 * (nullable, one per class, indexed by class) receives the best time.  Changes
 * apic_batch_workspace_bytes and drops a captured graph. */
apic_status apic_batch_autotune(apic_batch *batch, int32_t cls, const float *images,
                                float *zernike_out, float *field_out, uint32_t *tile_status,
                                void *workspace, size_t workspace_bytes, void *stream,
                                double slack, double *ms_per_tile);
/* Halve the largest classes' chunks until the classes' blocks together fit
 * `workspace_bytes` (done by apic_batch_autotune when cls < 0; call it after
 * tuning classes one by one).  APIC_EINVAL if one tile per class does not fit. */
apic_status apic_batch_fit(apic_batch *batch, size_t workspace_bytes);

/* ---------------------------------------------------------- patch assembly
 * Tiles placed at known canvas positions with blended overlaps (Sec. 2.5:
 * adjacent scans keep overlapping regions, blended to hide the seams; a tile
 * with no neighbour is placed by its scan position).  Registration by image
 * features is not done here: positions are given.
 * apic_assembly_create takes the layout: n_tiles tiles of side n, pos int32
 * [T][2] (host; canvas row and column of each tile's [0][0]; tiles may reach
 * outside the canvas), the pairs sharing at least min_overlap rows and
 * columns, and a canvas of canvas_h x canvas_w; it builds the overlapping
 * pairs and, per 32 x 32 canvas block, the covering tiles, and copies them to
 * device memory it owns (needs the device; not capturable).
 *   fields  complex64 [T][n][n] (device), tile t at fields + 2 * t * n * n
 *           (e.g. the fN x fN fields of a single-geometry reconstruction)
 * Every reconstructed tile carries its own constant phase (KK fixes each
 * tile's DC phase), so tiles are brought to a common phase first.
 * apic_assemble_phases: C_tu = sum over the overlap of F_t conj(F_u) for every
 * pair (FP64 sums on the GPU); then, on the host, theta = the phases of the
 * leading eigenvector of C (angular synchronisation) per connected group of
 * overlapping tiles, the group's lowest-numbered tile at 0 (a tile with no
 * neighbour gets 0).  theta_out float [T] (host).  Synchronises the host with
 * `stream`.
 * apic_blend: canvas(p) = sum_t w_t(p) F_t(p) exp(-j theta_t) / sum_t w_t(p)
 * (0 where no tile covers p), w = ramp(y) ramp(x) over each tile, ramp(v) =
 * min(1, (v + 1/2) / R, (n - v - 1/2) / R), R = ramp_width >= 1; theta
 * float [T] (DEVICE) or NULL (all 0); canvas complex64 [canvas_h][canvas_w]
 * (device).  One kernel launch, no host work: capturable. */
typedef struct apic_assembly apic_assembly;
apic_status apic_assembly_create(int32_t n_tiles, int32_t n, const int32_t *pos,
                                 int32_t min_overlap, int32_t canvas_h, int32_t canvas_w,
                                 apic_assembly **out);
apic_status apic_assembly_destroy(apic_assembly *assembly);
apic_status apic_assemble_phases(apic_assembly *assembly, const float *fields, float *theta_out,
                                 void *stream);
apic_status apic_blend(const apic_assembly *assembly, const float *fields, const float *theta,
                       float ramp_width, float *canvas, void *stream);

/* ------------------------------------------------------------ colour image
 * Sec. 3.3: for a stained slide the method runs once per colour channel (one
 * geometry per wavelength); the amplitudes of the three reconstructed fields
 * are combined and white balanced.  field_r/_g/_b complex64 [T][nf][nf]
 * (device, same layout); rgb_out float [T][3][nf][nf] (device, planar per
 * tile) = g_c |F_c|.  gains float [3] (host) or NULL for grey world: g_c =
 * mean_c' m_c' / m_c with m_c the mean amplitude of channel c over all pixels
 * (FP64 sums on the GPU; needs a workspace of 3 * 1024 doubles, 256-byte
 * aligned, and synchronises the host with `stream`).  gains_out float [3]
 * (host, nullable) receives the gains used. */
apic_status apic_rgb_combine(int32_t n_tiles, int32_t nf, const float *field_r,
                             const float *field_g, const float *field_b, const float *gains,
                             float *rgb_out, float *gains_out, void *workspace,
                             size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------- surrogate
 * Learned Zernike surrogate (not part of the paper's method): a perceptron
 * 34 -> 128 -> 128 -> 12 (ReLU) from (tile x, tile y, the 32 features of
 * apic_estimate_pupil) to c_4..c_15, bfloat16 operands on the matrix cores with
 * FP32 accumulation.  Parameters are one FP32 vector of APIC_MLP_PARAMS
 * values: W1[128][64] (input columns >= 34 unused), b1[128], W2[128][128],
 * b2[128], W3[16][128] (rows >= 12 unused), b3[16].  Inputs are normalised as
 * (x - in_mean) / in_std before use. */
#define APIC_MLP_PARAMS 26896
#define APIC_MLP_INPUTS 34
#define APIC_MLP_OUTPUTS 12
typedef struct {
  const float *theta;    /* [APIC_MLP_PARAMS] device */
  const float *in_mean;  /* [34] device */
  const float *in_std;   /* [34] device */
  int32_t seeds_solve;   /* pupil stages only.  0: the closed form (the
                            continuation of apic_geometry.pupil_bands, or one
                            pass seeded by the caller's zernike_seed) runs as
                            usual and the surrogate's prediction competes with
                            it.  1: the prediction seeds the solve instead (a
                            plain pass over the rows gives the features, then
                            one pass re-wrapped about the prediction, Eq. 10's
                            seeded variant); the closed form that results
                            judges the prediction.  A caller's zernike_seed is
                            not accepted with 1 (APIC_EINVAL).  In either case
                            both candidates are judged on the final pass's
                            sums, R(c - c0) with c0 that pass's seed.         */
} apic_mlp_model;

/* outputs[n][12] = network(inputs[n][34]). */
apic_status apic_mlp_forward(const apic_mlp_model *model, int32_t n, const float *inputs,
                             float *outputs, void *stream);

/* `steps` Adam steps (beta 0.9 / 0.999, eps 1e-8, learning rate lr) of the
 * mean-squared error against targets[n][12], in one single-workgroup launch.
 * order[steps * batch] lists the sample of each slot (-1 = empty slot); t0 is
 * the number of Adam steps already applied to (theta, adam_m, adam_v).  grad
 * [APIC_MLP_PARAMS] is scratch; loss_out[steps] receives each step's loss
 * (or NULL).  All pointers device memory; theta, adam_m, adam_v updated. */
apic_status apic_mlp_train(float *theta, float *adam_m, float *adam_v, float *grad,
                           const float *in_mean, const float *in_std, int32_t n,
                           const float *inputs, const float *targets, const int32_t *order,
                           int32_t steps, int32_t batch, int32_t t0, float lr, float *loss_out,
                           void *stream);

/* Gradient of the loss over the samples order[0..batch) into grad, no update. */
apic_status apic_mlp_grad(const float *theta, float *grad, const float *in_mean,
                          const float *in_std, int32_t n, const float *inputs,
                          const float *targets, const int32_t *order, int32_t batch,
                          float *loss_out, void *stream);

/* Utility for checking the matrix-core operand layout: c[m][n] = a[m][k] b[k][n],
 * bfloat16 row-major a and b (uint16 bit patterns), FP32 c; m, n, k in
 * {16, 32, 48, 64}. */
apic_status apic_bf16_gemm(int32_t m, int32_t n, int32_t k, const uint16_t *a, const uint16_t *b,
                           float *c, void *stream);

/* apic_estimate_pupil with the surrogate: positions[T][2] (device, batch
 * order) are the surrogate's tile coordinates.  For each tile the closed-form
 * solve and the surrogate both run; rho = sqrt(max(0, R(c_sur) - R(c_cf)))
 * with R the weighted linearised residual of Eq. 10; the closed form is kept
 * when rho > rho_max, kappa(A) <= kappa_max and R(c_cf) <= resid_max, the
 * surrogate otherwise (status APIC_TILE_FALLBACK_USED / _SURROGATE_USED).
 * zernike_cf_out and zernike_sur_out ([T][15], may be NULL) receive both
 * candidates; zernike_out the chosen one. */
apic_status apic_estimate_pupil_sur(const apic_plan *plan, int32_t n_tiles,
                                    const apic_tile_desc *tiles, const float *images,
                                    const float *positions, const apic_mlp_model *model,
                                    float rho_max, float kappa_max, float resid_max,
                                    float *zernike_out, float *zernike_cf_out,
                                    float *zernike_sur_out,
                                    float *diag_out, uint32_t *tile_status, void *workspace,
                                    size_t workspace_bytes, void *stream);

/* apic_reconstruct_tiles with the surrogate choosing the pupil as above. */
apic_status apic_reconstruct_tiles_sur(const apic_plan *plan, int32_t n_tiles,
                                       const apic_tile_desc *tiles, const float *images,
                                       const float *positions, const apic_mlp_model *model,
                                       float rho_max, float kappa_max, float resid_max,
                                       float *zernike_out, float *field_out,
                                       uint32_t *tile_status, void *workspace,
                                       size_t workspace_bytes, void *stream);

/* A prepared batch with the surrogate choosing each tile's pupil by the rule
 * of apic_estimate_pupil_sur (learned prior of the paper's discussion section,
 * checked against the closed form of Eq. 10).  After this call every
 * apic_batch_reconstruct, apic_batch_capture and apic_batch_autotune on
 * `batch` runs the surrogate and the fallback test between the pupil solve
 * and the stitching (apic_batch_capture refuses such a batch); model == NULL
 * switches it off again.  `positions`
 * float [T][2] (device, indexed by the batch's tile index) and the model's
 * device buffers are borrowed, not copied: they must stay valid, and may
 * change contents, while the batch uses them.  Drops a captured graph.
 * APIC_EINVAL for a bad batch, a malformed model, or a model without
 * positions. */
apic_status apic_batch_set_surrogate(apic_batch *batch, const apic_mlp_model *model,
                                     const float *positions, float rho_max, float kappa_max,
                                     float resid_max);

/* ------------------------------------------------------------- slide stream
 * Whole-slide scanning (Sec. 2.5 and 3.2: a slide is scanned tile by tile and
 * each patch is reconstructed independently; background patches are skipped):
 * tiles of one geometry whose images live in HOST memory are reconstructed in
 * chunks through device staging buffers.  apic_streamer_create allocates, for
 * each of `n_buffers` (2..4) default-priority streams, device room for `chunk`
 * tiles of geometry `geom` (image stacks, fields, coefficients, status,
 * statistic) plus that chunk's workspace, and pinned host staging for the
 * small per-tile arrays; apic_streamer_device_bytes reports the device total;
 * apic_streamer_destroy frees everything.  The streamer keeps a pointer to its
 * plan: destroy it first.  One streamer runs one apic_streamer_run at a time. */
typedef struct apic_streamer apic_streamer;
apic_status apic_streamer_create(apic_plan *plan, int32_t geom, int32_t chunk, int32_t n_buffers,
                                 apic_streamer **out);
apic_status apic_streamer_destroy(apic_streamer *streamer);
apic_status apic_streamer_device_bytes(const apic_streamer *streamer, size_t *bytes);
/* Reconstruct n_tiles tiles from host memory; returns when every tile is done.
 *   host_images[t]  float [n_bf + n_df][N][N] of tile t (host; pinned memory,
 *                   e.g. hipHostMalloc, for asynchronous full-speed copies;
 *                   tiles may share one buffer)
 *   host_fields[t]  complex64 [fN][fN] output of tile t (host, pinned)
 *   positions       float [T][2] (host) tile coordinates for the surrogate;
 *                   needed when model is not NULL
 *   zernike_out     float [T][15], tile_status uint32 [T], bg_stat_out float
 *                   [T] (nullable): host arrays
 * Chunk c (tiles c*chunk ...) runs on buffer c mod n_buffers: copy in,
 * apic_background_stat, the method on the chunk's tiles whose statistic is
 * >= bg_threshold, copy out.  The host enqueues chunk c's copy-in and
 * statistic, then waits for chunk c-1's statistic (a few bytes) and enqueues
 * its method, so copies overlap the kernels of the chunks in flight.  A tile
 * under the threshold (bg_threshold <= 0 disables the test) gets status
 * APIC_TILE_BACKGROUND and zero coefficients; its field buffer is not
 * written.  With `model` the pupil stage is apic_reconstruct_tiles_sur's
 * (rho_max, kappa_max, resid_max as there), else apic_reconstruct_tiles's;
 * results are those calls' on the same tiles.  Not capturable.  On an error
 * return every stream has been drained; outputs are then incomplete. */
apic_status apic_streamer_run(apic_streamer *streamer, int32_t n_tiles,
                              const float *const *host_images, float *const *host_fields,
                              const float *positions, const apic_mlp_model *model, float rho_max,
                              float kappa_max, float resid_max, float bg_threshold,
                              float *zernike_out, uint32_t *tile_status, float *bg_stat_out);

/* Opt-in profiling of kernel groups (for benchmarks).  apic_profile(1) clears
 * and enables recording: every later launch of a group records a HIP event
 * pair on the call's stream plus the group's algorithmic work; apic_profile(0)
 * stops recording (and clears).  apic_profile_read waits for the recorded
 * events and returns the summed duration, the number of recorded launches
 * and the summed work of one group.  Work is flops for the FP64 groups
 * (GRAM: 8 flops per complex MAC of the Hermitian E-sum; CHOL: (4/3) n^3 +
 * 8 n^2) and compulsory HBM bytes for the others.  Recording creates HIP
 * events, so it is not meant for graph capture. */
#define APIC_PROF_KK 0     /* statistics + 4 fused KK passes        (bytes) */
#define APIC_PROF_PUPIL 1  /* pupil rows, reduction, 12x12 solves   (bytes) */
#define APIC_PROF_STITCH 2 /* correction + stitching                (bytes) */
#define APIC_PROF_DF_FFT 3 /* P_hat, FP64 |P|^2 chain, image FFT    (bytes) */
#define APIC_PROF_DF_RHS 4 /* b on Q and C^H b                      (bytes) */
#define APIC_PROF_GRAM 5   /* darkfield gram                        (flops) */
#define APIC_PROF_CHOL 6   /* darkfield Cholesky + solves           (flops) */
#define APIC_PROF_OUT 7    /* embedding + upsampled inverse FFT     (bytes) */
#define APIC_PROF_GROUPS 8
apic_status apic_profile(int32_t enable);
apic_status apic_profile_read(int32_t group, double *total_ms, int64_t *launches,
                              double *total_work);

/* Measurement probes (roofline reporting, not part of the method).
 * apic_calib_fma64: `blocks` x 256 threads, each `iters` x 128 dependent-free
 *   FP64 FMAs (8 chains), writing one double per thread to out[blocks * 256];
 *   flops = blocks * 256 * iters * 256.
 * apic_calib_mfma64: the same on the FP64 matrix cores: `blocks` x 4 waves,
 *   each `iters` x 8 independent 16 x 16 x 4 FP64 matrix products
 *   (v_mfma_f64_16x16x4f64), one double per thread to out[blocks * 256];
 *   flops = blocks * 4 * iters * 8 * 2048.
 * apic_calib_copy: copies `bytes` (multiple of 16) from `in` to `out` with a
 *   grid-stride 16-byte loop; HBM traffic is bytes read + bytes written. */
apic_status apic_calib_fma64(double *out, int32_t blocks, int32_t iters, void *stream);
apic_status apic_calib_mfma64(double *out, int32_t blocks, int32_t iters, void *stream);
apic_status apic_calib_copy(const void *in, void *out, int64_t bytes, void *stream);

/* Library version string. */
const char *apic_version(void);

#ifdef __cplusplus
}
#endif
#endif /* APIC_H */
