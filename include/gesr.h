/* gesr.h — C ABI of the generalized-exponential-splat (GES) rasterizer for
 * AMD Instinct MI355X (gfx950).
 *
 * The library implements the differentiable rasterizer of DyGASR (arXiv
 * 2411.09156): each 3-D splat with shape parameter beta (epsilon in the paper,
 * Sec. 3.2, Eq. 1-3) is projected to a screen-space conic (Eq. 4 and the
 * Sigma' = J W Sigma W^T J^T passage, with the shape-modulated scale of
 * Eq. 6-7), binned into screen tiles, and alpha-composited front to back
 * (Eq. 5 evaluated as discrete alpha blending); the backward pass returns
 * gradients for position, scale, rotation, opacity, beta and SH colour.
 *
 * Conventions for every entry point
 *  - Array pointers marked DEVICE are device memory owned by the caller; the
 *    library never allocates, frees or retains them past the call.  HOST
 *    pointers are read during the call only.
 *  - All device work is enqueued on `stream` (a hipStream_t; NULL = default
 *    stream).  Calls return after enqueueing, except where a synchronous
 *    capacity check is requested (gesr_bin with GESR_BIN_SYNC).
 *  - Arguments are validated on the host before anything is enqueued.  An
 *    invalid argument returns GESR_ERR_INVALID and enqueues nothing; the
 *    message is available from gesr_last_error(ctx).
 *  - A HIP launch or copy failure returns GESR_ERR_HIP.  An asynchronous
 *    device fault surfaces as GESR_ERR_HIP from a later call.
 *  - Device pointers must be 16-byte aligned (torch allocations are).
 *  - A context is not thread-safe; use one per host thread.
 *  - Per-(view, splat) arrays are indexed vi = view * n + splat.
 *  - Images are float32, CHW per view, views concatenated in order.
 */
#ifndef GESR_H
#define GESR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GESR_OK = 0,
    GESR_ERR_INVALID = 1,     /* bad argument; nothing enqueued */
    GESR_ERR_CAPACITY = 2,    /* instance count exceeds bins->m_cap (see gesr_bin), or the
                                 static scratch (gesr_bin_static) */
    GESR_ERR_HIP = 3,         /* HIP runtime error */
    GESR_ERR_UNSUPPORTED = 4  /* valid but not supported by the library (e.g. tile shape) */
} gesr_status;

#define GESR_MAX_VIEWS 32
#define GESR_REC_FLOATS 16    /* floats per projected record (one 64-byte line) */
#define GESR_PARTIAL_FLOATS 10 /* colour and footprint terms of a gradient partial (du .. db) */
#define GESR_GRAD2D_FLOATS 12  /* floats per grad2d row and per instance partial: the ten
                                  terms, dz (depth channel, 0 without it) and a zero pad */

typedef struct gesr_ctx gesr_ctx;

/* Creates a context bound to HIP device `device`.  Host-only: no device
 * memory is allocated.  Returns GESR_ERR_INVALID for a NULL `out`. */
gesr_status gesr_ctx_create(int device, gesr_ctx** out);
void gesr_ctx_destroy(gesr_ctx* ctx);
/* Message of the last non-OK status returned on `ctx` ("" if none). */
const char* gesr_last_error(const gesr_ctx* ctx);
const char* gesr_status_string(gesr_status s);

/* Pinhole camera, OpenCV axes (x right, y down, z forward).  A pixel (i, j)
 * has its centre at (i + 1/2, j + 1/2). */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
    float viewmat[12]; /* world -> camera [R | t], row-major 3x4 (W of Sec. 3.2) */
    float campos[3];   /* camera centre in world coordinates (SH view direction) */
} gesr_camera;

/* Rasterizer constants.  gesr_default_settings() fills the defaults:
 *  kappa = 0.5   falloff exp(-kappa q^(beta/2)); 1/2 reproduces Eq. 3
 *  rho = 0.1     shape strength of Eq. 7 (value of Sec. 4.2), read as
 *                phi = 2 / (1 + exp(-rho (beta - 2)))
 *  alpha_min = 1/255, alpha_max = 0.99, t_min = 1e-4  blending thresholds
 *  blur = 0.3 (px^2 added to Sigma'), znear = 0.2, clip_fac = 1.3
 *  bg = (0, 0, 0)
 *  tile_w = tile_h = 16; batch = 0 (automatic); radix_bits = 8. */
typedef struct {
    int32_t sh_degree; /* 0..3; K = (sh_degree + 1)^2 coefficients per channel */
    float kappa, rho;
    float alpha_min, alpha_max, t_min;
    float blur, znear, clip_fac;
    float bg[3];
    int32_t tile_w, tile_h; /* supported: 16x16, 32x16, 32x32, 8x8 */
    int32_t batch;          /* splats staged per LDS round in the renderers: 0 (= 64), 32,
                               64 or 128 (128 only for the four-wave 16x16 and the 32x16
                               backward; other kernels clamp to what their tile holds) */
    int32_t radix_bits;     /* digit width of the (view, depth) sort of the (view, splat) pairs, 4..8 */
    int32_t variant;        /* 16x16 renderers: 0 = one wave per tile (4 px per lane),
                               1 = one workgroup of four waves per tile */
    int32_t reserved[3];
} gesr_settings;

void gesr_default_settings(gesr_settings* s);

/* Splat parameters, structure-of-arrays, DEVICE float32:
 *  mean[3][n], scale[3][n] (linear, > 0), quat[4][n] (w, x, y, z; normalised
 *  inside), opacity[n] (activated, in (0, 1)), beta[n] (> 0),
 *  sh[K * 3][n] (coefficient k of channel c at row k * 3 + c; real SH with
 *  the Condon-Shortley phase, index l*l + l + m). */
typedef struct {
    int32_t n;
    const float* mean;
    const float* scale;
    const float* quat;
    const float* opacity;
    const float* beta;
    const float* sh;
} gesr_splats;

/* Projection outputs, DEVICE, caller-allocated ([V * n] entries each):
 *  rec[V*n][16]: u, v, L00, L10, L11, opacity, beta, qmax, r, g, b, depth,
 *       then the two words of rect[] (bit patterns) and two zero words
 *       (the conic Sigma'^-1 = [[A, B], [B, C]] in Cholesky form:
 *        A = L00^2, B = L00 L10, C = L10^2 + L11^2, so that
 *        q = (L00 dx + L10 dy)^2 + (L11 dy)^2; qmax = largest q with
 *        alpha >= alpha_min, padded by 2^-10; rgb after the clamp at 0;
 *        one 64-byte line per record, so a renderer's gather of a listed
 *        splat touches one line)
 *  tiles_touched[V*n]: tiles covered (0 = culled)
 *  rect[V*n][2]: inclusive tile rectangle (tx0 | ty0 << 16, tx1 | ty1 << 16);
 *      (0xFFFFFFFF, 0) for a culled pair
 *  depth_key[V*n]: bit pattern of the float32 camera depth. */
typedef struct {
    float* rec;
    uint32_t* tiles_touched;
    uint32_t* rect;
    uint32_t* depth_key;
} gesr_proj;

/* Binning outputs, DEVICE, caller-allocated.  `scratch` must hold at least
 * gesr_sizes.bin_scratch_bytes for the same (cams, V, n, settings, m_cap).
 *  tile_sorted[m_cap], val_sorted[m_cap]: instances sorted by the 64-bit key
 *      (global tile id << 32 | depth_key), equal keys by val; val = view * n +
 *      splat, tile_sorted = the instance's global tile id.  tile_sorted may be
 *      NULL (the renderers read only ranges and val_sorted).
 *  ranges[T][2]: [first, end) of each global tile in the sorted list, (0, 0)
 *      when empty.  Global tile ids number the tiles of view 0 row-major,
 *      then view 1, and so on.
 *  worklist[T]: global tile ids ordered by decreasing list length (ties by
 *      id), or by decreasing tile_work with GESR_BIN_WORK_ORDER.
 *  inst_base[V*n]: exclusive scan of tiles_touched in (view, splat) order: the
 *      instance slots of pair vi are inst_base[vi] + (row-major position of the
 *      tile in the pair's rectangle); the backward's per-instance partials use
 *      these slots.
 *  counters[4]: [0] = M (instance slots: the tiles of every pair's
 *      rectangle), [1] = 1 if M > m_cap, [2] = min(M, m_cap), [3] = the
 *      instances in the tile lists (<= M: each rectangle row keeps only the
 *      columns its ellipse reaches).  Written on the device.
 *  tile_work[T] (nullable, kept by the caller across calls): gesr_render_fwd
 *      writes, per global tile, the list positions its renderer evaluated
 *      before every pixel of the tile had terminated (at most the list
 *      length); gesr_bin with GESR_BIN_WORK_ORDER orders the worklist by
 *      decreasing tile_work (ties by id) instead of list length.  Most tiles
 *      stop long before their lists end, so a previous forward's figures over
 *      the same views and tile shape (consecutive training iterations, repeated
 *      renders) start the longest-running tiles first.  The order schedules
 *      tiles only: every output is the same whatever tile_work holds. */
typedef struct {
    uint64_t m_cap;
    uint32_t* tile_sorted;
    uint32_t* val_sorted;
    uint32_t* ranges;
    uint32_t* worklist;
    uint32_t* inst_base;
    uint32_t* counters;
    void* scratch;
    size_t scratch_bytes;
    uint32_t* tile_work;
} gesr_bins;

/* Gradient outputs, DEVICE, same layouts as gesr_splats; overwritten. */
typedef struct {
    float* mean;
    float* scale;
    float* quat;
    float* opacity;
    float* beta;
    float* sh;
} gesr_grads;

typedef struct {
    uint64_t total_tiles;      /* T: tiles over all views */
    uint64_t total_pixels;     /* P: pixels over all views */
    size_t bin_scratch_bytes;  /* gesr_bins.scratch size for the given m_cap */
    size_t bwd_workspace_bytes; /* backward workspace (visited bits, partials) for m_cap */
    uint64_t max_sort_blocks;  /* informational */
} gesr_sizes;

/* Sizes of the caller-allocated buffers.  Host-only. */
gesr_status gesr_query_sizes(gesr_ctx* ctx, const gesr_camera* cams, int V, int n, const gesr_settings* st,
                             uint64_t m_cap, gesr_sizes* out);

/* Projection (Sec. 3.2: Eq. 4, Sigma' = J W Sigma W^T J^T, Eq. 6-7; SH colour).
 * For every (view, splat): camera transform, near-plane cull (depth <=
 * znear), Sigma = M M^T with M = R(q) diag(phi(beta) s), EWA screen
 * covariance with the Jacobian at the centre clamped to clip_fac times the
 * half field of view, plus blur; conic factor; SH colour + 0.5 clamped at 0;
 * alpha_min footprint qmax = (ln(o/alpha_min)/kappa)^(2/beta) (1 + 2^-10) and
 * its pixel and tile rectangles.  Non-finite results and opacity < alpha_min
 * cull the pair (tiles_touched = 0).  Reads each splat once for all views. */
gesr_status gesr_project(gesr_ctx* ctx, const gesr_splats* splats, const gesr_camera* cams, int V,
                         const gesr_settings* st, const gesr_proj* out, void* stream);

#define GESR_BIN_SYNC 1       /* read M back and fail with GESR_ERR_CAPACITY if M > m_cap */
#define GESR_BIN_WORK_ORDER 2 /* worklist by decreasing bins->tile_work (non-NULL) */

/* Tile binning: one instance per (view, splat, covered tile), sorted by the
 * (tile | depth) key (see gesr_bins).  A pair covers the tiles of its
 * rectangle whose square [tx tw, (tx + 1) tw] x [ty th, (ty + 1) th] meets
 * its footprint ellipse q = (L00 dx + L10 dy)^2 + (L11 dy)^2 <= Q,
 * Q = qmax (1 + 2^-8) (a superset of the tiles holding a pixel centre with
 * q <= qmax, the alpha_min footprint of Eq. 3).  Each rectangle row's columns
 * come from the x-extent of the ellipse over the row's band, in float32 with
 * correctly rounded square roots and quotients, so decisions within float32
 * rounding of the rule's boundary may go either way.  The pairs are radix-sorted by (view, depth); the lists
 * are then built in two stable bucketing levels (pairs into tile rows, row
 * entries into the tiles of their columns) without sorting instances.
 * Instance slots (inst_base, the backward's partials) keep the rectangle
 * layout.  With GESR_BIN_SYNC the call
 * synchronises `stream` once after counting; if M > m_cap it returns
 * GESR_ERR_CAPACITY with *m_out = M and leaves the sorted lists undefined.
 * Without it the call never synchronises (capturable in a HIP graph): lists
 * are truncated to m_cap and counters[1] is set.  *m_out (nullable) receives
 * M only with GESR_BIN_SYNC. */
gesr_status gesr_bin(gesr_ctx* ctx, const gesr_proj* proj, const gesr_camera* cams, int V, int n,
                     const gesr_settings* st, const gesr_bins* bins, int flags, uint64_t* m_out, void* stream);

/* gesr_bin for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * binning, bit for bit, with its scratch taken from a static device array of
 * GESR_BIN_STATIC_SCRATCH_BYTES held by each GPU the library runs on until the
 * process ends, instead of bins->scratch (ignored, may be NULL).  The caller
 * still passes every input and output (proj, the sorted lists, ranges,
 * worklist, inst_base, counters).  Allocates nothing (no hipMalloc, hipFree or
 * allocating library call); the first call on a device looks the array's
 * address up once.  GESR_ERR_CAPACITY when this binning needs more scratch
 * than the array holds (the message gives both sizes; gesr_query_sizes'
 * bin_scratch_bytes is the need), with nothing enqueued.  Every call on one
 * GPU shares its array and the array keeps the last call's contents (the
 * binning clears what it reads before writing it): calls that overlap on one
 * GPU -- on different streams, or from different host threads -- race. */
#define GESR_BIN_STATIC_SCRATCH_BYTES (64u << 20)
gesr_status gesr_bin_static(gesr_ctx* ctx, const gesr_proj* proj, const gesr_camera* cams, int V, int n,
                            const gesr_settings* st, const gesr_bins* bins, int flags, uint64_t* m_out,
                            void* stream);

/* Optional per-pixel counters of gesr_render_fwd: fragments evaluated up to
 * termination (listed) and those with alpha >= alpha_min (hit). */
typedef struct {
    uint32_t* n_listed;
    uint32_t* n_hit;
} gesr_fwd_counts;

/* Extended channels (the depth maps of the mesh-extraction passage of
 * Sec. 3.3): the splat depth and a unit opacity composited like a colour over
 * a zero background, with the colour's fragments and termination:
 *   depth[p] = sum_k alpha_k T_k z_k   (z: camera-space depth of the centre,
 *                                        the record's last field),
 *   alpha[p] = sum_k alpha_k T_k = 1 - final_T[p].
 * DEVICE float [P] each (P = total pixels, view-major); either may be NULL.
 * The normalised depth is depth / alpha where alpha > 0. */
typedef struct {
    float* depth;
    float* alpha;
} gesr_fwd_channels;

/* Upstream gradients of the extended channels: DEVICE float [P] each, either
 * may be NULL (a zero gradient). */
typedef struct {
    const float* dL_ddepth;
    const float* dL_dalpha;
} gesr_bwd_channels;

/* Forward compositing (Eq. 5 as front-to-back alpha blending).  Per pixel,
 * over its tile's sorted list: q from the conic at the pixel centre,
 * alpha = min(alpha_max, o exp(-kappa q^(beta/2))); fragments with
 * alpha < alpha_min are skipped; compositing stops before a fragment that
 * would take T below t_min.  Outputs (DEVICE, P = total pixels):
 * image[3P] (CHW per view), final_T[P], n_contrib[P] (1-based list position
 * of the last composited fragment, 0 if none).  counts may be NULL.  Tiles are
 * rendered in bins->worklist order; bins->tile_work, when non-NULL, receives
 * each tile's evaluated list positions (see gesr_bins). */
gesr_status gesr_render_fwd(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins, const gesr_camera* cams,
                            int V, int n, const gesr_settings* st, float* image, float* final_T,
                            uint32_t* n_contrib, const gesr_fwd_counts* counts, void* stream);

/* gesr_render_fwd that also writes the extended channels (channels may be NULL:
 * then it is gesr_render_fwd).  The colour outputs are bitwise those of
 * gesr_render_fwd.  Channels need the one-wave 16x16 renderer (tile 16x16,
 * variant 0); other settings return GESR_ERR_UNSUPPORTED. */
gesr_status gesr_render_fwd_ext(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins,
                                const gesr_camera* cams, int V, int n, const gesr_settings* st, float* image,
                                float* final_T, uint32_t* n_contrib, const gesr_fwd_counts* counts,
                                const gesr_fwd_channels* channels, void* stream);

/* Backward pass: adjoint of gesr_render_fwd and gesr_project for upstream
 * dL_dimage (same layout as image).  Transmittance is recovered per pixel by
 * division from final_T and n_contrib (no per-fragment state is stored in the
 * forward); each tile reduces its pixels' contributions per instance without
 * atomics; a fixed-order segmented sum per (view, splat) then feeds the
 * projection adjoint, summed over views in ascending order.
 * `workspace` (DEVICE, gesr_sizes.bwd_workspace_bytes) holds, in order and
 * 256-byte aligned: the visited bits (uint32 [ceil(m_cap / 32)], one bit per
 * instance slot), the screen-space gradients (float [V*n][12]) and the
 * per-instance partials (float [m_cap][12], indexed by instance slot, see
 * inst_base).  grad2d (DEVICE [V*n][12], 16-byte aligned, nullable) receives
 * the screen-space gradients du, dv, dL00, dL10, dL11, dopacity, dbeta, dr,
 * dg, db, dz and a zero pad (dbeta here is the falloff term only; the
 * phi(beta) term is added in the projection adjoint; dz, the gradient of the
 * centre's camera depth, comes only from the extended channels).  `out` arrays are overwritten.  Results are bitwise
 * reproducible, and identical whether views are batched or rendered alone. */
gesr_status gesr_render_bwd(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj, const gesr_bins* bins,
                            const gesr_camera* cams, int V, const gesr_settings* st, const float* final_T,
                            const uint32_t* n_contrib, const float* dL_dimage, void* workspace, float* grad2d,
                            const gesr_grads* out, void* stream);

/* gesr_render_bwd with upstream gradients of the extended channels as well
 * (channels may be NULL: then it is gesr_render_bwd).  Each channel adds to
 * every composited fragment's dL/dalpha the term T_k (c_k - B_k) g, with
 * c_k = z_k (depth) or 1 (alpha) and B_k the channel composited behind the
 * fragment per unit transmittance; depth adds dz = alpha_k T_k g_depth.
 * Same renderer requirement as gesr_render_fwd_ext. */
gesr_status gesr_render_bwd_ext(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj,
                                const gesr_bins* bins, const gesr_camera* cams, int V, const gesr_settings* st,
                                const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                                const gesr_bwd_channels* channels, void* workspace, float* grad2d,
                                const gesr_grads* out, void* stream);

/* The two halves of gesr_render_bwd, for callers that schedule or time them
 * separately.  gesr_render_bwd_tiles: the per-tile render adjoint.  Each tile
 * visits its list up to the deepest position any of its pixels composited and
 * writes one gradient partial (grad2d order) per visited instance
 * with a non-zero contribution into the workspace, setting the instance
 * slot's visited bit (the bits are cleared first).  gesr_project_bwd: per
 * (view, splat), the fixed-order sum of the partials whose bits are set, then
 * the projection adjoint (Eq. 4, 6-7 and the EWA
 * passage of Sec. 3.2) summed over views in ascending order.  Arguments as in
 * gesr_render_bwd; n = splats->n. */
gesr_status gesr_render_bwd_tiles(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins,
                                  const gesr_camera* cams, int V, int n, const gesr_settings* st,
                                  const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                                  void* workspace, void* stream);
/* gesr_render_bwd_tiles with the extended channels' upstream gradients
 * (channels may be NULL). */
gesr_status gesr_render_bwd_tiles_ext(gesr_ctx* ctx, const gesr_proj* proj, const gesr_bins* bins,
                                      const gesr_camera* cams, int V, int n, const gesr_settings* st,
                                      const float* final_T, const uint32_t* n_contrib, const float* dL_dimage,
                                      const gesr_bwd_channels* channels, void* workspace, void* stream);
gesr_status gesr_project_bwd(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj, const gesr_bins* bins,
                             const gesr_camera* cams, int V, const gesr_settings* st, void* workspace,
                             float* grad2d, const gesr_grads* out, void* stream);

/* Autotuner (set-up call; it allocates, synchronises and is not capturable).
 * Times the whole forward + backward pipeline (gesr_project, gesr_bin with
 * capacity exactly M, gesr_render_fwd, gesr_render_bwd) on the caller's splats
 * and cameras, `reps` timed repetitions after one warm-up (whose forward
 * measures the tiles' work: the timed binnings order their worklists by it,
 * GESR_BIN_WORK_ORDER), for each candidate
 * (tile shape, 16x16 renderer variant, LDS batch), then for the best of those
 * each depth-sort digit width 5..8, and writes the fastest into *inout (the
 * numeric settings are kept).  The upstream gradient is a constant.  Device
 * buffers for the trials are allocated with hipMalloc and freed before
 * returning.  times_ms (HOST, nullable, max_trials entries) receives each
 * trial's milliseconds per pipeline (-1 for a trial that could not run, e.g.
 * out of memory), in the order the candidates are listed by
 * gesr_autotune_candidate; *n_trials (nullable) the number of trials run.
 * n = 0: nothing to time, *inout unchanged.  Errors: GESR_ERR_INVALID for bad
 * arguments (reps outside 1..100), GESR_ERR_HIP if no candidate could run. */
gesr_status gesr_autotune(gesr_ctx* ctx, const gesr_splats* splats, const gesr_camera* cams, int V,
                          gesr_settings* inout, int reps, float* times_ms, int max_trials, int* n_trials,
                          void* stream);

/* Candidate k of the autotuner's trial list (k = 0 .. count - 1, where count is
 * returned by gesr_autotune_candidate(-1, ...)): writes its tile shape, variant,
 * batch and radix bits into *out (other fields untouched).  Returns the number
 * of candidates for k = -1, else 0 on success and -1 when k is out of range. */
int gesr_autotune_candidate(int k, gesr_settings* out);

/* Level-set surface points (the sampling step of the mesh extraction,
 * Sec. 3.3).  For each of the R pixels in `pixels` (DEVICE uint32 [R], global
 * pixel ids of the concatenated views) the ray from the camera centre through
 * the pixel centre starts at the depth-map point, at camera depth
 * depth[p] / alpha[p] (DEVICE float [P] each, the extended channels of
 * gesr_render_fwd_ext; rays with alpha < min_alpha give no point).  The
 * density of Eq. 9, d(x) = sum_i o_i exp(-kappa m_i(x)^beta_i) with m_i the 3-D
 * Mahalanobis distance under Sigma_i = M_i M_i^T, M_i = R(q_i) diag(phi s_i),
 * is summed over the splats of the pixel's tile list whose screen footprint
 * covers the pixel (q <= qmax); g is the splat with the largest term at the
 * depth-map point and sigma_g(w) = |M_g^T w| for the ray direction w.
 * n_samples points spread evenly over +-span sigma_g(w) around it; the first
 * pair with d_k < level <= d_{k+1} brackets the surface closest to the camera
 * and the point is placed by linear interpolation; its normal is
 * -grad d / |grad d| (the direction of grad f for the SDF of Eq. 11).
 * Outputs (DEVICE float [R][4], 16-byte aligned): points (x, y, z, valid 1/0)
 * and normals (nx, ny, nz, t* = distance from the camera centre along w);
 * dominant (DEVICE uint32 [R], nullable): g as view * n + splat, 0xFFFFFFFF
 * when the ray has no candidate or alpha < min_alpha; n_candidates (DEVICE
 * uint32 [R], nullable): the number of candidate splats of the ray (0 when
 * alpha < min_alpha).  workspace: DEVICE, at least GESR_SURFACE_BYTES_PER_SPLAT
 * * n bytes, 16-byte aligned (per-splat frames, overwritten).  proj and bins are the
 * same step's (records and tile lists).  Errors: GESR_ERR_INVALID for
 * n_samples outside 2..GESR_SURFACE_MAX_SAMPLES, level <= 0, span <= 0, NULL
 * arrays or a misaligned workspace. */
#define GESR_SURFACE_MAX_SAMPLES 32
#define GESR_SURFACE_BYTES_PER_SPLAT 64
typedef struct {
    int32_t n_samples; /* samples per ray, 2..GESR_SURFACE_MAX_SAMPLES (32) */
    float level;       /* density level of the surface (0.3) */
    float span;        /* half-width of the sampled interval in sigma_g(w) (3) */
    float min_alpha;   /* rays whose alpha map value is below this give no point (0.5) */
} gesr_surface_settings;

gesr_status gesr_surface_points(gesr_ctx* ctx, const gesr_splats* splats, const gesr_proj* proj,
                                const gesr_bins* bins, const gesr_camera* cams, int V, const gesr_settings* st,
                                const gesr_surface_settings* ss, const float* depth, const float* alpha,
                                const uint32_t* pixels, uint32_t n_rays, float* points, float* normals,
                                uint32_t* dominant, uint32_t* n_candidates, void* workspace, void* stream);

/* L1 photometric term of Eq. 8 (the (1 - lambda) L1 part):
 * grad[i] = scale * sign(image[i] - target[i]) (sign(0) = 0), DEVICE, count
 * elements. */
gesr_status gesr_l1_grad(gesr_ctx* ctx, const float* image, const float* target, uint64_t count, float scale,
                         float* grad, void* stream);

/* Photometric loss of Eq. 8 (Sec. 3.2): per view v,
 *   L_v = (1 - lambda) mean|X - Y| + lambda (1 - mean SSIM(X, Y))
 * over the view's 3 H W values (X the rendered image, Y the target), with the
 * SSIM of an 11 x 11 Gaussian window (GESR_LOSS_RADIUS = 5) of standard
 * deviation `sigma`, zero padding outside the image, the map
 *   S = (2 mu_x mu_y + c1)(2 s_xy + c2) / ((mu_x^2 + mu_y^2 + c1)(s_x^2 + s_y^2 + c2))
 * per channel and pixel (mu, s^2, s_xy the window means, variances and
 * covariance).  gesr_default_loss_settings(): lambda 0.2 (the paper's value),
 * c1 = 0.01^2, c2 = 0.03^2, sigma = 1.5 (not given in the paper; the usual
 * SSIM constants for images in [0, 1]). */
#define GESR_LOSS_RADIUS 5
typedef struct {
    float lambda_dssim;
    float c1, c2;
    float sigma;
} gesr_loss_settings;

void gesr_default_loss_settings(gesr_loss_settings* s);

/* Workspace bytes of gesr_loss_eq8 for the views.  Host-only; 0 for invalid views. */
size_t gesr_loss_workspace_size(const gesr_camera* cams, int V);

/* Gradient of sum_v L_v with respect to the image into grad (DEVICE [3P], the
 * image layout; overwritten): (1 - lambda) sign(X - Y) / n_v (sign(0) = 0)
 * minus lambda / n_v times the SSIM map's gradient, n_v = 3 H W.  loss
 * (DEVICE float [V], nullable) receives L_v.  image, target, grad: DEVICE,
 * 16-byte aligned, grad may not alias image or target.  Fixed-order sums:
 * results are bitwise reproducible.  workspace: DEVICE, at least
 * gesr_loss_workspace_size bytes.  GESR_ERR_INVALID for bad views, NULL or
 * misaligned arrays, a small workspace, lambda outside [0, 1] or non-positive
 * c1, c2, sigma; nothing is enqueued then. */
gesr_status gesr_loss_eq8(gesr_ctx* ctx, const gesr_camera* cams, int V, const gesr_loss_settings* ls,
                          const float* image, const float* target, float* grad, float* loss, void* workspace,
                          size_t workspace_bytes, void* stream);

/* Surface-alignment regulariser of the flattened-splat workload (the paper
 * drives its splats flat onto the surface, Sec. 3.3; this loss is the reading
 * used for that workload): with k* the axis of the smallest scale of splat i
 * (lowest index on ties), n_i = R(q_i) e_k* and m_i its true surface normal
 * (normals DEVICE [3][n], unit length, sign-free),
 *   L = w_scale / n sum_i s_ik* + w_normal / n sum_i (1 - <n_i, m_i>^2).
 * Its gradient with respect to the scales and the raw quaternions (through the
 * normalisation) is ADDED to grads->scale and grads->quat (other gradient
 * arrays untouched; k* held fixed).  losses (DEVICE float [2], nullable): the
 * two terms, summed in a fixed order; they need a workspace of
 * gesr_align_workspace_size(n) bytes (else workspace may be NULL).  DEVICE
 * arrays 16-byte aligned.  GESR_ERR_INVALID for NULL or misaligned arrays,
 * non-finite weights or a small workspace. */
size_t gesr_align_workspace_size(int n);
gesr_status gesr_surface_align(gesr_ctx* ctx, const gesr_splats* splats, const float* normals, float w_scale,
                               float w_normal, const gesr_grads* grads, float* losses, void* workspace,
                               size_t workspace_bytes, void* stream);

/* Optimised (raw) splat parameters, DEVICE float32, structure-of-arrays with
 * the layouts of gesr_splats: mean[3][n], log_scale[3][n] (scale =
 * exp(log_scale)), quat[4][n], opacity_logit[n] (opacity = sigmoid(logit)),
 * beta[n], sh[sh_coeffs * 3][n].  The same struct holds Adam's first and
 * second moments. */
typedef struct {
    int32_t n;
    int32_t sh_coeffs; /* K = (sh_degree + 1)^2, 1..16 */
    float* mean;
    float* log_scale;
    float* quat;
    float* opacity_logit;
    float* beta;
    float* sh;
} gesr_params;

/* Adam with one learning rate per parameter group (the training schedule of
 * Sec. 4.2: 1.5e-3 for the shape parameter beta; the others follow 3DGS
 * practice) and the opacity-entropy term of Sec. 4.2 (binary opacities).
 * gesr_default_adam_settings() fills lr_mean 1.6e-4, lr_scale 5e-3, lr_quat
 * 1e-3, lr_opacity 0.05, lr_beta 1.5e-3, lr_sh_dc 2.5e-3, lr_sh_rest
 * 1.25e-4, beta1 0.9, beta2 0.999, eps 1e-15, entropy_weight 0, step 1. */
typedef struct {
    float lr_mean, lr_scale, lr_quat, lr_opacity, lr_beta, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    float entropy_weight; /* weight w of w * mean_i H(opacity_i), H the binary entropy */
    int32_t step;         /* 1-based step number t of the bias corrections 1 - beta^t */
    int32_t reserved[4];
} gesr_adam_settings;

void gesr_default_adam_settings(gesr_adam_settings* s);

/* One fused Adam step of every raw parameter, in place, from the gradients of
 * the activated parameters that gesr_render_bwd writes (`grads`, layouts of
 * gesr_splats):
 *   g_log_scale = g_scale * exp(log_scale),
 *   g_logit = (g_opacity + (w / n) * (-logit)) * o (1 - o),  o = sigmoid(logit)
 *     (the second term is the derivative of w * mean_i H(o_i)),
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   p -= lr * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps),
 * with lr by group (SH coefficient 0 uses lr_sh_dc, the rest lr_sh_rest).
 * Also writes the activated parameters of the updated values for the next
 * forward: scale_out[3][n] = exp(log_scale), opacity_out[n] = sigmoid(logit)
 * (DEVICE, caller-owned; these may be the gesr_splats arrays the renderer
 * reads).  `p`, `m`, `v` must have equal n and sh_coeffs and no aliasing.
 * Errors: GESR_ERR_INVALID for NULL or misaligned (16-byte) arrays, mismatched
 * sizes, step < 1, non-finite or negative learning rates, beta1/beta2 outside
 * [0, 1), eps <= 0; nothing is enqueued then. */
gesr_status gesr_adam_step(gesr_ctx* ctx, const gesr_params* p, const gesr_params* m, const gesr_params* v,
                           const gesr_grads* grads, const gesr_adam_settings* st, float* scale_out,
                           float* opacity_out, void* stream);

/* Pruning rule of the training schedule (Sec. 4.2: splats whose opacity falls
 * below 0.5 are removed; the shape pruning threshold 0.5 is read as a lower
 * bound on beta, since beta -> 0 flattens exp(-kappa q^(beta/2)) into an
 * unbounded footprint).  The opacity test is taken on the logit so that both
 * sides of a comparison see the same float32 number: a splat is kept iff
 *   logit >= float32(ln(min_opacity / (1 - min_opacity)))  and  beta >= min_beta.
 * min_opacity = 0 or min_beta <= 0 disables that test. */
typedef struct {
    float min_opacity; /* in [0, 1); 0.5 in the paper */
    float min_beta;
} gesr_prune_settings;

/* Workspace bytes gesr_prune needs for n splats.  Host-only. */
size_t gesr_prune_workspace_size(int n);

/* Stable compaction of the kept splats: the raw parameters `p` and, when `m`
 * and `v` are given (both or neither), Adam's moments, into `out_p` (`out_m`,
 * `out_v`), whose arrays must each hold as many floats as the corresponding
 * input array (rows x n).  The outputs are written packed with row stride
 * n_kept, in the input order: row r of an output array occupies
 * [r * n_kept, (r + 1) * n_kept); their n and sh_coeffs fields are ignored.
 * Optional scale_out[3][n_kept] and opacity_out[n_kept] receive the activated
 * values of the kept splats.  n_kept (DEVICE, one uint32) receives the count;
 * the call never synchronises (read n_kept back before using the outputs'
 * sizes).  Inputs and outputs must not overlap.  All arrays DEVICE, 16-byte
 * aligned.  GESR_ERR_INVALID for NULL or misaligned arrays, a workspace
 * smaller than gesr_prune_workspace_size(n), min_opacity outside [0, 1) or a
 * non-finite min_beta; nothing is enqueued then. */
gesr_status gesr_prune(gesr_ctx* ctx, const gesr_params* p, const gesr_params* m, const gesr_params* v,
                       const gesr_prune_settings* ps, const gesr_params* out_p, const gesr_params* out_m,
                       const gesr_params* out_v, float* scale_out, float* opacity_out, uint32_t* n_kept,
                       void* workspace, size_t workspace_bytes, void* stream);

/* Shape reset of the training schedule (Sec. 4.2: every 1000 iterations),
 * read as: beta of every splat set to `value` (2, the Gaussian case, where
 * phi(beta) = 1), and beta's Adam moments in `m` and `v` (nullable) zeroed so
 * that the optimiser restarts that parameter.  GESR_ERR_INVALID for a NULL p
 * or beta array, a non-positive or non-finite value. */
gesr_status gesr_shape_reset(gesr_ctx* ctx, const gesr_params* p, const gesr_params* m, const gesr_params* v,
                             float value, void* stream);

/* ------------------------------------------------------------------------
 * Surface regulariser (Sec. 3.3, Eq. 9-13; neighbour lists of Sec. 4.2).
 * ------------------------------------------------------------------------ */
#define GESR_KNN_MAX 16

/* Workspace bytes of gesr_knn for n splats and k neighbours.  Host-only. */
size_t gesr_knn_workspace_size(int n, int k);

/* Neighbour lists of the density of Eq. 9 (Sec. 4.2: 16 nearest splats,
 * refreshed periodically): knn[j][0] = j, then the k - 1 nearest other
 * centres by squared distance (float32), ties by index; 0xFFFFFFFF pads the
 * rows when n < k.  order [n]: the splats sorted by the cell of the search
 * grid (a spatial order; gesr_gsr runs its samples in it).  Inverse lists:
 * inv_entries[inv_offsets[i] .. inv_offsets[i + 1]) are the entries
 * e = p * k + s with knn[order[p]][s] = i, in increasing e (inv_offsets
 * [n + 1], inv_entries [n * k]); inv_slot [n * k] is their inverse,
 * inv_slot[inv_entries[t]] = t (undefined for padding entries).  Reads the
 * means of `splats` only.  DEVICE arrays, 16-byte aligned; the call never
 * synchronises.  GESR_ERR_INVALID for k outside 1..16, n * k >= 2^32, NULL or
 * misaligned arrays, or a workspace smaller than gesr_knn_workspace_size. */
gesr_status gesr_knn(gesr_ctx* ctx, const gesr_splats* splats, int k, uint32_t* knn, uint32_t* order,
                     uint32_t* inv_offsets, uint32_t* inv_entries, uint32_t* inv_slot, void* workspace,
                     size_t workspace_bytes, void* stream);

/* Weights of the two regulariser terms (lambda_1, lambda_2 of Eq. 14, which
 * the paper does not give; fold the 1 / |X| of Eq. 12-13 in as well). */
typedef struct {
    float w_sdf;
    float w_nor;
} gesr_gsr_settings;

/* Workspace bytes of gesr_gsr (frames, and partials when gradients are
 * wanted).  Host-only. */
size_t gesr_gsr_workspace_size(int n, int k, int with_grads);

/* Surface-regulariser losses and gradients on one sample per splat:
 *   x_j = mu_j + R_j diag(phi s_j) xi_j  (xi DEVICE [3][n], e.g. standard
 *   normal draws; samples with mask[j] == 0 are skipped, mask nullable);
 *   d(x) = sum over knn[j] of o_i exp(-kappa m_i(x)^beta_i)  (Eq. 9);
 *   g* = the neighbour with the largest term, n = its rotation column of the
 *   smallest scale, s_min = phi s of that axis, h = <x - mu_g*, n>;
 *   ideal density (Eq. 10, with s_min^beta: the falloff of Eq. 9 along the
 *   normal of a flat splat of opacity 1) exp(-kappa (|h| / s_min)^beta*);
 *   SDF (Eq. 11) f = sign(h) s_min sqrt(-ln d / kappa) for both densities
 *   (d floored at 1e-30, f = 0 where d >= 1);
 *   l_sdf = |fbar - f| (Eq. 12), l_nor = |-sign(h) grad d / |grad d| - n|^2
 *   (Eq. 13; 0 where grad d = 0).
 * knn, order, inv_offsets and inv_slot are gesr_knn's for the same k.
 * kappa and rho come from `st`.  sample_out [n][4] (DEVICE, nullable):
 * l_sdf, l_nor, g*'s slot in knn[j] (-1 when masked), d.  losses [2] (DEVICE,
 * nullable): the sums of l_sdf and l_nor over the samples, in a fixed order.
 * When `grads` is non-null, the gradient of
 * sum_j (w_sdf l_sdf + w_nor l_nor) with respect to mean, scale, quat,
 * opacity and beta (activated, layouts of gesr_splats) is ADDED to it, each
 * splat's terms summed in inverse-list order (the partial of entry e is
 * written to record inv_slot[e], so a splat's records are contiguous; no
 * atomics; every discrete choice held fixed); grads->sh is not touched.  The workspace needs
 * gesr_gsr_workspace_size(n, k, grads != NULL) bytes.  GESR_ERR_INVALID for
 * NULL or misaligned arrays, k outside 1..16, non-finite weights or a small
 * workspace. */
gesr_status gesr_gsr(gesr_ctx* ctx, const gesr_splats* splats, const gesr_settings* st, int k, const uint32_t* knn,
                     const uint32_t* order, const uint32_t* inv_offsets, const uint32_t* inv_slot, const float* xi,
                     const uint8_t* mask,
                     const gesr_gsr_settings* gs, float* sample_out, float* losses, const gesr_grads* grads,
                     void* workspace, size_t workspace_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GESR_H */
