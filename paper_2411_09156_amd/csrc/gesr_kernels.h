// Kernel argument blocks and launchers of the GES rasterizer (host + device).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gesr_device.h"

namespace gesr {

struct ProjectArgs {
    int n;
    const float *mean, *scale, *quat, *opacity, *beta, *sh;
    float* rec;
    uint32_t* tiles_touched;
    uint32_t* rect;
    uint32_t* depth_key;
    DevSettings st;
    DevCams cams;
};

struct ProjectBwdArgs {
    int n;
    const float *mean, *scale, *quat, *opacity, *beta, *sh;
    const uint32_t* tiles_touched;
    const float* grad2d;  // [V*n][GESR_GRAD2D_FLOATS] screen-space gradients
    float *g_mean, *g_scale, *g_quat, *g_opacity, *g_beta, *g_sh;
    DevSettings st;
    DevCams cams;
};

// Segmented sum of the per-instance partials of each (view, splat), reading
// only the instance slots whose bit the render adjoint set in `visited`.
struct SegReduceArgs {
    uint32_t vn;
    const uint32_t* tiles_touched;
    const uint32_t* inst_base;
    const uint32_t* visited;  // [ceil(m_cap / 32)] bit per instance slot
    const float* partials;
    uint64_t m_cap;
    float* grad2d;
};

struct RenderArgs {
    int n;
    const float* rec;
    const uint32_t* val_sorted;
    const uint32_t* ranges;
    const uint32_t* worklist;
    const uint32_t* inst_base;
    uint32_t n_items;  // number of work items (tiles) in the worklist
    int batch;         // records staged in LDS per round (one-wave renderers: 32 or 64)
    uint32_t* tile_work;  // forward: list positions each tile evaluated (nullable)
    // forward outputs / backward inputs
    float* image;
    float* final_T;
    uint32_t* n_contrib;
    uint32_t* n_listed;  // nullable
    uint32_t* n_hit;     // nullable
    float* out_depth;    // extended channels (nullable; only the one-wave 16x16 renderer)
    float* out_alpha;
    // backward
    const float* dL_dimage;
    const float* dL_ddepth;  // extended channels' upstream gradients (nullable)
    const float* dL_dalpha;
    float* partials;
    uint32_t m_cap;      // capacity of partials (instances); only reached when the lists overflowed
    uint32_t* visited;   // bit per instance slot, set where non-zero partials were written
    DevSettings st;
    DevCams cams;
};

// Level-set surface points along depth-map rays (gesr_surface.hip).
struct SurfaceArgs {
    int n;
    const float *mean, *scale, *quat, *opacity, *beta;  // splat parameters, SoA
    const float* rec;
    const uint32_t* val_sorted;
    const uint32_t* ranges;
    const float* depth;   // [P] extended channels of the forward
    const float* alpha;   // [P]
    const uint32_t* pixels;
    uint32_t n_rays;
    int n_samples;
    float level, span, min_alpha;
    int tile_w, tile_h;
    float* points;        // [R][4]: x, y, z, valid
    float* normals;       // [R][4]: nx, ny, nz, t*
    uint32_t* dominant;   // [R] nullable
    uint32_t* n_candidates;  // [R] nullable
    float* frames;        // [n][16] per-splat M^-1, mean, opacity, beta/2 (workspace)
    DevSettings st;
    DevCams cams;
};
hipError_t launch_surface_points(const SurfaceArgs& a, hipStream_t stream);

hipError_t launch_project(const ProjectArgs& a, int sh_degree, hipStream_t stream);
hipError_t launch_project_bwd(const ProjectBwdArgs& a, int sh_degree, hipStream_t stream);
hipError_t launch_seg_reduce(const SegReduceArgs& a, hipStream_t stream);
// Channels (a.out_depth / a.out_alpha, a.dL_ddepth / a.dL_dalpha non-null) need
// tile 16x16 with batch 32 or 64 (the one-wave renderers); callers check.
hipError_t launch_render_fwd(const RenderArgs& a, int tile_w, int tile_h, bool counts, hipStream_t stream);
hipError_t launch_render_bwd(const RenderArgs& a, int tile_w, int tile_h, int batch, hipStream_t stream);

// ---------------------------------------------------------------- sorting
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;  // keys per sort block
constexpr int SCAN_TILE = 4096;                       // items per scan block
constexpr int SCAN_TOP_MAX = 32768;                   // max blocks of a two-level scan

// Exclusive scan of `count` uint32 values; the grand total goes to *total
// (device, nullable).  `partials` needs ceil(count / SCAN_TILE) entries.
hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, uint64_t count, uint32_t* partials, uint32_t* total,
                          hipStream_t stream);

// Stable LSD radix sort of `count_static` (or *count_dev when non-null, which
// must not exceed count_static) 32-bit keys over bits [0, key_bits) carrying
// 32-bit values.  vals_in == nullptr means values are the positions 0..n-1.
// With view_n != 0 the key is 64 bits, (value / view_n) << 32 | key, sorted
// over bits [0, key_bits) (key_bits > 32: the view bits of (view, splat) pair
// values), so no separate pass over a view key is needed.
// Ping-pongs between (keys_a, vals_a) and (keys_b, vals_b); the first pass
// reads keys_in / vals_in.  Returns (via *result_in_b) whether the result
// ends in the b buffers.
struct SortBuffers {
    uint32_t *keys_a, *vals_a, *keys_b, *vals_b;
    uint32_t* block_hist;  // 2^radix_bits * ceil(count_static / SORT_TILE)
    uint32_t* scan_partials;
};
hipError_t radix_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint64_t count_static,
                      const uint32_t* count_dev, int key_bits, int radix_bits, const SortBuffers& b,
                      bool* result_in_b, hipStream_t stream, uint32_t view_n = 0);
int radix_passes(int key_bits, int radix_bits);

// Binning helper kernels.
// out[k] = the rectangle in pair order[k]'s record (x = 0xFFFFFFFF when the pair touches no tile);
// with ell (nullable, [2 count]) also the pair's footprint ellipse and its per-row constants.
hipError_t launch_gather_rects(const uint32_t* order, const float* rec, uint64_t count, uint2* out, float4* ell,
                               hipStream_t stream);

// Interval scatter (tile lists from rectangles, see gesr_bin.hip).  Level 1
// writes each pair into the row lists of the rows its rectangle covers; level
// 2 writes each row-list entry into the tile lists of the columns it covers.
struct IsArgs {
    int n;
    uint32_t vn;
    const uint32_t* items;          // level 1: pairs in (view, depth) order; level 2: row lists
    const uint2* item_rect;         // level 1: the items' tile rectangles (empty: x = 0xFFFFFFFF)
    const uint32_t* item_cols;      // level 2: the items' columns, tx0 | tx1 << 16
    const uint32_t* items_listed;   // level 2: valid entries of the row lists (device)
    const uint32_t* row_start;      // level 2: [total rows]
    const uint32_t* row_count;      // level 2: [total rows]
    uint32_t* chunk_off;            // [segments + 1]
    uint32_t* chunk_total;          // device
    uint32_t nseg;                  // set by launch_interval_scatter
    uint32_t* mat;                  // [mat_chunks][window] per-chunk bucket counts, then prefixes
    uint64_t mat_chunks;
    uint32_t* bucket_count;         // [buckets]
    uint32_t* bucket_start;         // [buckets]
    uint32_t* out_vals;             // [out_cap]
    uint32_t* out_keys;             // nullable: bucket id of every entry
    uint32_t* out_cols;             // level 1: columns of every entry (tx0 | tx1 << 16)
    uint64_t out_cap;
    const float4* item_ell;         // level 1 (nullable): per item, the footprint ellipse; each entry
    int tile_w, tile_h;             //   then carries the columns it reaches in the entry's row
    DevCams cams;
};
uint32_t is_segments(const DevCams& cams, int level);
// Upper bound on the chunks of a level (level2_items: capacity of the row lists).
uint64_t is_chunk_bound(const DevCams& cams, int level, int n, uint64_t level2_items);
uint32_t is_window();
// seg_chunks: [segments + 1] scratch.  Writes bucket_count, bucket_start and
// the bucket total (*bucket_total, device) and scatters the items.
hipError_t launch_interval_scatter(IsArgs a, int level, uint32_t n_buckets, uint32_t* bucket_total,
                                   uint32_t* seg_chunks, uint32_t* scan_partials, hipStream_t stream);
hipError_t launch_ranges_from_counts(const uint32_t* counts, const uint32_t* starts, uint64_t total_tiles,
                                     const uint32_t* listed, uint32_t* ranges, hipStream_t stream);
hipError_t launch_set_counters(uint32_t* counters, uint64_t m_cap, hipStream_t stream);
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t count, hipStream_t stream);
hipError_t launch_worklist_keys(const uint32_t* ranges, const uint32_t* work, uint64_t total_tiles, uint32_t* keys,
                                hipStream_t stream);
// Photometric loss of Eq. 8 (gesr_loss.hip).
struct LossView {
    int W, H;
    uint32_t pix_base;   // first pixel of the view
    uint32_t tile_base;  // first 16 x 16 loss tile of the view
    float inv_n;         // 1 / (3 W H)
};
struct LossArgs {
    int V;
    LossView v[GESR_MAX_VIEWS];
    float w[2 * GESR_LOSS_RADIUS + 1];  // normalised Gaussian weights, offsets -r..r
    float lam, c1, c2;
    const float* image;
    const float* target;
    float* amap;     // [3P] dS/dmu_x per value (CHW per view, as the image)
    float* bmap;     // [3P] dS/dm2x
    float* cmap;     // [3P] dS/dmxy
    float* partial;  // [tiles][2]: per-tile sums of S and |X - Y|
    float* grad;     // [3P]
    float* loss;     // [V]
};
hipError_t launch_ssim_loss(const LossArgs& a, uint32_t n_tiles, bool want_loss, hipStream_t stream);

// Surface-alignment regulariser (gesr_loss.hip).
struct AlignArgs {
    int n;
    const float* scale;   // [3][n]
    const float* quat;    // [4][n]
    const float* normal;  // [3][n] true surface normals
    float w_scale_n, w_normal_n;  // weights / n
    float* g_scale;       // [3][n], added to
    float* g_quat;        // [4][n], added to
    float* partial;       // [blocks][2] (nullable when losses is)
    float* losses;        // [2] (nullable)
};
hipError_t launch_surface_align(const AlignArgs& a, hipStream_t stream);
hipError_t launch_l1_grad(const float* image, const float* target, uint64_t count, float scale, float* grad,
                          hipStream_t stream);

// Fused Adam step (gesr_optim.hip).  Rows of the parameter matrix: mean 0-2,
// log scale 3-5, quaternion 6-9, logit 10, beta 11, SH 12 .. 12 + 3K - 1.
struct AdamArgs {
    int n;
    gesr_params p, m, v;
    const float *g_mean, *g_scale, *g_quat, *g_opacity, *g_beta, *g_sh;
    float lr_mean, lr_scale, lr_quat, lr_opacity, lr_beta, lr_sh_dc, lr_sh_rest;
    float beta1, beta2, eps;
    float inv_c1, inv_c2;   // 1 / (1 - beta^t)
    float entropy_scale;    // w / n
    float* scale_out;
    float* opacity_out;
};
hipError_t launch_adam_step(const AdamArgs& a, int rows, hipStream_t stream);

// Stable compaction of the splats kept by the pruning rule (gesr_optim.hip).
constexpr uint32_t PRUNE_BLOCK = 1024;  // splats per flag / scatter block
struct PruneArgs {
    int n;
    const float* logit;
    const float* beta;
    float t_logit, min_beta;  // keep iff logit >= t_logit and beta >= min_beta
    uint32_t* bits;           // [blocks * 32] keep bits
    uint32_t* counts;         // [blocks]
    uint32_t* offsets;        // [blocks], exclusive scan of counts
    uint32_t* n_kept;         // device total
    const float* in_p[6];     // mean, log scale, quaternion, logit, beta, SH
    const float* in_m[6];     // nullable (all or none)
    const float* in_v[6];
    float* out_p[6];
    float* out_m[6];
    float* out_v[6];
    float* scale_out;         // nullable: exp(log scale) of the kept splats
    float* opacity_out;       // nullable: sigmoid(logit) of the kept splats
};
uint32_t prune_blocks(int n);
size_t prune_workspace_bytes(int n);
hipError_t launch_prune(PruneArgs a, int rows, uint32_t* partials, hipStream_t stream);
hipError_t launch_shape_reset(float* beta, float* m, float* v, int n, float value, hipStream_t stream);

// Surface regulariser (gesr_gsr.hip).
struct KnnGrid {
    float lo[3];
    int dim[3];
    float cs, inv_cs;
};
// Word offsets of the neighbour-list workspace.
struct KnnLayout {
    uint32_t bound_parts, cell_cap;
    uint64_t o_grid, o_parts, o_keys, o_ka, o_va, o_kb, o_vb, o_hist, o_scan, o_pos, o_start, o_end, words;
};
KnnLayout knn_layout(int n, int k);
hipError_t launch_knn(const float* mean, int n, int k, uint32_t* knn, uint32_t* order_out, uint32_t* inv_offsets,
                      uint32_t* inv_entries, uint32_t* inv_slot, uint32_t* ws, hipStream_t stream);

constexpr int GSR_PARTIAL_FLOATS = 12;  // mean 3, scale 3, quaternion 4, opacity, beta
constexpr int GSR_PARTIAL_STRIDE = 16;  // one aligned 64-byte record per (sample, slot)
constexpr int GSR_SUM_BLOCK = 4096;     // samples per first-level loss-sum block
constexpr int GSR_FRAME_FLOATS = 16;  // one 64-byte record per splat
struct GsrArgs {
    int n, k;
    const float *mean, *scale, *quat, *opacity, *beta;
    const uint32_t* knn;
    const uint32_t* order;  // samples in cell order
    const uint32_t* inv_offsets;
    const uint32_t* inv_slot;  // [n * k]: record of entry p * k + s
    const float* xi;        // [3][n]
    const uint8_t* mask;    // nullable
    float kappa, rho, w_sdf, w_nor;
    float* frames;          // [n][GSR_FRAME_FLOATS]
    float* partials;        // [n * k][16] records in inverse-list order, null: no gradients
    float* sample_out;      // [n][4]: l_sdf, l_nor, g* slot (-1 when masked), d
    float* losses;          // nullable: sums of l_sdf and l_nor
    float* sum_parts;       // [ceil(n / GSR_SUM_BLOCK)][2] first-level sums
    float *g_mean, *g_scale, *g_quat, *g_opacity, *g_beta;
};
hipError_t launch_gsr(GsrArgs a, hipStream_t stream);

}  // namespace gesr
